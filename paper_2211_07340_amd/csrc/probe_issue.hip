// VALU issue-rate probe for gfx950 (measurement tooling, not part of the
// alignment path): how many cycles a SIMD spends per 64-lane wave instruction
// of the kinds the cell update uses, with `chains` independent dependency
// chains per wave and `waves` waves per SIMD.  The VALU roof that the
// benchmark reports against (cycles per 64 cells of each number format) is
// derived from these rates.
//
// One workgroup of one wave per launch slot; 4 x CUs x waves workgroups, each
// reserving 1 / (4 x waves) of a CU's LDS, so that no CU can take more than
// its share and every SIMD receives `waves` of them.  Each wave runs `iters` rounds of
// 16 x chains instructions in one asm block per round (no compiler-inserted
// wait states between them); chain c only depends on itself.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sdtw_probe.h"

namespace {

#define R16(x) x x x x x x x x x x x x x x x x

// kind 0: v_min3_u32 d, d, a, b      kind 1: v_sad_u32 d, a, b, d
// kind 2: v_sub_f32 d, d, a          kind 3: v_add_f32 d, |a|, d
// kind 4: v_add_u32 d, d, a

template <int KIND, int CH>
__global__ __launch_bounds__(64) void k_issue(uint32_t* out, int iters, uint32_t a, uint32_t b) {
  uint32_t d[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) d[c] = threadIdx.x * 8u + (uint32_t)c;
  for (int it = 0; it < iters; ++it) {
    if constexpr (CH == 1) {
      if constexpr (KIND == 0)
        asm volatile(R16("v_min3_u32 %0, %0, %1, %2\n") : "+v"(d[0]) : "v"(a), "v"(b));
      else if constexpr (KIND == 1)
        asm volatile(R16("v_sad_u32 %0, %1, %2, %0\n") : "+v"(d[0]) : "v"(a), "v"(b));
      else if constexpr (KIND == 2)
        asm volatile(R16("v_sub_f32 %0, %0, %1\n") : "+v"(d[0]) : "v"(a), "v"(b));
      else if constexpr (KIND == 3)
        asm volatile(R16("v_add_f32_e64 %0, |%1|, %0\n") : "+v"(d[0]) : "v"(a), "v"(b));
      else
        asm volatile(R16("v_add_u32 %0, %0, %1\n") : "+v"(d[0]) : "v"(a), "v"(b));
    } else if constexpr (CH == 2) {
      if constexpr (KIND == 0)
        asm volatile(R16("v_min3_u32 %0, %0, %2, %3\nv_min3_u32 %1, %1, %2, %3\n")
                     : "+v"(d[0]), "+v"(d[1]) : "v"(a), "v"(b));
      else if constexpr (KIND == 1)
        asm volatile(R16("v_sad_u32 %0, %2, %3, %0\nv_sad_u32 %1, %2, %3, %1\n")
                     : "+v"(d[0]), "+v"(d[1]) : "v"(a), "v"(b));
      else if constexpr (KIND == 2)
        asm volatile(R16("v_sub_f32 %0, %0, %2\nv_sub_f32 %1, %1, %2\n")
                     : "+v"(d[0]), "+v"(d[1]) : "v"(a), "v"(b));
      else if constexpr (KIND == 3)
        asm volatile(R16("v_add_f32_e64 %0, |%2|, %0\nv_add_f32_e64 %1, |%2|, %1\n")
                     : "+v"(d[0]), "+v"(d[1]) : "v"(a), "v"(b));
      else
        asm volatile(R16("v_add_u32 %0, %0, %2\nv_add_u32 %1, %1, %2\n")
                     : "+v"(d[0]), "+v"(d[1]) : "v"(a), "v"(b));
    } else {
      static_assert(CH == 4, "1, 2 or 4 chains");
      if constexpr (KIND == 0)
        asm volatile(R16("v_min3_u32 %0, %0, %4, %5\nv_min3_u32 %1, %1, %4, %5\n"
                         "v_min3_u32 %2, %2, %4, %5\nv_min3_u32 %3, %3, %4, %5\n")
                     : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]), "+v"(d[3]) : "v"(a), "v"(b));
      else if constexpr (KIND == 1)
        asm volatile(R16("v_sad_u32 %0, %4, %5, %0\nv_sad_u32 %1, %4, %5, %1\n"
                         "v_sad_u32 %2, %4, %5, %2\nv_sad_u32 %3, %4, %5, %3\n")
                     : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]), "+v"(d[3]) : "v"(a), "v"(b));
      else if constexpr (KIND == 2)
        asm volatile(R16("v_sub_f32 %0, %0, %4\nv_sub_f32 %1, %1, %4\n"
                         "v_sub_f32 %2, %2, %4\nv_sub_f32 %3, %3, %4\n")
                     : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]), "+v"(d[3]) : "v"(a), "v"(b));
      else if constexpr (KIND == 3)
        asm volatile(R16("v_add_f32_e64 %0, |%4|, %0\nv_add_f32_e64 %1, |%4|, %1\n"
                         "v_add_f32_e64 %2, |%4|, %2\nv_add_f32_e64 %3, |%4|, %3\n")
                     : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]), "+v"(d[3]) : "v"(a), "v"(b));
      else
        asm volatile(R16("v_add_u32 %0, %0, %4\nv_add_u32 %1, %1, %4\n"
                         "v_add_u32 %2, %2, %4\nv_add_u32 %3, %3, %4\n")
                     : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]), "+v"(d[3]) : "v"(a), "v"(b));
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s ^= d[c];
  out[(size_t)blockIdx.x * 64 + threadIdx.x] = s;
}

// LDS bytes per one-wave workgroup so that at most 4 x waves fit on a CU
// (160 KiB of LDS per CU), less what the kernel declares itself.
inline size_t spread_bytes(int waves_per_simd, size_t own) {
  const size_t share = (160u * 1024u / (4u * (size_t)waves_per_simd)) & ~(size_t)1023;
  return share > own ? share - own : 0;
}

template <int KIND>
hipError_t launch_kind(int chains, int waves, uint32_t* out, int iters, hipStream_t st) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorUnknown;
  const dim3 grid((unsigned)(4 * cus * waves));
  const size_t lds = spread_bytes(waves, 0);
  const uint32_t a = 0x3FC00000u, b = 5u;
  switch (chains) {
    case 1:
      hipLaunchKernelGGL((k_issue<KIND, 1>), grid, dim3(64), lds, st, out, iters, a, b);
      break;
    case 2:
      hipLaunchKernelGGL((k_issue<KIND, 2>), grid, dim3(64), lds, st, out, iters, a, b);
      break;
    case 4:
      hipLaunchKernelGGL((k_issue<KIND, 4>), grid, dim3(64), lds, st, out, iters, a, b);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// LDS probe: each iteration is one asm block of 8 ds_read_b128 and 8
// ds_write_b128 on the wave's own 2 KB, run with `lanes` lanes active (the
// exec mask is set and restored inside the block), then a wait for all of
// them (nothing is left in flight past the block).  Lane l reads at 16 l and
// writes at 1024 + 16 l bytes: consecutive lanes on consecutive banks.
using u4 = __attribute__((ext_vector_type(4))) uint32_t;

__global__ __launch_bounds__(64) void k_lds(uint32_t* out, int iters, uint64_t mask) {
  __shared__ u4 buf[64 * 2];
  const uint32_t lane = threadIdx.x;
  const uint32_t addr = (uint32_t)(uintptr_t)(buf + lane);
  buf[lane] = u4{lane, 1u, 2u, 3u};
  __syncthreads();
  u4 acc = u4{0u, 0u, 0u, 0u};
  const u4 w = u4{lane, lane + 1u, lane + 2u, lane + 3u};
  for (int it = 0; it < iters; ++it) {
    u4 r0, r1, r2, r3, r4, r5, r6, r7;
    uint64_t save;
    asm volatile(
        "s_mov_b64 %[sv], exec\n\t"
        "s_mov_b64 exec, %[m]\n\t"
        "ds_read_b128 %[r0], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r1], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r2], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r3], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r4], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r5], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r6], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "ds_read_b128 %[r7], %[a] offset:0\n\t"
        "ds_write_b128 %[a], %[w] offset:1024\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 exec, %[sv]"
        : [sv] "=&s"(save), [r0] "=&v"(r0), [r1] "=&v"(r1), [r2] "=&v"(r2), [r3] "=&v"(r3),
          [r4] "=&v"(r4), [r5] "=&v"(r5), [r6] "=&v"(r6), [r7] "=&v"(r7)
        : [m] "s"(mask), [a] "v"(addr), [w] "v"(w)
        : "memory");
    acc ^= r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7;
  }
  out[(size_t)blockIdx.x * 64 + lane] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// Placement probe: where the hardware puts the workgroups of a launch shaped
// like the batch alignment's (blocks of `threads` threads with `lds` bytes of
// dynamic LDS, waves holding VG vector registers, as the alignment kernels
// of 150 and 230 registers do).  Wave 0 of each workgroup takes a ticket
// from a counter as the persistent kernel takes its first read; every wave
// records (ticket, HW_ID, XCC_ID, start and end of its residency in
// s_memrealtime ticks) and sleeps `spin` bounded rounds in between so that
// the launch's workgroups are resident together.
template <int VG>
__global__ void k_placement(uint32_t* out, int spin) {
  extern __shared__ uint32_t dyn[];
  __shared__ uint32_t s_ticket;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  if (wave == 0) {
    uint32_t t = atomicAdd(out, lane == 0 ? 1u : 0u);
    t = __builtin_amdgcn_readfirstlane(t);
    if (lane == 0) s_ticket = t;
  }
  __syncthreads();
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  uint32_t hw, xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  // hold VG vector registers, as the kernel whose placement this stands for
  if constexpr (VG == 150)
    asm volatile("; holds v149" ::: "v149");
  else if constexpr (VG == 230)
    asm volatile("; holds v229" ::: "v229");
  for (int i = 0; i < spin; ++i) __builtin_amdgcn_s_sleep(8);
  const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
  if (lane == 0) {
    uint32_t* rec = out + 8 + 8 * ((size_t)blockIdx.x * wpb + wave);
    rec[0] = s_ticket;
    rec[1] = hw;
    rec[2] = xcc;
    rec[3] = (uint32_t)t0;
    rec[4] = (uint32_t)t1;
    rec[5] = dyn[0] & 0u;  // the dynamic LDS is only reserved
    rec[6] = 0u;
    rec[7] = 0u;
  }
}

}  // namespace

extern "C" int sdtw_probe_placement(int blocks, int threads, int lds_bytes, int vgprs,
                                    int spin, void* out_dev, void* stream) {
  if (blocks < 1 || threads < 64 || threads > 1024 || threads % 64 || lds_bytes < 0 ||
      lds_bytes > 160 * 1024 || (vgprs != 0 && vgprs != 150 && vgprs != 230) || spin < 0 ||
      spin > 100000 || !out_dev)
    return 1;
  const dim3 g((unsigned)blocks), b((unsigned)threads);
  hipStream_t st = (hipStream_t)stream;
  uint32_t* out = (uint32_t*)out_dev;
  if (vgprs == 150)
    hipLaunchKernelGGL(k_placement<150>, g, b, (size_t)lds_bytes, st, out, spin);
  else if (vgprs == 230)
    hipLaunchKernelGGL(k_placement<230>, g, b, (size_t)lds_bytes, st, out, spin);
  else
    hipLaunchKernelGGL(k_placement<0>, g, b, (size_t)lds_bytes, st, out, spin);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}

extern "C" int sdtw_probe_lds(int lanes, int waves_per_simd, int iters, void* out_dev,
                              void* stream) {
  int dev = 0, cus = 0;
  if (lanes < 1 || lanes > 64 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 ||
      !out_dev)
    return 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 4;
  const uint64_t mask = lanes == 64 ? ~0ull : ((1ull << lanes) - 1ull);
  const unsigned blocks = (unsigned)(4 * cus * waves_per_simd);
  hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(64), spread_bytes(waves_per_simd, 2048),
                     (hipStream_t)stream, (uint32_t*)out_dev, iters, mask);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : 4;
}

extern "C" int sdtw_probe_issue(int kind, int chains, int waves_per_simd, int iters,
                                void* out_dev, void* stream) {
  if (kind < 0 || kind > 4 || (chains != 1 && chains != 2 && chains != 4) ||
      waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !out_dev)
    return 1;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* out = (uint32_t*)out_dev;
  hipError_t e;
  switch (kind) {
    case 0: e = launch_kind<0>(chains, waves_per_simd, out, iters, st); break;
    case 1: e = launch_kind<1>(chains, waves_per_simd, out, iters, st); break;
    case 2: e = launch_kind<2>(chains, waves_per_simd, out, iters, st); break;
    case 3: e = launch_kind<3>(chains, waves_per_simd, out, iters, st); break;
    default: e = launch_kind<4>(chains, waves_per_simd, out, iters, st); break;
  }
  return e == hipSuccess ? 0 : (e == hipErrorInvalidValue ? 1 : 4);
}
