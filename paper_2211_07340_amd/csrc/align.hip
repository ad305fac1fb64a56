// sDTW alignment kernels for gfx950 (section 2.3 Eq. 1; section 4.3).
//
// Work decomposition.  One wave64 aligns one read.  The reference is cut
// into tiles of T = 64*W columns; lane l owns the strip of W consecutive
// columns [l*W, l*W + W) of the current tile and keeps the reference values
// y[W] and the previous row gamma(i-1, strip) in registers.  The query sits
// in LDS.  Rows advance one per step; lane l works one row behind lane l-1
// (the oblique, anti-diagonal front of section 4.3 "operation pipelining",
// here across lanes), so the value a lane needs from its left neighbour,
// gamma(i, j0-1), is that neighbour's last column computed one step earlier
// and arrives by a DPP wave_shr:1 move.  The value received one step earlier
// is the diagonal gamma(i-1, j0-1).  Lane 0 takes its left boundary from an
// LDS column B[0..M) that lane 63 fills while sweeping the previous tile
// (gamma(., j) depends on Y[1..j] only, so tiling is exact).
//
// Per cell: int16 path  v_min3_u32 + v_sad_u32          (2 VALU)
//           fp32 path   v_sub_f32 + v_min3_u32 + v_add_f32 |.|  (3 VALU)
// Costs travel as uint32 bit patterns in both formats: every DP value is a
// sum of absolute differences (>= +0) or +inf, and IEEE encodings of
// non-negative floats order like their values, so one unsigned min3 serves
// both and never changes a result.
//
// The last row of every tile is folded into a per-lane running (cost, j)
// minimum with strict '<' in increasing j, and a lexicographic wave
// reduction gives the first column attaining the minimum (the strict-less
// last-row scan of Algorithms 1 and 2).
//
// k_align_skew (M >= 65): continuous skew.  Lanes never wait for each other
// at tile boundaries: lane l enters tile p at step p*M + l, so each period
// of M steps starts with 64 "switch" steps in which exactly one lane swaps
// its strip under a one-lane mask: new y from registers loaded one period
// ahead, its finished last row out to LDS, gamma(0, .) = 0 in.  A one-lane
// LDS instruction costs the CU about as much LDS time as any other, so the
// switch keeps its LDS instructions few.  The wave runs ntiles*M + 64 steps
// for ntiles*T*M cells.  Reads are pulled longest-first from a work list by
// a persistent grid.
//
// k_align_plain (any M >= 1): synchronised tiles; every tile costs M + 63
// steps with lanes idle during fill and drain.  Used for reads shorter than
// 65 rows and as the one-read-per-launch baseline.
#include <limits.h>

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace sdtw {
namespace {

struct FmtI16 {
  using qin = int16_t;
  using xlds = uint16_t;  // biased copy of the query in LDS
  static constexpr uint32_t kInf = 0xFFFFFFFFu;
  __device__ static __forceinline__ xlds to_lds(int16_t v) {
    return (uint16_t)((int32_t)v + (int32_t)kI16Bias);
  }
  __device__ static __forceinline__ uint32_t cell(uint32_t x, uint32_t y, uint32_t m) {
    const uint32_t d = x > y ? x - y : y - x;  // with the add: v_sad_u32
    return d + m;
  }
  __device__ static __forceinline__ void store_cost(void* cost, int32_t r, uint32_t v) {
    ((int32_t*)cost)[r] = (int32_t)v;
  }
};

struct FmtF32 {
  using qin = float;
  using xlds = uint32_t;
  static constexpr uint32_t kInf = 0x7F800000u;
  __device__ static __forceinline__ xlds to_lds(float v) { return __float_as_uint(v); }
  __device__ static __forceinline__ uint32_t cell(uint32_t x, uint32_t y, uint32_t m) {
    return __float_as_uint(fabsf(__uint_as_float(x) - __uint_as_float(y)) + __uint_as_float(m));
  }
  __device__ static __forceinline__ void store_cost(void* cost, int32_t r, uint32_t v) {
    ((float*)cost)[r] = __uint_as_float(v);
  }
};

// f(integral_constant<int, I>) for I in [B, E), unrolled at compile time
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
  return min(min(a, b), c);
}

// nw[w] = gamma(i, j0+w) from up[w] = gamma(i-1, j0+w), the diagonal
// dprev = gamma(i-1, j0-1) and left = gamma(i, j0-1).
template <class F, int W>
__device__ __forceinline__ void strip_row(uint32_t x, const uint32_t (&y)[W],
                                          const uint32_t (&up)[W], uint32_t (&nw)[W],
                                          uint32_t dprev, uint32_t left) {
  nw[0] = F::cell(x, y[0], min3u(up[0], dprev, left));
#pragma unroll
  for (int w = 1; w < W; ++w) nw[w] = F::cell(x, y[w], min3u(up[w], up[w - 1], nw[w - 1]));
}

// Lane l receives lane l-1's `v`; lane 0 keeps `lane0` (DPP wave_shr:1 with
// bound_ctrl off leaves the destination of the source-less lane unchanged).
__device__ __forceinline__ uint32_t from_left_lane(uint32_t v, uint32_t lane0) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)lane0, (int)v, 0x138, 0xF, 0xF, false);
}

// Issue-order-pinned forms of the cell operations for the multi-chain
// kernel.  The compiler's scheduler models these instructions as cheap and
// emits each chain back to back; measured on gfx950 a dependent VALU
// instruction issues about 10 cycles after its producer, so the K chains of
// a lane are interleaved explicitly (volatile asm keeps its order).
__device__ __forceinline__ uint32_t asm_min3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm volatile("v_min3_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
__device__ __forceinline__ uint32_t asm_sad(uint32_t x, uint32_t y, uint32_t m) {
  uint32_t d;  // |x - y| + m on unsigned operands
  asm volatile("v_sad_u32 %0, %1, %2, %3" : "=v"(d) : "v"(x), "v"(y), "v"(m));
  return d;
}
__device__ __forceinline__ uint32_t asm_subf(uint32_t x, uint32_t y) {
  uint32_t d;  // x - y in float32 (bit patterns in and out)
  asm volatile("v_sub_f32 %0, %1, %2" : "=v"(d) : "v"(x), "v"(y));
  return d;
}
__device__ __forceinline__ uint32_t asm_addabs(uint32_t d, uint32_t m) {
  uint32_t r;  // |d| + m in float32
  asm volatile("v_add_f32_e64 %0, |%1|, %2" : "=v"(r) : "v"(d), "v"(m));
  return r;
}
// from_left_lane with its DPP in asm; the leading s_nop covers the two wait
// states a DPP read needs after a VALU write of its source.
__device__ __forceinline__ uint32_t asm_from_left_lane(uint32_t v, uint32_t lane0) {
  uint32_t r = lane0;
  asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 wave_shr:1 row_mask:0xf bank_mask:0xf"
               : "+v"(r)
               : "v"(v));
  return r;
}

// Four consecutive columns of one chain in one asm statement:
// n_c = |x - y_c| + min3(u_c, u_{c-1}, n_{c-1}) for c = 0..3, given the
// diagonal um = u_{-1} and the left value l = n_{-1}.
template <class F>
__device__ __forceinline__ void cells4(uint32_t x, uint32_t y0, uint32_t y1, uint32_t y2,
                                       uint32_t y3, uint32_t u0, uint32_t u1, uint32_t u2,
                                       uint32_t u3, uint32_t um, uint32_t l, uint32_t& n0,
                                       uint32_t& n1, uint32_t& n2, uint32_t& n3) {
  uint32_t t;
  if constexpr (std::is_same<F, FmtF32>::value) {
    uint32_t d0, d1, d2, d3;
    asm volatile(
        "v_sub_f32 %[d0], %[x], %[y0]\n\t"
        "v_min3_u32 %[t], %[u0], %[um], %[l]\n\t"
        "v_sub_f32 %[d1], %[x], %[y1]\n\t"
        "v_add_f32_e64 %[n0], |%[d0]|, %[t]\n\t"
        "v_sub_f32 %[d2], %[x], %[y2]\n\t"
        "v_min3_u32 %[t], %[u1], %[u0], %[n0]\n\t"
        "v_sub_f32 %[d3], %[x], %[y3]\n\t"
        "v_add_f32_e64 %[n1], |%[d1]|, %[t]\n\t"
        "v_min3_u32 %[t], %[u2], %[u1], %[n1]\n\t"
        "v_add_f32_e64 %[n2], |%[d2]|, %[t]\n\t"
        "v_min3_u32 %[t], %[u3], %[u2], %[n2]\n\t"
        "v_add_f32_e64 %[n3], |%[d3]|, %[t]"
        : [n0] "=&v"(n0), [n1] "=&v"(n1), [n2] "=&v"(n2), [n3] "=&v"(n3), [t] "=&v"(t),
          [d0] "=&v"(d0), [d1] "=&v"(d1), [d2] "=&v"(d2), [d3] "=&v"(d3)
        : [x] "v"(x), [y0] "v"(y0), [y1] "v"(y1), [y2] "v"(y2), [y3] "v"(y3), [u0] "v"(u0),
          [u1] "v"(u1), [u2] "v"(u2), [u3] "v"(u3), [um] "v"(um), [l] "v"(l));
  } else {
    asm volatile(
        "v_min3_u32 %[t], %[u0], %[um], %[l]\n\t"
        "v_sad_u32 %[n0], %[x], %[y0], %[t]\n\t"
        "v_min3_u32 %[t], %[u1], %[u0], %[n0]\n\t"
        "v_sad_u32 %[n1], %[x], %[y1], %[t]\n\t"
        "v_min3_u32 %[t], %[u2], %[u1], %[n1]\n\t"
        "v_sad_u32 %[n2], %[x], %[y2], %[t]\n\t"
        "v_min3_u32 %[t], %[u3], %[u2], %[n2]\n\t"
        "v_sad_u32 %[n3], %[x], %[y3], %[t]"
        : [n0] "=&v"(n0), [n1] "=&v"(n1), [n2] "=&v"(n2), [n3] "=&v"(n3), [t] "=&v"(t)
        : [x] "v"(x), [y0] "v"(y0), [y1] "v"(y1), [y2] "v"(y2), [y3] "v"(y3), [u0] "v"(u0),
          [u1] "v"(u1), [u2] "v"(u2), [u3] "v"(u3), [um] "v"(um), [l] "v"(l));
  }
}

// One row step of K interleaved chains over a lane's strip: chain h owns
// columns [h*H, (h+1)*H).  nw[c] = gamma(i_h, c) from up[c] = gamma(i_h - 1, c),
// the diagonal dprev[h] and left[h] = gamma(i_h, first column - 1), where
// i_h is chain h's row.  Instructions are issued column by column across the
// chains so that consecutive instructions of one chain are K apart.
// after(integral_constant<int, w>) runs once the cells of column w of every
// chain have been issued (the tile switch issues its LDS operations there).
struct NoAfter {
  template <class C>
  __device__ __forceinline__ void operator()(C) const {}
};
template <class F, int K, int H, int W, class After = NoAfter>
__device__ __forceinline__ void chains_row(const uint32_t (&x)[K], const uint32_t (&y)[W],
                                           const uint32_t (&up)[W], uint32_t (&nw)[W],
                                           const uint32_t (&dprev)[K],
                                           const uint32_t (&left)[K], After&& after = After{}) {
  if constexpr (K == 1) {
    // one chain: four columns per asm statement (the compiler separates
    // consecutive asm statements with a wait state)
    static_for<0, H / 4>([&](auto bc) {
      constexpr int c = 4 * decltype(bc)::value;
      cells4<F>(x[0], y[c], y[c + 1], y[c + 2], y[c + 3], up[c], up[c + 1], up[c + 2],
                up[c + 3], c ? up[c > 0 ? c - 1 : 0] : dprev[0],
                c ? nw[c > 0 ? c - 1 : 0] : left[0], nw[c], nw[c + 1], nw[c + 2], nw[c + 3]);
      after(std::integral_constant<int, c>{});
      after(std::integral_constant<int, c + 1>{});
      after(std::integral_constant<int, c + 2>{});
      after(std::integral_constant<int, c + 3>{});
    });
    return;
  }
  static_for<0, H>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    uint32_t m[K];
    if constexpr (std::is_same<F, FmtF32>::value) {
      uint32_t d[K];
#pragma unroll
      for (int h = 0; h < K; ++h) d[h] = asm_subf(x[h], y[h * H + w]);
#pragma unroll
      for (int h = 0; h < K; ++h) {
        const int c = h * H + w;
        m[h] = asm_min3(up[c], w ? up[c - 1] : dprev[h], w ? nw[c - 1] : left[h]);
      }
#pragma unroll
      for (int h = 0; h < K; ++h) nw[h * H + w] = asm_addabs(d[h], m[h]);
    } else {
#pragma unroll
      for (int h = 0; h < K; ++h) {
        const int c = h * H + w;
        m[h] = asm_min3(up[c], w ? up[c - 1] : dprev[h], w ? nw[c - 1] : left[h]);
      }
#pragma unroll
      for (int h = 0; h < K; ++h) nw[h * H + w] = asm_sad(x[h], y[h * H + w], m[h]);
    }
    after(wc);
  });
}

__device__ __forceinline__ void wave_argmin(uint32_t& best, int32_t& bestj) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t ob = (uint32_t)__shfl_xor((int)best, off);
    const int32_t oj = __shfl_xor(bestj, off);
    if (ob < best || (ob == best && oj < bestj)) {
      best = ob;
      bestj = oj;
    }
  }
}

template <int W>
__device__ __forceinline__ void load_strip(uint32_t (&dst)[W], const uint32_t* __restrict__ src) {
#pragma unroll
  for (int w = 0; w < W; w += 4) {
    const uint4 v = *(const uint4*)(src + w);
    dst[w] = v.x;
    dst[w + 1] = v.y;
    dst[w + 2] = v.z;
    dst[w + 3] = v.w;
  }
}

// ---------------------------------------------------------------------------
// Continuous-skew kernel
// ---------------------------------------------------------------------------

// K chains per lane.  Lane l's strip of W columns is cut into K sub-strips of
// H = W/K columns; sub-strip h is "sub-lane" s = K*l + h and works on row
// (t - s) mod M of its tile at step t.  Within a step the K sub-strips of a
// lane are independent dependency chains (each needs the edge its left
// neighbour produced one step earlier), which the hardware can overlap:
// chain 0 takes lane l-1's last-column edge by DPP, chain h > 0 takes the
// lane's own chain h-1 edge, still in its row buffer.
//
// P row bands.  A workgroup of P waves aligns one read: its M rows are cut
// into Pe <= P bands of consecutive rows (band g: rows [g M / Pe,
// (g + 1) M / Pe), each at least 64K + 1 rows) and wave g sweeps band g over
// every tile with the one-wave schedule above.  Row i of Eq. 1 depends on the
// rows above it only through row i - 1, so band g's "previous row" on a tile
// is band g - 1's last row on that tile; it is handed over through an LDS ring
// of two tile slots (and a ring of four values for each tile's last column,
// the diagonal lane 0 needs when it enters the next tile).  The workgroup
// runs global periods with one barrier after each; wave g runs its local
// period p = G - 2g, so a slot is written (during the writer's switch steps
// of its period t + 1) one barrier before it is read (during the reader's
// switch steps of its period t) and rewritten only after its last read.
// Pe = min(P, M / (64K + 1)), or fewer when a target band height is given
// (reads of different lengths then get bands of about the same height and
// finish together); waves g >= Pe idle through the barriers.
//
// LDS layout of the query and the left-boundary column of a band, one 8-byte
// entry per k in [0, M_g + 64K):
//   bx[k].x = band row (k - (64K - 1)) mod M_g   (biased int16 or float bits)
//   bx[k].y = boundary gamma(band row k - (64K - 1), last column of the
//             previous tile) for k in [64K - 1, M_g + 64K - 1)
// Chain h of lane l reads its row r of the current period at entry
// K(63 - l) + r + (K - 1 - h); so lane 0's chain 0 finds boundary row r at
// entry 64K - 1 + r, and the last sub-lane (lane 63, chain K-1) writes its
// boundary row r - (64K - 1) at entry r, its own entry (at r + M_g while that
// row is in the previous period).
//
// STREAM: each work item extends a resident row acc = gamma(m_old, .) by the
// M rows of one chunk (rows m_old+1 .. m_old+M of the read): when a sub-lane
// of band 0 enters a tile its previous row is acc's strip (instead of zeros)
// and its diagonal is acc one column to the left (+inf left of column 0),
// both copied into LDS a period ahead (the tile's reference values go to
// registers); the last band writes the finished last row of every tile back
// to acc.  A tile's acc is read at least one period before that tile's
// write-back, so reads see the row as it was before this extension.
//
// LDS (uint32 words, every array on 16 bytes): zeros[W] and a +inf cell
// (4 words); ring[P-1][2][64W]; edge[P-1][4]; then per band stage[64W] (in
// the last band the finished last rows, folded once a period) and bx; or,
// for STREAM, one stage[64W] (used by a read's last band alone), acc's
// next tile for band 0 (64W, after a 4-word block whose last word is the
// value left of the tile) and per band bx.  With the shared stage and no
// registers held for acc, two workgroups of four bands fit on a CU, so a
// launch of one chunk per CU (one wave per SIMD) leaves room for the next
// launch, of the same reference or another, to run beside it.
template <class F, int W, int K, int P, bool STREAM>
__global__ __launch_bounds__(64 * P, STREAM ? 2 : 1) void k_align_skew(AlignArgs args) {
  constexpr int T = 64 * W;
  constexpr int H = W / K;
  constexpr int S = 64 * K;                   // sub-lanes = switch steps per period
  constexpr int U = K > 2 ? K : 2;            // phase-A unroll: chain index compile-time
  constexpr bool kZeroRow = P == 1 && !STREAM;
  // Pipelined switches (issued between the previous step's cells) except
  // with one band and no resident row, where a switch loads nothing from LDS.
  constexpr bool kPipe = !kZeroRow;
  // columns per group of a pipelined switch's operations (each group is one
  // masked block: fewer, larger groups cost fewer exec-mask changes)
  constexpr int kGc = 8 < H ? 8 : H;
  static_assert(H % kGc == 0 && kGc % 4 == 0, "switch groups are whole uint4 groups");
  static_assert(W % K == 0 && H % 4 == 0, "sub-strips are whole uint4 groups");
  extern __shared__ __align__(16) uint32_t smem[];
  __shared__ int32_t s_item;
  const int lane = (int)threadIdx.x & 63;
  const int wave = P > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) : 0;
  uint32_t* const zeros = smem;
  uint32_t* const inf_cell = zeros + W;
  uint32_t* const ring = inf_cell + 4;
  uint32_t* const edge = ring + (P - 1) * 2 * T;
  // the last band's finished rows: one stage per band, or when extending
  // resident rows one for every band, followed by the first band's copy of
  // the resident row's next tile (a strip per lane) after a word holding
  // the value left of it
  uint32_t* const stage =
      edge + (P - 1) * 4 + (STREAM ? 0 : wave * skew_band_words(W, K, args.max_band));
  [[maybe_unused]] uint32_t* const accst = stage + T + 4;
  uint2* const bx = STREAM ? (uint2*)(accst + T + wave * skew_entry_words(K, args.max_band))
                           : (uint2*)(stage + T);
  uint32_t* const my_stage = stage + lane * W;
  uint2* const bxl = bx + K * (63 - lane);
  uint32_t* const ring_in = ring + (wave > 0 ? wave - 1 : 0) * 2 * T + lane * W;
  uint32_t* const ring_out = ring + (wave < P - 1 ? wave : 0) * 2 * T + lane * W;
  uint32_t* const edge_in = edge + (wave > 0 ? wave - 1 : 0) * 4;
  uint32_t* const edge_out = edge + (wave < P - 1 ? wave : 0) * 4;

  if (wave == 0) {
    if (lane < W) zeros[lane] = 0u;
    if (lane == 0) *inf_cell = F::kInf;
  }
  const int32_t N = (int32_t)args.n;
  const int32_t ntiles = (N + T - 1) / T;

  // Batch launches: where this wave runs.  A SIMD slot from the hardware ids
  // (XCC, shader engine, shader array, CU, SIMD) and the wave's place among
  // the launch's waves on that SIMD (j).  With two waves on a SIMD each
  // publishes the work its read has left once a period and takes the higher
  // issue priority while it has more left than the other: the SIMD then
  // finishes both together instead of running the longer one alone at the
  // end (one wave issues slower than two).  When a launch of two-wave
  // workgroups has no more reads than workgroups (each takes one, so no later
  // pull evens the load out), half the workgroups take theirs from the back
  // of the longest-first list: the dispatcher places the four workgroups of
  // a CU with their two waves on SIMDs (0, 2), (1, 3), (2, 1) and (3, 0), so
  // those whose first wave runs on SIMD 2 or 3 taking short reads pairs a
  // short read with a long one on every SIMD.  (Placement decides nothing
  // but speed: any placement gets every read exactly once.)
  [[maybe_unused]] uint32_t* rem_mine = nullptr;
  [[maybe_unused]] const uint32_t* rem_other = nullptr;
  [[maybe_unused]] uint32_t rem_seen = 0u;
  [[maybe_unused]] bool back = false;
  if constexpr (!STREAM) {
    uint32_t hw, xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    const uint32_t simd = (hw >> 4) & 3u;
    const uint32_t slot = (((((xcc & 7u) << 3 | ((hw >> 13) & 7u)) << 1 | ((hw >> 12) & 1u))
                            << 4 | ((hw >> 8) & 15u)) << 2) | simd;
    uint32_t* const cnt = args.sched + kSchedHead;
    uint32_t j = atomicAdd(cnt + slot, lane == 0 ? 1u : 0u);
    j = __builtin_amdgcn_readfirstlane(j);
    if (j < 2) {
      rem_mine = cnt + kSchedSimds + 2 * slot + j;
      rem_other = cnt + kSchedSimds + 2 * slot + (1 - j);
    }
    if (args.nwork <= (int32_t)gridDim.x) back = P > 1 && simd >= 2;
  }
  // Work pull without a divergent branch around the atomic: every lane of
  // the pulling wave takes part and only lane 0 adds, so lane 0's return
  // value is the item whatever order the lanes are serviced in.  (Guarding
  // the atomic with `if (lane == 0)` lets the loop structurizer split the
  // wave around the readfirstlane, leaving lanes 1..63 a stale item.)  A
  // batch pull takes the next item from the front or the back of the list
  // in one 64-bit add: the list is exhausted once front + back reaches its
  // length, so every item is taken exactly once.
  auto pull = [&]() -> int32_t {
    if constexpr (STREAM) {
      return __builtin_amdgcn_readfirstlane(atomicAdd(args.counter, lane == 0 ? 1 : 0));
    } else {
      const unsigned long long inc = back ? 1ull << 32 : 1ull;
      const unsigned long long old =
          atomicAdd((unsigned long long*)args.sched, lane == 0 ? inc : 0ull);
      const uint32_t f = __builtin_amdgcn_readfirstlane((uint32_t)old);
      const uint32_t b = __builtin_amdgcn_readfirstlane((uint32_t)(old >> 32));
      if (f + b >= (uint32_t)args.nwork) return args.nwork;
      return back ? args.nwork - 1 - (int32_t)b : (int32_t)f;
    }
  };

  for (;;) {
    int32_t item;
    if constexpr (P == 1) {
      item = pull();
      if (item >= args.nwork) break;
      __syncthreads();  // previous read's LDS use is complete
    } else {
      __syncthreads();  // every wave is done with the previous item and its LDS
      if (wave == 0) {
        const int32_t it = pull();
        if (lane == 0) s_item = it;
      }
      __syncthreads();
      item = __builtin_amdgcn_readfirstlane(s_item);
      if (item >= args.nwork) break;
    }
    int32_t rd, M, m_old = 0;
    int64_t q0;
    uint32_t* acc = nullptr;
    if constexpr (STREAM) {
      const StreamItem it = args.items[item];
      q0 = it.q0;
      M = __builtin_amdgcn_readfirstlane(it.m);
      m_old = __builtin_amdgcn_readfirstlane(it.m_old);
      rd = __builtin_amdgcn_readfirstlane(it.out);
      acc = it.acc;
    } else {
      rd = __builtin_amdgcn_readfirstlane(args.order ? args.order[item] : item);
      q0 = args.offs ? args.offs[rd] : 0;
      M = __builtin_amdgcn_readfirstlane(args.offs ? (int32_t)(args.offs[rd + 1] - q0)
                                                   : args.single_m);
    }
    int32_t Pe = 1;
    if constexpr (P > 1) Pe = skew_read_bands(M, K, P, args.band_target);
    const bool active = wave < Pe;
    const bool last = wave == Pe - 1;
    const int32_t r0 = (wave * M) / Pe;
    const int32_t Mb = ((wave + 1) * M) / Pe - r0;  // this band's rows
    const typename F::qin* __restrict__ qv = (const typename F::qin*)args.q + q0 + r0;
    // A lane's strip of the tile it enters next waits in registers: loaded
    // from global memory once every lane has entered the current tile,
    // copied by each lane when it enters the next one.  When a resident row
    // is extended (m_old > 0), band 0's previous row of the next tile goes
    // from global memory straight into LDS (accst, no registers: the copies
    // land while the band computes) and the value left of the tile into one
    // register, which lane 0 stores in front of the copy before the tile's
    // switch steps.  A fresh read (m_old == 0) has gamma(0, .) = 0.
    uint32_t ynext[W];
    [[maybe_unused]] uint32_t accleftnext = F::kInf;
    [[maybe_unused]] const bool resident = STREAM && m_old > 0;
    auto load_acc = [&](int32_t t) {
      if constexpr (STREAM) {
        if (resident) {
          // 64 lanes x 16 bytes per copy, lane l's bytes at 16 l: copy c of
          // the tile's 4 T bytes covers words [256 c, 256 c + 256)
          const uint32_t* src = acc + (int64_t)t * T + 4 * lane;
#pragma unroll
          for (int c = 0; c < T / 256; ++c)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void*)(src + 256 * c),
                (__attribute__((address_space(3))) void*)(accst + 256 * c), 16, 0, 0);
          accleftnext = t > 0 ? acc[(int64_t)t * T - 1] : F::kInf;
        }
      }
    };

    if (active) {
      for (int k = lane; k < Mb + S; k += 64) {
        int s = k - (S - 1);
        s = s < 0 ? s + Mb : (s >= Mb ? s - Mb : s);
        bx[k] = make_uint2((uint32_t)F::to_lds(qv[s]), F::kInf);  // gamma(i, 0) = +inf
      }
      load_strip<W>(ynext, args.ref + lane * W);
      if (wave == 0) load_acc(0);
    }
    __syncthreads();

    uint32_t y[W], a[W], b[W], dprev[K];
#pragma unroll
    for (int w = 0; w < W; ++w) y[w] = a[w] = b[w] = 0u;
#pragma unroll
    for (int h = 0; h < K; ++h) dprev[h] = F::kInf;
    uint32_t best = 0xFFFFFFFFu;
    int32_t bestj = INT_MAX;

    // The entries of step r + 1 are read during step r (before step r's own
    // boundary write): lane 0's row r + 1 was written by the last sub-lane
    // at least two steps earlier when M_g >= 64K + 1, which the launcher
    // guarantees.  Only chain 0 takes a boundary value; chains h > 0 load the
    // query half of their entry alone, so that every register a prefetch
    // writes stays live until the next step (a dead half would let the
    // register allocator reuse it at once and wait for the load right there).
    uint2 nxt0;
    uint32_t nxtx[K];
    auto load_entries = [&](int32_t r) {
      nxt0 = bxl[r + (K - 1)];
#pragma unroll
      for (int h = 1; h < K; ++h) nxtx[h] = bxl[r + (K - 1 - h)].x;
    };
    // Per period: where a sub-lane entering tile p takes its previous row
    // (zeros, the staged resident row, or the band above's ring slot) and the
    // diagonal left of it, and where its finished strip of tile p - 1 goes
    // (the stage in the last band, for the fold; the ring otherwise).
    int32_t p = 0;
    const uint32_t* upsrc = zeros;
    const uint32_t* d0src = zeros;
    uint32_t* fin = my_stage;
    // The last lane's boundary store of a step is issued at the top of the
    // next step, after that step's lane shift and before its prefetch: the
    // store still precedes every read of its row, and the shift then waits
    // only for the prefetch issued a whole step earlier (a store issued just
    // before it, under the lane mask, would be waited for as well).
    bool pend = false;
    int32_t pend_i = 0;
    uint32_t pend_v = 0;
    auto flush = [&]() {
      if (pend && lane == 63) bxl[pend_i].y = pend_v;
      pend = false;
    };
    // One row step.
    //   SW >= 0: sub-lane r (lane r / K, chain SW == r % K) enters its next
    //     tile in this step.  With FULL its whole switch is done here, at the
    //     top of the step (the first step of a period); otherwise the switch
    //     was issued during the previous step and only the previous-row
    //     reload of its last group of four columns is left, done here after
    //     the edges its right neighbours need have been read from it.
    //   NX >= 0: sub-lane r + 1 (chain NX) enters its next tile in the next
    //     step; this step has computed its last row on the old tile, and its
    //     switch is issued between this step's cells, each group of four
    //     columns right after the cell that last reads the group's registers:
    //     new reference values from the stage, the finished row out (the last
    //     band's fin is the stage itself, so each group is read before it is
    //     overwritten), the new previous row into the registers just stored
    //     (zeros, the staged resident row or the band above's ring slot).
    //     The next step's cells then find their operands in place instead of
    //     waiting for a round of LDS operations.
    // Where a sub-lane entering a tile takes its previous row: band 0 of a
    // fresh read from registers (gamma(0, .) = 0, as every other column
    // cleared, which puts a zero in every cell's minimum once the diagonal
    // left of the sub-strip is 0 too), band 0 of a resident row from its LDS
    // copy, the other bands from the band above's ring slot in LDS.
    // (UR: band 0 of a fresh read, whose phase A is compiled apart)
    auto diag_in = [&](auto ur, auto hc) -> uint32_t {  // the value left of sub-strip h
      constexpr bool UR = decltype(ur)::value;
      constexpr int h = decltype(hc)::value;
      if constexpr (UR) {
        return 0u;
      } else if constexpr (h == 0) {
        return *d0src;
      } else {
        return upsrc[h > 0 ? h * H - 1 : 0];
      }
    };
    auto prev_in = [&](auto ur, uint32_t(&dst)[W], int w) {  // columns [w, w + 4)
      if constexpr (decltype(ur)::value) {
        dst[w + 1] = 0u;
        dst[w + 3] = 0u;
      } else {
        const uint4 zv = *(const uint4*)(upsrc + w);
        dst[w] = zv.x;
        dst[w + 1] = zv.y;
        dst[w + 2] = zv.z;
        dst[w + 3] = zv.w;
      }
    };
    auto step = [&](auto ur, auto sw, auto nx, auto full, int32_t r, uint32_t(&up)[W],
                    uint32_t(&nw)[W], bool write_b, bool wrap) {
      constexpr int SW = decltype(sw)::value;
      constexpr int NX = decltype(nx)::value;
      constexpr bool FULL = decltype(full)::value;
      const uint2 e0 = nxt0;
      uint32_t xs[K];
#pragma unroll
      for (int h = 1; h < K; ++h) xs[h] = nxtx[h];
      xs[0] = e0.x;
      uint32_t left[K];
      if constexpr (K == 1)
        left[0] = from_left_lane(up[W - 1], e0.y);
      else
        left[0] = asm_from_left_lane(up[W - 1], e0.y);
      flush();
      load_entries(r + 1);
      // keep the prefetch at the top of the step: scheduled next to its use,
      // as the compiler would otherwise place it, every step waits for it
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = 1; h < K; ++h) left[h] = up[h * H - 1];
      if constexpr (SW >= 0) {
        if (lane == r / K) {
          // the band below needs this tile's last column (lane 63's last
          // value of the finished row), read before the last group reloads
          if constexpr (P > 1 && SW == K - 1) {
            if (!last && lane == 63) edge_out[(p - 1) & 3] = up[W - 1];
          }
          if constexpr (FULL) {
            dprev[SW] = diag_in(ur, std::integral_constant<int, SW>{});
#pragma unroll
            for (int w = SW * H; w < (SW + 1) * H; w += 4) {
              y[w] = ynext[w];
              y[w + 1] = ynext[w + 1];
              y[w + 2] = ynext[w + 2];
              y[w + 3] = ynext[w + 3];
              *(uint4*)(fin + w) = make_uint4(up[w], up[w + 1], up[w + 2], up[w + 3]);
              prev_in(ur, up, w);
              __builtin_amdgcn_sched_barrier(0);
            }
          } else {
#pragma unroll
            for (int w = (SW + 1) * H - kGc; w < (SW + 1) * H; w += 4) prev_in(ur, up, w);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // the next sub-lane's switch, issued between the cells
      [[maybe_unused]] const bool nxt = NX >= 0 && lane == (r + 1) / K;
      [[maybe_unused]] uint32_t dnext = 0;
      auto after = [&](auto wc) {
        if constexpr (NX >= 0) {
          constexpr int wl = decltype(wc)::value;  // column within the sub-strips
          // group g of the next sub-strip, once column 4g + 4 (the last cell
          // reading the group's previous and current row) has been issued;
          // the last group's reference values and finished row after the
          // last column, its previous row at the top of the next step
          constexpr int g = wl == H - 1 ? H / kGc - 1 : wl / kGc - 1;
          if constexpr ((wl >= kGc && wl % kGc == 0) || wl == H - 1) {
            __builtin_amdgcn_sched_barrier(0);
            if (nxt) {
              // the diagonal left of the next strip, early: the next step's
              // first cell needs it
              if constexpr (g == 0) dnext = diag_in(ur, std::integral_constant<int, NX>{});
#pragma unroll
              for (int w = NX * H + kGc * g; w < NX * H + kGc * (g + 1); w += 4) {
                y[w] = ynext[w];
                y[w + 1] = ynext[w + 1];
                y[w + 2] = ynext[w + 2];
                y[w + 3] = ynext[w + 3];
                *(uint4*)(fin + w) = make_uint4(nw[w], nw[w + 1], nw[w + 2], nw[w + 3]);
                if constexpr (wl != H - 1) prev_in(ur, nw, w);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      };
      if constexpr (K == 1 && NX < 0)
        strip_row<F, W>(xs[0], y, up, nw, dprev[0], left[0]);
      else
        chains_row<F, K, H, W>(xs, y, up, nw, dprev, left, after);
#pragma unroll
      for (int h = 0; h < K; ++h) dprev[h] = left[h];
      if constexpr (NX >= 0) {
        if (nxt) dprev[NX] = dnext;
      }
      pend = write_b;
      pend_i = wrap ? r + Mb : r;
      pend_v = nw[W - 1];
    };
    auto plain = [&](int32_t r, uint32_t(&up)[W], uint32_t(&nw)[W]) {
      using NoSwitch = std::integral_constant<int, -1>;
      step(std::false_type{}, NoSwitch{}, NoSwitch{}, std::false_type{}, r, up, nw, true, false);
    };

    const int32_t nglob = ntiles + 1 + 2 * (Pe - 1);
    for (int32_t G = 0; G < nglob; ++G) {
      p = G - 2 * wave;
      if (active && p >= 0 && p <= ntiles) {
        if (wave == 0) {
          upsrc = zeros;  // not read: a fresh read's previous row is cleared registers
          d0src = zeros;
          if constexpr (STREAM) {
            if (resident) {
              // the copies of tile p (issued a period earlier, or for tile 0
              // when the read was taken) have landed
              asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
              if (lane == 0) accst[-1] = accleftnext;
              upsrc = accst + lane * W;
              d0src = upsrc - 1;  // lane 0: the value left of the tile
            }
          }
        } else {
          upsrc = ring_in + (p & 1) * T;
          d0src = lane > 0 ? upsrc - 1 : (p > 0 ? edge_in + ((p - 1) & 3) : inf_cell);
        }
        fin = last ? my_stage : ring_out + ((p - 1) & 1) * T;
        // phase A: the 64K switch steps.  Step 0 switches sub-lane 0 at its
        // top (its previous row may come from the ring slot the band above
        // wrote in the previous global period); every later switch is issued
        // one step early, between the cells of the step before.
        const bool first = (p == 0);
        load_entries(0);  // row 0 of the period (entry 64K - 1 + M_g is not kept)
        // phase A is compiled twice: band 0 takes its previous row from
        // registers, the other bands from the ring
        auto phase_a = [&](auto ur) {
          if constexpr (kPipe) {
            using C0 = std::integral_constant<int, 0>;
            using C1 = std::integral_constant<int, 1 % K>;
            using Yes = std::true_type;
            using No = std::false_type;
            step(ur, C0{}, C1{}, Yes{}, 0, a, b, !first || S == 1, true);
            // steps 1 .. S - U: blocks of U (step r's sub-lane chain is r % K
            // and its registers alternate with r's parity; U is even and a
            // multiple of K)
            for (int32_t r = 1; r + U - 1 < S; r += U) {
              static_for<0, U>([&](auto uu) {
                constexpr int u = decltype(uu)::value;
                constexpr int sw = (1 + u) % K, nx = (2 + u) % K;
                using Sw = std::integral_constant<int, sw>;
                using Nx = std::integral_constant<int, nx>;
                if constexpr (u % 2 == 0)
                  step(ur, Sw{}, Nx{}, No{}, r + u, b, a, !first, true);
                else
                  step(ur, Sw{}, Nx{}, No{}, r + u, a, b, !first, true);
              });
            }
            // steps S - U + 1 .. S - 1 (the last has no successor to switch)
            static_for<0, U - 1>([&](auto uu) {
              constexpr int u = decltype(uu)::value;
              constexpr int rr = S - U + 1 + u;
              constexpr int sw = rr % K;
              using Nx = std::integral_constant<int, rr + 1 < S ? (rr + 1) % K : -1>;
              if constexpr (rr % 2 == 1)
                step(ur, std::integral_constant<int, sw>{}, Nx{}, No{}, rr, b, a,
                     !first || rr == S - 1, rr != S - 1);
              else
                step(ur, std::integral_constant<int, sw>{}, Nx{}, No{}, rr, a, b,
                     !first || rr == S - 1, rr != S - 1);
            });
          } else {
            for (int32_t r = 0; r < S; r += U) {
              static_for<0, U / 2>([&](auto uu) {
                constexpr int u = 2 * decltype(uu)::value;
                using NoNext = std::integral_constant<int, -1>;
                using Sw0 = std::integral_constant<int, u % K>;
                using Sw1 = std::integral_constant<int, (u + 1) % K>;
                step(ur, Sw0{}, NoNext{}, std::true_type{}, r + u, a, b,
                     !first || r + u == S - 1, r + u != S - 1);
                step(ur, Sw1{}, NoNext{}, std::true_type{}, r + u + 1, b, a,
                     !first || r + u + 1 == S - 1, r + u + 1 != S - 1);
              });
            }
          }
        };
        if (wave == 0 && !resident)
          phase_a(std::true_type{});
        else if constexpr (P > 1 || STREAM)
          phase_a(std::false_type{});
        flush();
        // every lane has finished tile p-1: the last band folds its last row
        // (and writes it back as the new resident row); stage tile p+1
        if (p >= 1 && last) {
          const int32_t jb = (p - 1) * T + lane * W;
          uint32_t lr[W];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            lr[w] = my_stage[w];
            if (jb + w < N && lr[w] < best) {
              best = lr[w];
              bestj = jb + w;
            }
          }
          if constexpr (STREAM) {
#pragma unroll
            for (int w = 0; w < W; w += 4)
              *(uint4*)(acc + jb + w) = make_uint4(lr[w], lr[w + 1], lr[w + 2], lr[w + 3]);
          }
        }
        if (p + 1 < ntiles) {
          // every lane has copied tile p: fetch tile p + 1
          load_strip<W>(ynext, args.ref + (int64_t)(p + 1) * T + lane * W);
          if (wave == 0) load_acc(p + 1);
        }
        if (p < ntiles) {
          // phase B: plain steps, four per iteration
          int32_t r = S;
          for (; r + 3 < Mb; r += 4) {
            plain(r, a, b);
            plain(r + 1, b, a);
            plain(r + 2, a, b);
            plain(r + 3, b, a);
          }
          for (; r + 1 < Mb; r += 2) {
            plain(r, a, b);
            plain(r + 1, b, a);
          }
          if (r < Mb) {
            plain(r, a, b);
#pragma unroll
            for (int w = 0; w < W; ++w) a[w] = b[w];
          }
          flush();
        }
        if constexpr (!STREAM) {
          if (rem_mine) {
            const uint32_t rem =
                (uint32_t)std::min<int64_t>((int64_t)(ntiles - p) * Mb, 0xFFFFFFFFll);
            if (rem > rem_seen)
              __builtin_amdgcn_s_setprio(1);
            else
              __builtin_amdgcn_s_setprio(0);
            if (lane == 0) __hip_atomic_store(rem_mine, rem, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            // read now, used at the end of the next period
            rem_seen = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(rem_other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          }
        }
      }
      if constexpr (P > 1) __syncthreads();
    }

    if (last) {
      wave_argmin(best, bestj);
      if (lane == 0) {
        F::store_cost(args.cost, rd, best);
        args.end[rd] = bestj;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Synchronised-tile kernel (any M >= 1)
// ---------------------------------------------------------------------------

template <class F, int W>
struct PlainLds {
  static size_t bytes(int max_m) {
    size_t b = 4 * ((size_t)64 * W + (size_t)max_m) + sizeof(typename F::xlds) * (size_t)max_m;
    return (b + 15) & ~(size_t)15;
  }
};

// STREAM: as k_align_skew's streaming mode, per tile: the previous row is
// the resident row's strip and the diagonal the resident value to its left;
// the finished last row of tile t-1 is written back after tile t's resident
// values have been read (lane 0 reads the column that lane 63 writes back).
template <class F, int W, bool STREAM>
__global__ __launch_bounds__(64) void k_align_plain(AlignArgs args) {
  constexpr int T = 64 * W;
  using X = typename F::xlds;
  extern __shared__ __align__(16) uint32_t smem[];
  const int lane = (int)threadIdx.x;
  const int32_t item = (int32_t)blockIdx.x;
  if (item >= args.nwork) return;
  uint32_t* const slot = smem;  // last-row strips
  uint32_t* const B = slot + 64 * W;
  X* const xs = (X*)(B + args.max_m);
  uint32_t* const my_slot = slot + lane * W;

  int32_t rd, M, m_old = 0;
  int64_t q0;
  uint32_t* acc = nullptr;
  if constexpr (STREAM) {
    const StreamItem it = args.items[item];
    q0 = it.q0;
    M = it.m;
    m_old = it.m_old;
    rd = it.out;
    acc = it.acc;
  } else {
    rd = args.order ? args.order[item] : item;
    q0 = args.offs ? args.offs[rd] : 0;
    M = args.offs ? (int32_t)(args.offs[rd + 1] - q0) : args.single_m;
  }
  const typename F::qin* __restrict__ qv = (const typename F::qin*)args.q + q0;
  for (int k = lane; k < M; k += 64) {
    xs[k] = F::to_lds(qv[k]);
    B[k] = F::kInf;
  }
  __syncthreads();

  const int64_t N = args.n;
  const int32_t ntiles = (int32_t)((N + T - 1) / T);
  uint32_t best = 0xFFFFFFFFu;
  int32_t bestj = INT_MAX;
  for (int32_t t = 0; t < ntiles; ++t) {
    uint32_t y[W], a[W], b[W];
    load_strip<W>(y, args.ref + (int64_t)t * T + lane * W);
    uint32_t dprev = F::kInf;
    const int64_t c0 = (int64_t)t * T + lane * W;
    if (STREAM && m_old > 0) {
      load_strip<W>(a, acc + c0);
      if (c0 > 0) dprev = acc[c0 - 1];
#pragma unroll
      for (int w = 0; w < W; ++w) b[w] = a[w];
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) a[w] = b[w] = 0u;
    }
    if constexpr (STREAM) {
      if (t > 0) {
        // the resident values above are in registers before any write-back
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int w = 0; w < W; w += 4)
          *(uint4*)(acc + c0 - T + w) =
              make_uint4(my_slot[w], my_slot[w + 1], my_slot[w + 2], my_slot[w + 3]);
      }
    }
    auto step = [&](int32_t s, const uint32_t(&up)[W], uint32_t(&nw)[W]) {
      const uint32_t left = from_left_lane(up[W - 1], B[s < M ? s : M - 1]);
      const int32_t i = s - lane;
      if ((uint32_t)i < (uint32_t)M) {
        strip_row<F, W>((uint32_t)xs[i], y, up, nw, dprev, left);
        dprev = left;
        if (lane == 63) B[i] = nw[W - 1];
        if (i == M - 1) {
#pragma unroll
          for (int w = 0; w < W; ++w) my_slot[w] = nw[w];
        }
      }
    };
    for (int32_t s = 0; s < M + 63; s += 2) {
      step(s, a, b);
      step(s + 1, b, a);
    }
    __syncthreads();
    const int32_t jb = t * T + lane * W;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t v = my_slot[w];
      if (jb + w < N && v < best) {
        best = v;
        bestj = jb + w;
      }
    }
    __syncthreads();
  }
  if constexpr (STREAM) {
    const int64_t c0 = (int64_t)(ntiles - 1) * T + lane * W;
#pragma unroll
    for (int w = 0; w < W; w += 4)
      *(uint4*)(acc + c0 + w) =
          make_uint4(my_slot[w], my_slot[w + 1], my_slot[w + 2], my_slot[w + 3]);
  }
  wave_argmin(best, bestj);
  if (lane == 0) {
    F::store_cost(args.cost, rd, best);
    args.end[rd] = bestj;
  }
}

__global__ void k_reset_counter(int32_t* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

__global__ void k_reset_sched(uint32_t* s) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kSchedWords; i += gridDim.x * blockDim.x)
    s[i] = 0u;
}

template <class F, int W, int K, int P, bool STREAM>
hipError_t launch_skew_t(int blocks, const AlignArgs& a, hipStream_t st) {
  const size_t lds = std::max(skew_lds_bytes(W, K, P, a.max_band, STREAM), (size_t)a.lds_bytes);
  hipError_t e = hipFuncSetAttribute((const void*)k_align_skew<F, W, K, P, STREAM>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (STREAM)
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, a.counter);
  else
    hipLaunchKernelGGL(k_reset_sched, dim3(kSchedWords / 1024), dim3(256), 0, st, a.sched);
  hipLaunchKernelGGL((k_align_skew<F, W, K, P, STREAM>), dim3(blocks), dim3(64 * P), lds, st, a);
  return hipGetLastError();
}

template <class F, int W, int K, int P>
hipError_t launch_skew_s(int blocks, const AlignArgs& a, hipStream_t st, bool stream) {
  return stream ? launch_skew_t<F, W, K, P, true>(blocks, a, st)
                : launch_skew_t<F, W, K, P, false>(blocks, a, st);
}

template <class F, int W>
hipError_t launch_plain_t(const AlignArgs& a, hipStream_t st, bool stream) {
  const size_t lds = PlainLds<F, W>::bytes(a.max_m);
  const void* fn = stream ? (const void*)k_align_plain<F, W, true>
                          : (const void*)k_align_plain<F, W, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (stream)
    hipLaunchKernelGGL((k_align_plain<F, W, true>), dim3(a.nwork), dim3(64), lds, st, a);
  else
    hipLaunchKernelGGL((k_align_plain<F, W, false>), dim3(a.nwork), dim3(64), lds, st, a);
  return hipGetLastError();
}

// the (strip, chains, bands) set valid_skew_config() admits
template <class F>
hipError_t launch_skew_f(int strip, int chains, int bands, int blocks, const AlignArgs& a,
                         hipStream_t st, bool stream) {
  switch ((strip * 8 + chains) * 8 + bands) {
    case (8 * 8 + 1) * 8 + 1: return launch_skew_s<F, 8, 1, 1>(blocks, a, st, stream);
    case (8 * 8 + 2) * 8 + 1: return launch_skew_s<F, 8, 2, 1>(blocks, a, st, stream);
    case (16 * 8 + 1) * 8 + 1: return launch_skew_s<F, 16, 1, 1>(blocks, a, st, stream);
    case (16 * 8 + 2) * 8 + 1: return launch_skew_s<F, 16, 2, 1>(blocks, a, st, stream);
    case (16 * 8 + 4) * 8 + 1: return launch_skew_s<F, 16, 4, 1>(blocks, a, st, stream);
    case (32 * 8 + 1) * 8 + 1: return launch_skew_s<F, 32, 1, 1>(blocks, a, st, stream);
    case (32 * 8 + 2) * 8 + 1: return launch_skew_s<F, 32, 2, 1>(blocks, a, st, stream);
    case (32 * 8 + 4) * 8 + 1: return launch_skew_s<F, 32, 4, 1>(blocks, a, st, stream);
    case (16 * 8 + 1) * 8 + 2: return launch_skew_s<F, 16, 1, 2>(blocks, a, st, stream);
    case (16 * 8 + 1) * 8 + 4: return launch_skew_s<F, 16, 1, 4>(blocks, a, st, stream);
    case (16 * 8 + 2) * 8 + 2: return launch_skew_s<F, 16, 2, 2>(blocks, a, st, stream);
    case (16 * 8 + 2) * 8 + 4: return launch_skew_s<F, 16, 2, 4>(blocks, a, st, stream);
    case (16 * 8 + 1) * 8 + 3: return launch_skew_s<F, 16, 1, 3>(blocks, a, st, stream);
    case (32 * 8 + 1) * 8 + 2: return launch_skew_s<F, 32, 1, 2>(blocks, a, st, stream);
    case (32 * 8 + 2) * 8 + 2: return launch_skew_s<F, 32, 2, 2>(blocks, a, st, stream);
    case (32 * 8 + 1) * 8 + 3: return launch_skew_s<F, 32, 1, 3>(blocks, a, st, stream);
    case (32 * 8 + 1) * 8 + 4: return launch_skew_s<F, 32, 1, 4>(blocks, a, st, stream);
  }
  return hipErrorInvalidValue;
}

template <class F>
hipError_t launch_plain_f(int strip, const AlignArgs& a, hipStream_t st, bool stream) {
  switch (strip) {
    case 8: return launch_plain_t<F, 8>(a, st, stream);
    case 16: return launch_plain_t<F, 16>(a, st, stream);
    case 32: return launch_plain_t<F, 32>(a, st, stream);
  }
  return hipErrorInvalidValue;
}

template <class F>
size_t plain_bytes_f(int strip, int max_m) {
  switch (strip) {
    case 8: return PlainLds<F, 8>::bytes(max_m);
    case 16: return PlainLds<F, 16>::bytes(max_m);
    case 32: return PlainLds<F, 32>::bytes(max_m);
  }
  return 0;
}

}  // namespace

hipError_t launch_align_skew(int dtype, int strip, int chains, int bands, int blocks,
                             const AlignArgs& a, hipStream_t st, bool stream) {
  if (!valid_skew_config(strip, chains, bands)) return hipErrorInvalidValue;
  return dtype == SDTW_I16 ? launch_skew_f<FmtI16>(strip, chains, bands, blocks, a, st, stream)
                           : launch_skew_f<FmtF32>(strip, chains, bands, blocks, a, st, stream);
}

hipError_t launch_align_plain(int dtype, int strip, const AlignArgs& a, hipStream_t st,
                              bool stream) {
  return dtype == SDTW_I16 ? launch_plain_f<FmtI16>(strip, a, st, stream)
                           : launch_plain_f<FmtF32>(strip, a, st, stream);
}

size_t plain_lds_bytes(int dtype, int strip, int max_m) {
  return dtype == SDTW_I16 ? plain_bytes_f<FmtI16>(strip, max_m)
                           : plain_bytes_f<FmtF32>(strip, max_m);
}

}  // namespace sdtw
