// Best and runner-up ends of resident last rows (section 5.1: a mapping
// quality is computed from the mapped positions and their scores before the
// selection decision).
//
// For a row gamma(m, 0..N): best = the first column with the minimum (the
// strict-less last-row scan of Algorithms 1 and 2, the same end as the
// extension that produced the row); second = the first column with the
// minimum among the columns farther than `window` from best.  Values are the
// kernels' cost encoding (uint32 sums on the int16 path, float32 bits of
// non-negative values on the float32 path), so one unsigned comparison
// orders both, and the 64-bit key (value << 32) | column orders (value,
// column) lexicographically: "first column with the minimum" is the minimum
// key.
//
// Two launches, so that a long row is read by many compute units:
//   k_segment_min  one workgroup per (row, segment of kSegment columns): the
//                  segment's minimum key -> part[row * S + segment].
//   k_best_two     one workgroup per row: best = minimum over the row's S
//                  keys; second = minimum over the keys of segments that lie
//                  wholly outside [best - window, best + window], and over a
//                  rescan of the (at most two) segments the window cuts,
//                  skipping the columns inside it.
// HBM-bound: 4N bytes per row in the first launch, at most 2 * 4 * kSegment
// plus 8 S in the second.
#include <limits.h>

#include "common.h"

namespace sdtw {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kNone = ~0ull;

__device__ __forceinline__ uint64_t key_of(uint32_t v, int64_t c) {
  return ((uint64_t)v << 32) | (uint64_t)(uint32_t)c;
}

// minimum key over the workgroup, returned to every thread
__device__ __forceinline__ uint64_t block_min(uint64_t k, uint64_t* sk) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)k, off);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(k >> 32), off);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    k = o < k ? o : k;
  }
  if ((threadIdx.x & 63) == 0) sk[threadIdx.x >> 6] = k;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) k = sk[w] < k ? sk[w] : k;
  __syncthreads();  // sk may be reused by the next call
  return k;
}

// Minimum key of columns [a, b) of `row` (a a multiple of 4), skipping the
// columns in [lo, hi]; this thread's share only.
__device__ __forceinline__ uint64_t scan_min(const uint32_t* __restrict__ row, int64_t a,
                                             int64_t b, int64_t lo, int64_t hi) {
  uint64_t k = kNone;
  const uint4* __restrict__ p = (const uint4*)row;
  const int64_t g0 = a / 4, g1 = (b + 3) / 4;  // rows are padded past n to whole uint4s
#pragma unroll 4
  for (int64_t g = g0 + threadIdx.x; g < g1; g += kThreads) {
    const uint4 q = p[g];
    const uint32_t e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t c = 4 * g + t;
      if (c < b && (c < lo || c > hi)) {
        const uint64_t kk = key_of(e[t], c);
        k = kk < k ? kk : k;
      }
    }
  }
  return k;
}

__global__ __launch_bounds__(kThreads) void k_segment_min(const StreamItem* __restrict__ items,
                                                          int64_t n, int32_t S,
                                                          uint64_t* __restrict__ part) {
  __shared__ uint64_t sk[kThreads / 64];
  const int64_t blk = (int64_t)blockIdx.x;
  const int32_t s = (int32_t)(blk / S), seg = (int32_t)(blk % S);
  const int64_t a = (int64_t)seg * kBestTwoSegment;
  const int64_t b = a + kBestTwoSegment < n ? a + kBestTwoSegment : n;
  const uint64_t k = block_min(scan_min(items[s].acc, a, b, 1, 0), sk);  // lo > hi: no skip
  if (threadIdx.x == 0) part[blk] = k;
}

template <bool F32>
__global__ __launch_bounds__(kThreads) void k_best_two(const StreamItem* __restrict__ items,
                                                       int64_t n, int32_t S, int32_t window,
                                                       const uint64_t* __restrict__ part,
                                                       void* best_cost, int32_t* best_end,
                                                       void* second_cost, int32_t* second_end) {
  __shared__ uint64_t sk[kThreads / 64];
  const int32_t s = (int32_t)blockIdx.x;
  const uint64_t* __restrict__ my = part + (int64_t)s * S;

  uint64_t k = kNone;
  for (int32_t g = threadIdx.x; g < S; g += kThreads) k = my[g] < k ? my[g] : k;
  const uint64_t best = block_min(k, sk);
  const int64_t jb = (int64_t)(uint32_t)best;
  const int64_t lo = jb - window, hi = jb + window;

  // segments wholly outside the window keep their minimum
  k = kNone;
  for (int32_t g = threadIdx.x; g < S; g += kThreads) {
    const int64_t a = (int64_t)g * kBestTwoSegment;
    const int64_t last = (a + kBestTwoSegment < n ? a + kBestTwoSegment : n) - 1;
    if (last < lo || a > hi) k = my[g] < k ? my[g] : k;
  }
  // segments the window cuts hold lo or hi: rescan them without the window
  const int64_t glo = lo >= 0 && lo < n ? lo / kBestTwoSegment : -1;
  const int64_t ghi = hi >= 0 && hi < n ? hi / kBestTwoSegment : -1;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t g = t == 0 ? glo : (ghi != glo ? ghi : -1);
    if (g < 0) continue;
    const int64_t a = g * kBestTwoSegment;
    const int64_t b = a + kBestTwoSegment < n ? a + kBestTwoSegment : n;
    if (a >= lo && b - 1 <= hi) continue;  // wholly inside: nothing to rescan
    const uint64_t kk = scan_min(items[s].acc, a, b, lo, hi);
    k = kk < k ? kk : k;
  }
  const uint64_t second = block_min(k, sk);

  if (threadIdx.x == 0) {
    const int32_t out = items[s].out;
    const bool none = second == kNone;
    const uint32_t vb = (uint32_t)(best >> 32), v2 = (uint32_t)(second >> 32);
    if constexpr (F32) {
      ((float*)best_cost)[out] = __uint_as_float(vb);
      ((float*)second_cost)[out] = none ? __uint_as_float(0x7F800000u) : __uint_as_float(v2);
    } else {
      ((int32_t*)best_cost)[out] = (int32_t)vb;
      ((int32_t*)second_cost)[out] = none ? INT_MAX : (int32_t)v2;
    }
    best_end[out] = (int32_t)jb;
    second_end[out] = none ? -1 : (int32_t)(uint32_t)second;
  }
}

}  // namespace

int64_t best_two_segments(int64_t n) { return (n + kBestTwoSegment - 1) / kBestTwoSegment; }

hipError_t launch_best_two(int dtype, const StreamItem* items, int32_t ns, int64_t n,
                           int32_t window, uint64_t* part, void* best_cost, int32_t* best_end,
                           void* second_cost, int32_t* second_end, hipStream_t st) {
  const int64_t S = best_two_segments(n);
  if (ns < 1 || n < 1 || S > INT_MAX || (int64_t)ns * S > (int64_t)INT_MAX)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_segment_min, dim3((uint32_t)((int64_t)ns * S)), dim3(kThreads), 0, st,
                     items, n, (int32_t)S, part);
  if (dtype == SDTW_F32)
    hipLaunchKernelGGL(k_best_two<true>, dim3(ns), dim3(kThreads), 0, st, items, n, (int32_t)S,
                       window, part, best_cost, best_end, second_cost, second_end);
  else
    hipLaunchKernelGGL(k_best_two<false>, dim3(ns), dim3(kThreads), 0, st, items, n,
                       (int32_t)S, window, part, best_cost, best_end, second_cost, second_end);
  return hipGetLastError();
}

}  // namespace sdtw
