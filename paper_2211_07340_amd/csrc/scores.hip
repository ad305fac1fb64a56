// Best and runner-up ends of resident last rows (section 5.2: a mapping
// quality is computed from the mapped positions and their scores before the
// selection decision).
//
// For a row gamma(m, 0..N): best = the first column with the minimum (the
// strict-less last-row scan of Algorithms 1 and 2, the same end as the
// extension that produced the row); second = the first column with the
// minimum among the columns farther than `window` from best.  Values are the
// kernels' cost encoding (uint32 sums on the int16 path, float32 bits of
// non-negative values on the float32 path), so one unsigned comparison
// orders both.
//
// One workgroup of 256 threads per row, two passes over the row (uint4
// loads, lexicographic (value, column) minimum per thread, then across the
// workgroup).  The row is HBM-bound: 8N bytes read per row.
#include <limits.h>

#include "common.h"

namespace sdtw {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void lex_min(uint32_t& v, int32_t& j, uint32_t ov, int32_t oj) {
  if (ov < v || (ov == v && oj < j)) {
    v = ov;
    j = oj;
  }
}

// (v, j) of every thread -> the workgroup's lexicographic minimum, in every thread
__device__ __forceinline__ void block_lex_min(uint32_t& v, int32_t& j, uint32_t* sv,
                                              int32_t* sj) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t ov = (uint32_t)__shfl_xor((int)v, off);
    const int32_t oj = __shfl_xor(j, off);
    lex_min(v, j, ov, oj);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[wave] = v;
    sj[wave] = j;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) lex_min(v, j, sv[w], sj[w]);
  __syncthreads();  // sv / sj may be reused by the next call
}

template <bool F32>
__global__ __launch_bounds__(kThreads) void k_best_two(const StreamItem* __restrict__ items,
                                                       int32_t ns, int64_t n, int32_t window,
                                                       void* best_cost, int32_t* best_end,
                                                       void* second_cost, int32_t* second_end) {
  __shared__ uint32_t sv[kThreads / 64];
  __shared__ int32_t sj[kThreads / 64];
  const int32_t s = (int32_t)blockIdx.x;
  if (s >= ns) return;
  const uint32_t* __restrict__ row = items[s].acc;
  const int32_t out = items[s].out;
  const int64_t nq = (n + 3) / 4;  // uint4 groups; the row is padded to a multiple of 2048

  uint32_t v = 0xFFFFFFFFu;
  int32_t j = INT_MAX;
  for (int64_t g = threadIdx.x; g < nq; g += kThreads) {
    const uint4 q = ((const uint4*)row)[g];
    const uint32_t e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * g + k < n) lex_min(v, j, e[k], (int32_t)(4 * g + k));
  }
  block_lex_min(v, j, sv, sj);
  const uint32_t vb = v;
  const int32_t jb = j;

  v = 0xFFFFFFFFu;
  j = INT_MAX;
  const int64_t lo = (int64_t)jb - window, hi = (int64_t)jb + window;
  for (int64_t g = threadIdx.x; g < nq; g += kThreads) {
    const uint4 q = ((const uint4*)row)[g];
    const uint32_t e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t c = 4 * g + k;
      if (c < n && (c < lo || c > hi)) lex_min(v, j, e[k], (int32_t)c);
    }
  }
  block_lex_min(v, j, sv, sj);

  if (threadIdx.x == 0) {
    const bool none = (j == INT_MAX);
    if constexpr (F32) {
      ((float*)best_cost)[out] = __uint_as_float(vb);
      ((float*)second_cost)[out] = none ? __uint_as_float(0x7F800000u) : __uint_as_float(v);
    } else {
      ((int32_t*)best_cost)[out] = (int32_t)vb;
      ((int32_t*)second_cost)[out] = none ? INT_MAX : (int32_t)v;
    }
    best_end[out] = jb;
    second_end[out] = none ? -1 : j;
  }
}

}  // namespace

hipError_t launch_best_two(int dtype, const StreamItem* items, int32_t ns, int64_t n,
                           int32_t window, void* best_cost, int32_t* best_end,
                           void* second_cost, int32_t* second_end, hipStream_t st) {
  if (dtype == SDTW_F32)
    hipLaunchKernelGGL(k_best_two<true>, dim3(ns), dim3(kThreads), 0, st, items, ns, n, window,
                       best_cost, best_end, second_cost, second_end);
  else
    hipLaunchKernelGGL(k_best_two<false>, dim3(ns), dim3(kThreads), 0, st, items, ns, n, window,
                       best_cost, best_end, second_cost, second_end);
  return hipGetLastError();
}

}  // namespace sdtw
