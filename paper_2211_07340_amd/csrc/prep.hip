// Reference and query preparation (section 4.1; section 2.2 k-mer model).
//
// Reference: k-mer model lookup of both strands (one thread per output
// sample), then a joint z-score over the concatenation whose mean and
// population sd are accumulated in double in index order by one lane (the
// same sequence of IEEE double operations as a plain sequential loop; it is
// a one-time step), then fixed-point codes.
//
// Queries: one wave per read; lane 0 walks the read's events in index order
// for the mean and for the sum of squared deviations, so each read's
// statistics come from exactly the same sequence of IEEE double operations as
// a plain sequential loop (no contraction: the library is built with
// -ffp-contract=off).
#include <math.h>

#include "common.h"

namespace sdtw {
namespace {

constexpr int kPrepThreads = 256;

__device__ __forceinline__ int16_t to_code(float z, double scale, unsigned long long* nsat_local) {
  double r = rint((double)z * scale);  // round half to even
  if (r > 32767.0) { r = 32767.0; ++*nsat_local; }
  if (r < -32768.0) { r = -32768.0; ++*nsat_local; }
  return (int16_t)r;
}

// Expected current of k-mer p of the forward strand (p < nk) or of k-mer
// p - nk of the reverse-complement strand read 5'->3'.
__global__ void k_kmer(const uint8_t* __restrict__ g, int64_t L, int k,
                       const float* __restrict__ table, float* __restrict__ sig) {
  const int64_t nk = L - k + 1;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 2 * nk) return;
  uint32_t idx = 0;
  if (p < nk) {
    for (int m = 0; m < k; ++m) idx = idx * 4u + (g[p + m] & 3u);
  } else {
    const int64_t q = p - nk;  // position in revcomp(g)
    for (int m = 0; m < k; ++m) idx = idx * 4u + (3u - (g[L - 1 - (q + m)] & 3u));
  }
  sig[p] = table[idx];
}

// x and z may be the same array (normalised in place): each thread reads its
// element before writing it, so neither pointer is declared restrict.
__global__ void k_normalize(const float* x, int64_t n, const double* __restrict__ stats,
                            double scale, float* z, int16_t* __restrict__ codes,
                            int64_t* __restrict__ nsat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long sat = 0;
  if (i < n) {
    const double mean = stats[0], sd = stats[1];
    const float zi = sd > 0.0 ? (float)(((double)x[i] - mean) / sd) : 0.0f;
    z[i] = zi;
    if (codes) codes[i] = to_code(zi, scale, &sat);
  }
  if (nsat && sat) atomicAdd((unsigned long long*)nsat, sat);
}

__global__ void k_zero_i64(int64_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// One wave per read.  Events are staged through LDS in coalesced chunks and
// lane 0 accumulates the sum and then the sum of squared deviations in index
// order, so the statistics come from the same sequence of double operations
// as a plain sequential loop; all lanes then normalise and quantise.  The
// next chunk's loads are issued before lane 0 sums the current one (two LDS
// buffers), so memory latency hides behind the sequential sum.
constexpr int kQChunk = 512;
constexpr int kQPer = kQChunk / 64;

__device__ __forceinline__ double wave_seq_sum(const float* __restrict__ raw, int64_t a, int64_t b,
                                               double mean, bool squares, float* buf) {
  const int lane = (int)threadIdx.x;
  double acc = 0.0;
  float pre[kQPer];
  auto fetch = [&](int64_t base) {
#pragma unroll
    for (int j = 0; j < kQPer; ++j) {
      const int64_t i = base + lane + 64 * j;
      pre[j] = i < b ? raw[i] : 0.0f;
    }
  };
  fetch(a);
  int cur = 0;
  for (int64_t base = a; base < b; base += kQChunk) {
    const int n = (int)min<int64_t>(kQChunk, b - base);
    float* const cb = buf + cur * kQChunk;
#pragma unroll
    for (int j = 0; j < kQPer; ++j) cb[lane + 64 * j] = pre[j];
    // one barrier per chunk: the other buffer, written next, was last read
    // by lane 0 before it reached this barrier
    __syncthreads();
    if (base + kQChunk < b) fetch(base + kQChunk);
    if (lane == 0) {
      for (int k = 0; k < n; ++k) {
        const double v = (double)cb[k];
        if (squares) {
          const double d = v - mean;
          acc += d * d;
        } else {
          acc += v;
        }
      }
    }
    cur ^= 1;
  }
  __syncthreads();  // lane 0 is done with both buffers before they are reused
  return __shfl(acc, 0);
}

// One wave: stats[0] = mean and stats[1] = population sd of x[0..n), each
// sum accumulated by lane 0 in index order; nsat (optional) cleared.
__global__ __launch_bounds__(64) void k_seq_stats(const float* __restrict__ x, int64_t n,
                                                  double* __restrict__ stats,
                                                  int64_t* __restrict__ nsat) {
  __shared__ float buf[2 * kQChunk];
  const double mean = wave_seq_sum(x, 0, n, 0.0, false, buf) / (double)n;
  const double sd = sqrt(wave_seq_sum(x, 0, n, mean, true, buf) / (double)n);
  if (threadIdx.x == 0) {
    stats[0] = mean;
    stats[1] = sd;
    if (nsat) *nsat = 0;
  }
}

// stats_in (optional): per-read (mean, sd) to apply instead of the read's
// own statistics; stats_out (optional): the (mean, sd) applied.
__global__ __launch_bounds__(64) void k_prep_queries(const float* __restrict__ raw,
                                                     const int64_t* __restrict__ offs, int32_t nq,
                                                     double scale,
                                                     const double* __restrict__ stats_in,
                                                     double* __restrict__ stats_out,
                                                     float* __restrict__ z,
                                                     int16_t* __restrict__ codes,
                                                     int64_t* __restrict__ nsat) {
  __shared__ float buf[2 * kQChunk];
  const int32_t r = (int32_t)blockIdx.x;
  if (r >= nq) return;
  const int64_t a = offs[r], b = offs[r + 1];
  if (b <= a) return;
  double mean, sd;
  if (stats_in) {
    mean = stats_in[2 * r];
    sd = stats_in[2 * r + 1];
  } else {
    const double n = (double)(b - a);
    mean = wave_seq_sum(raw, a, b, 0.0, false, buf) / n;
    sd = sqrt(wave_seq_sum(raw, a, b, mean, true, buf) / n);
  }
  if (stats_out && threadIdx.x == 0) {
    stats_out[2 * r] = mean;
    stats_out[2 * r + 1] = sd;
  }
  unsigned long long sat = 0;
  for (int64_t i = a + threadIdx.x; i < b; i += 64) {
    const float zi = sd > 0.0 ? (float)(((double)raw[i] - mean) / sd) : 0.0f;
    z[i] = zi;
    if (codes) codes[i] = to_code(zi, scale, &sat);
  }
  if (nsat && sat) atomicAdd((unsigned long long*)nsat, sat);
}

// Device layout of a reference: int16 -> u32 with +32768 bias, float -> bits;
// zero padding up to n_pad.  Non-finite float values are counted.
__global__ void k_layout(const void* __restrict__ src, int64_t n, int dtype,
                         uint32_t* __restrict__ dst, int64_t n_pad, int32_t* __restrict__ nonfinite) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  uint32_t v = 0;
  if (i < n) {
    if (dtype == SDTW_I16) {
      v = (uint32_t)((int32_t)((const int16_t*)src)[i] + (int32_t)kI16Bias);
    } else {
      const float f = ((const float*)src)[i];
      if (!isfinite(f)) atomicAdd(nonfinite, 1);
      v = __float_as_uint(f);
    }
  }
  dst[i] = v;
}

inline unsigned grid_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

hipError_t launch_prepare_reference(const uint8_t* g, int64_t L, const float* table, int k,
                                    double scale, float* z, int16_t* codes, int64_t* nsat,
                                    double* scratch, hipStream_t st) {
  const int64_t n = 2 * (L - k + 1);
  // the raw signal is produced in z and normalised in place
  hipLaunchKernelGGL(k_kmer, dim3(grid_for(n, kPrepThreads)), dim3(kPrepThreads), 0, st,
                     g, L, k, table, z);
  double* stats = scratch;
  hipLaunchKernelGGL(k_seq_stats, dim3(1), dim3(64), 0, st, z, n, stats, nsat);
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(n, kPrepThreads)), dim3(kPrepThreads), 0, st,
                     z, n, stats, scale, z, codes, nsat);
  return hipGetLastError();
}

hipError_t launch_prepare_queries(const float* raw, const int64_t* offs, int32_t nq,
                                  double scale, const double* stats_in, double* stats_out,
                                  float* z, int16_t* codes, int64_t* nsat, hipStream_t st) {
  if (nsat) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, nsat);
  hipLaunchKernelGGL(k_prep_queries, dim3(nq), dim3(64), 0, st, raw, offs, nq, scale, stats_in,
                     stats_out, z, codes, nsat);
  return hipGetLastError();
}

hipError_t launch_layout_reference(const void* src, int64_t n, int dtype, uint32_t* dst,
                                   int64_t n_pad, int32_t* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_layout, dim3(grid_for(n_pad, kPrepThreads)), dim3(kPrepThreads), 0, st,
                     src, n, dtype, dst, n_pad, nonfinite);
  return hipGetLastError();
}

}  // namespace sdtw
