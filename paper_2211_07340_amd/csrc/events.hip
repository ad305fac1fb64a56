// Event detection on the device: raw samples of each read -> the event values
// the alignment uses as its query (section 4.1 segments raw samples into
// events before normalisation; section 5.2 takes its R9.4 parameters from the
// two-window t-test detector of f5c and nanopolish).
//
// The detector, as this library reads it:
//  1. t statistic at each boundary position i (between samples i-1 and i),
//     window length w: means m1, m2 and population variances v1, v2 of the w
//     samples before and the w samples from i;
//         t_w(i) = |m2 - m1| / max(sqrt((v1 + v2) / w), 1e-30),
//     0 outside w <= i <= L - w.  float64, sums in index order.
//  2. Short (w = 3, threshold 1.4) and long (w = 6, threshold 9.0) peak
//     detectors with peak height 0.2 scan the positions in order (short
//     first).  Without a candidate a detector follows the running minimum of
//     t and opens a candidate once t rises more than the peak height above
//     it; with one it moves the candidate to any higher t, the short
//     detector's candidate above its threshold masks the long detector up to
//     candidate + 6 (dropping its candidate), a candidate above threshold
//     becomes valid once t falls more than the peak height below it, and a
//     valid candidate is emitted as a boundary once the position is more
//     than w / 2 past it; the detector restarts from the current t.
//  3. Events are the segments between consecutive distinct boundaries (0 and
//     L the outer ends); an event's value is the float32 rounding of the
//     float64 mean of its samples, summed in index order.
//  4. The first `trim` events (adaptor) are dropped, the next `keep` kept.
//
// One wave per one, two or four reads (as many as keep two waves per SIMD
// and fit their boundary lists in LDS).  Positions are taken in blocks (512 per wave): all lanes
// compute both t statistics of the block for each read into LDS, then lane
// r runs the two detectors of read r over it (a sequential state machine;
// the reads' machines run side by side) and inserts each emitted boundary
// into a sorted list that keeps only the trim + keep smallest.
// Boundaries can be emitted out of order (a candidate stays open while the
// other detector emits), so the list is final below the smallest open
// candidate; the read stops as soon as its first trim + keep boundaries are
// final, which is the first few thousand samples of a read in Read Until.
// Then every lane sums one event at a time.
#include <float.h>
#include <math.h>

#include "common.h"

namespace sdtw {
namespace {

constexpr int kEvBlock = 512;  // positions per block
constexpr int kWShort = 3, kWLong = 6;
constexpr double kTShort = 1.4, kTLong = 9.0, kPeakHeight = 0.2, kDenFloor = 1e-30;

template <int W>
__device__ __forceinline__ double tstat(const float* __restrict__ x, int64_t L, int64_t i) {
  if (i < W || i > L - W) return 0.0;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    s1 += (double)x[i - W + k];
    s2 += (double)x[i + k];
  }
  const double m1 = s1 / (double)W, m2 = s2 / (double)W;
  double q1 = 0.0, q2 = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const double d1 = (double)x[i - W + k] - m1;
    const double d2 = (double)x[i + k] - m2;
    q1 += d1 * d1;
    q2 += d2 * d2;
  }
  const double v1 = q1 / (double)W, v2 = q2 / (double)W;
  const double den = fmax(sqrt((v1 + v2) / (double)W), kDenFloor);
  return fabs(m2 - m1) / den;
}

struct Detector {
  int64_t masked_to, peak_pos;
  double peak_val;
  bool valid;
};

// Insert b into the sorted distinct list bs[0..n) that keeps at most cap
// entries (the smallest).
__device__ __forceinline__ void insert_bound(int64_t* bs, int32_t& n, int32_t cap, int64_t b) {
  if (n == cap && b >= bs[n - 1]) return;
  int32_t k = n;
  while (k > 0 && bs[k - 1] > b) --k;
  if (k > 0 && bs[k - 1] == b) return;
  const int32_t last = n < cap ? n : cap - 1;  // the largest falls off when full
  for (int32_t j = last; j > k; --j) bs[j] = bs[j - 1];
  bs[k] = b;
  if (n < cap) ++n;
}

// Insert b into the sorted distinct list bs[0..n) of at most cap entries;
// a full list sets *overflow instead (nothing may be dropped).
__device__ __forceinline__ void insert_pending(int64_t* bs, int32_t& n, int32_t cap, int64_t b,
                                               int32_t* overflow) {
  int32_t k = n;
  while (k > 0 && bs[k - 1] > b) --k;
  if (k > 0 && bs[k - 1] == b) return;
  if (n == cap) {
    *overflow = 1;
    return;
  }
  for (int32_t j = n; j > k; --j) bs[j] = bs[j - 1];
  bs[k] = b;
  ++n;
}

// One detector step at position i with statistic v (lane 0 only).  Emitted
// boundaries go to the truncating list, or with `overflow` to the pending
// list.
__device__ __forceinline__ void step(Detector& d, Detector* other, int w, double threshold,
                                     int64_t i, double v, int64_t* bs, int32_t& nb,
                                     int32_t cap, int32_t* overflow = nullptr) {
  if (d.masked_to >= i) return;
  if (d.peak_pos < 0) {
    if (v < d.peak_val) {
      d.peak_val = v;
    } else if (v - d.peak_val > kPeakHeight) {
      d.peak_val = v;
      d.peak_pos = i;
    }
    return;
  }
  if (v > d.peak_val) {
    d.peak_val = v;
    d.peak_pos = i;
  }
  if (other && d.peak_val > threshold) {  // the short detector masks the long one
    other->masked_to = d.peak_pos + kWLong;
    other->peak_pos = -1;
    other->peak_val = INFINITY;
    other->valid = false;
  }
  if (d.peak_val - v > kPeakHeight && d.peak_val > threshold) d.valid = true;
  if (d.valid && i - d.peak_pos > w / 2) {
    if (overflow)
      insert_pending(bs, nb, cap, d.peak_pos, overflow);
    else
      insert_bound(bs, nb, cap, d.peak_pos);
    d.peak_pos = -1;
    d.peak_val = v;
    d.valid = false;
  }
}

// R reads per wave: the t statistics of a block are computed by all lanes for
// all R reads, then lane r runs the detectors of read r (R state machines
// side by side instead of one lane at a time), then all lanes write the
// events of each read in turn.
//
// Read r is raw[offs[stride r] .. offs[stride r + 1]) (stride 1: CSR offsets;
// stride 2: start/end pairs).  Its events trim_r .. trim_r + keep - 1 are
// wanted, trim_r = trims[r] (or `trim` without trims; trim_r <= trim).  With
// `prefix` the samples are only the beginning of a longer read: the scan
// stops where the t statistics still depend on samples not yet received
// (position L - 5), and only events whose end boundary is final are written.
template <int R>
__global__ __launch_bounds__(64) void k_detect_events(const float* __restrict__ raw,
                                                      const int64_t* __restrict__ offs,
                                                      int32_t stride,
                                                      const int32_t* __restrict__ trims,
                                                      int32_t nreads, int32_t trim, int32_t keep,
                                                      int32_t prefix, float* __restrict__ out,
                                                      int32_t* __restrict__ counts) {
  constexpr int B = kEvBlock / R;  // positions per block and read
  extern __shared__ double ev_lds[];
  double* ts = ev_lds;                              // [R][B]
  double* tl = ev_lds + R * B;                      // [R][B]
  int64_t* bs_all = (int64_t*)(ev_lds + 2 * R * B);  // [R][trim + keep]
  __shared__ int32_t s_nb[R], s_closed[R], s_active;

  const int lane = threadIdx.x;
  const int32_t r0 = (int32_t)blockIdx.x * R;
  const int32_t list = trim + keep;  // LDS words per read's list
  int64_t Lr[R];
  const float* xr[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const bool ok = r0 + k < nreads;
    const int64_t a = ok ? offs[(int64_t)stride * (r0 + k)] : 0;
    Lr[k] = ok ? offs[(int64_t)stride * (r0 + k) + 1] - a : 0;
    xr[k] = raw + a;
  }
  // this lane's read (lanes >= R run no detector)
  const int me = lane < R ? lane : 0;
  int64_t* bs = bs_all + (int64_t)me * list;
  int64_t myL = 0;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (k == me) myL = Lr[k];
  // a first event outside [0, trim] marks the read as bad (count -1)
  const int32_t first = trims && r0 + me < nreads ? trims[r0 + me] : trim;
  const bool bad = first < 0 || first > trim;
  const int32_t cap = (bad ? 0 : first) + keep;
  // positions whose t statistics are final (all of them for a whole read)
  const int64_t scanL = prefix ? (myL > kWLong - 1 ? myL - (kWLong - 1) : 0) : myL;
  Detector ds{-1, -1, INFINITY, false}, dl{-1, -1, INFINITY, false};
  int32_t nb = 0;
  bool active = lane < R && scanL > 0 && !bad;
  if (lane < R) {
    s_nb[lane] = 0;
    s_closed[lane] = prefix ? 0 : (myL > 0 ? 1 : 0);  // no samples, no event
  }
  for (int64_t b0 = 0;; b0 += B) {
    if (lane == 0) s_active = 0;
    __syncthreads();
    if (active) atomicOr(&s_active, 1 << lane);
    __syncthreads();
    const int32_t act = s_active;
    if (!act) break;
    for (int idx = lane; idx < R * B; idx += 64) {
      const int k = idx / B, j = idx % B;
      if (!((act >> k) & 1)) continue;
      int64_t L = 0;
      const float* x = raw;
#pragma unroll
      for (int kk = 0; kk < R; ++kk)
        if (kk == k) {
          L = Lr[kk];
          x = xr[kk];
        }
      if (b0 + j < L) {
        ts[idx] = tstat<kWShort>(x, L, b0 + j);
        tl[idx] = tstat<kWLong>(x, L, b0 + j);
      }
    }
    __syncthreads();
    if (active) {
      const int64_t nblk = scanL - b0 < B ? scanL - b0 : B;
      const double* mts = ts + me * B;
      const double* mtl = tl + me * B;
      for (int64_t j = 0; j < nblk; ++j) {
        step(ds, &dl, kWShort, kTShort, b0 + j, mts[j], bs, nb, cap);
        step(dl, nullptr, kWLong, kTLong, b0 + j, mtl[j], bs, nb, cap);
      }
      // below the smallest open candidate no boundary can still appear
      int64_t cut = b0 + nblk;
      if (ds.peak_pos >= 0 && ds.peak_pos < cut) cut = ds.peak_pos;
      if (dl.peak_pos >= 0 && dl.peak_pos < cut) cut = dl.peak_pos;
      s_nb[me] = nb;
      if (nb == cap && bs[cap - 1] < cut) {
        s_closed[me] = cap;  // stopped early: events 0 .. cap-1 are closed
        active = false;
      } else if (b0 + nblk >= scanL) {
        active = false;  // scanned to the end
        if (prefix) {    // events whose end boundary is final
          int32_t nf = 0;
          while (nf < nb && bs[nf] < cut) ++nf;
          s_closed[me] = nf;
        } else {         // the last event ends at L
          s_closed[me] = nb + 1;
        }
      }
    }
    __syncthreads();
  }
  // events of each read: cut_0 = 0, cut_j = bs[j-1], and L after the last
  for (int k = 0; k < R; ++k) {
    const int32_t r = r0 + k;
    if (r >= nreads) break;
    const int64_t* kb = bs_all + (int64_t)k * list;
    const int32_t knb = s_nb[k];
    const int64_t L = Lr[k];
    const float* __restrict__ x = xr[k];
    const int32_t tr0 = trims ? trims[r] : trim;
    const bool kbad = tr0 < 0 || tr0 > trim;
    const int32_t tr = kbad ? 0 : tr0;
    const int32_t closed = kbad ? 0 : s_closed[k];
    const int32_t hi = closed < tr + keep ? closed : tr + keep;
    const int32_t n_out = hi > tr ? hi - tr : 0;
    for (int32_t e = lane; e < keep; e += 64) {
      float v = 0.0f;
      if (e < n_out) {
        const int32_t j = tr + e;
        const int64_t lo = j == 0 ? 0 : kb[j - 1];
        const int64_t up = j < knb ? kb[j] : L;
        double sum = 0.0;
        for (int64_t q = lo; q < up; ++q) sum += (double)x[q];
        v = (float)(sum / (double)(up - lo));
      }
      out[(int64_t)r * keep + e] = v;
    }
    if (lane == 0) counts[r] = kbad ? -1 : n_out;
  }
}

// ---- reads received chunk by chunk: the detectors' state kept between calls

constexpr int kPending = 32;  // emitted boundaries not yet delivered, per read

struct EventState {
  int64_t pos;           // next position to scan (from the read's first sample)
  int64_t last;          // start of the next undelivered event
  int64_t s_masked, s_peak, l_masked, l_peak;
  double s_val, l_val;
  int32_t s_valid, l_valid;
  int32_t index;         // index of the next undelivered event in the read
  int32_t npend;
  int64_t pend[kPending];
};

__global__ void k_event_state_init(EventState* __restrict__ states,
                                   const int32_t* __restrict__ slots, int32_t n) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  EventState& e = states[slots[i]];
  e.pos = 0;
  e.last = 0;
  e.s_masked = e.l_masked = -1;
  e.s_peak = e.l_peak = -1;
  e.s_val = e.l_val = INFINITY;
  e.s_valid = e.l_valid = 0;
  e.index = 0;
  e.npend = 0;
}

// One wave per read.  Read r's samples so far are raw[ranges[2r] ..
// ranges[2r+1]) (the start fixed across calls); its state is
// states[slots[r]].  Positions pos .. L-6 are scanned (those whose t
// statistics are final) and emitted boundaries join the pending list (in
// LDS, room for keep + 32); then the final ones (below every open
// candidate) are delivered in order as events last .. boundary, events
// below `trim` consumed without being written, at most keep written; at most
// 32 undelivered boundaries may carry over to the next call.
__global__ __launch_bounds__(64) void k_events_continue(
    const float* __restrict__ raw, const int64_t* __restrict__ ranges,
    const int32_t* __restrict__ slots, EventState* __restrict__ states, int32_t nreads,
    int32_t trim, int32_t keep, float* __restrict__ out, int32_t* __restrict__ counts) {
  __shared__ double ts[kEvBlock], tl[kEvBlock];
  extern __shared__ int64_t pend[];  // [keep + kPending]
  __shared__ int32_t s_nout, s_skip, s_over;
  __shared__ int64_t s_start;
  const int32_t r = (int32_t)blockIdx.x;
  if (r >= nreads) return;
  const int lane = threadIdx.x;
  const int32_t room = keep + kPending;
  const int64_t a = ranges[2 * (int64_t)r];
  const int64_t L = ranges[2 * (int64_t)r + 1] - a;
  const float* __restrict__ x = raw + a;
  EventState* __restrict__ st = states + slots[r];
  const int64_t scanL = L > kWLong - 1 ? L - (kWLong - 1) : 0;
  const int64_t pos0 = st->pos;
  int32_t np = st->npend;
  if (lane < kPending) pend[lane] = st->pend[lane];
  Detector ds{st->s_masked, st->s_peak, st->s_val, st->s_valid != 0};
  Detector dl{st->l_masked, st->l_peak, st->l_val, st->l_valid != 0};
  int32_t over = 0;
  __syncthreads();
  for (int64_t b0 = pos0; b0 < scanL; b0 += kEvBlock) {
    const int64_t nblk = scanL - b0 < kEvBlock ? scanL - b0 : kEvBlock;
    for (int64_t j = lane; j < nblk; j += 64) {
      ts[j] = tstat<kWShort>(x, L, b0 + j);
      tl[j] = tstat<kWLong>(x, L, b0 + j);
    }
    __syncthreads();
    if (lane == 0) {
      for (int64_t j = 0; j < nblk; ++j) {
        step(ds, &dl, kWShort, kTShort, b0 + j, ts[j], pend, np, room, &over);
        step(dl, nullptr, kWLong, kTLong, b0 + j, tl[j], pend, np, room, &over);
      }
    }
    __syncthreads();
  }
  int32_t used = 0;
  if (lane == 0) {
    const int64_t scanned = scanL > pos0 ? scanL : pos0;
    // below the smallest open candidate no boundary can still appear
    int64_t cut = scanned;
    if (ds.peak_pos >= 0 && ds.peak_pos < cut) cut = ds.peak_pos;
    if (dl.peak_pos >= 0 && dl.peak_pos < cut) cut = dl.peak_pos;
    int64_t start = st->last;
    int32_t index = st->index, nout = 0, skip = 0;
    while (used < np && pend[used] < cut && nout < keep) {
      if (index >= trim) {
        ++nout;
      } else {
        start = pend[used];
        ++skip;
      }
      ++index;
      ++used;
    }
    st->pos = scanned;
    st->last = used > 0 ? pend[used - 1] : st->last;
    st->index = index;
    st->s_masked = ds.masked_to;
    st->s_peak = ds.peak_pos;
    st->s_val = ds.peak_val;
    st->s_valid = ds.valid;
    st->l_masked = dl.masked_to;
    st->l_peak = dl.peak_pos;
    st->l_val = dl.peak_val;
    st->l_valid = dl.valid;
    if (np - used > kPending) over = 1;
    s_nout = nout;
    s_skip = skip;
    s_start = start;
    s_over = over;
  }
  __syncthreads();
  // the delivered events: start .. pend[skip], pend[skip] .. pend[skip+1], ...
  const int32_t nout = s_nout, skip = s_skip;
  const int64_t start = s_start;
  for (int32_t e = lane; e < keep; e += 64) {
    float v = 0.0f;
    if (e < nout) {
      const int64_t lo = e == 0 ? start : pend[skip + e - 1];
      const int64_t up = pend[skip + e];
      double sum = 0.0;
      for (int64_t q = lo; q < up; ++q) sum += (double)x[q];
      v = (float)(sum / (double)(up - lo));
    }
    out[(int64_t)r * keep + e] = v;
  }
  __syncthreads();
  if (lane == 0) {
    const int32_t left = np - used < kPending ? np - used : kPending;
    for (int32_t j = 0; j < left; ++j) st->pend[j] = pend[used + j];
    st->npend = left;
    counts[r] = s_over ? -1 : nout;
  }
}

}  // namespace

size_t event_state_bytes() { return sizeof(EventState); }

hipError_t launch_event_state_init(void* states, const int32_t* slots, int32_t n,
                                   hipStream_t st) {
  hipLaunchKernelGGL(k_event_state_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (EventState*)states, slots, n);
  return hipGetLastError();
}

hipError_t launch_events_continue(const float* raw, const int64_t* ranges, const int32_t* slots,
                                  void* states, int32_t nreads, int32_t trim, int32_t keep,
                                  float* out, int32_t* counts, hipStream_t st) {
  const size_t lds = sizeof(int64_t) * (size_t)(keep + kPending);
  hipLaunchKernelGGL(k_events_continue, dim3((unsigned)nreads), dim3(64), lds, st, raw, ranges,
                     slots, (EventState*)states, nreads, trim, keep, out, counts);
  return hipGetLastError();
}

// Reads per wave: more reads share a wave (their detectors run side by side)
// only while the launch still has two waves per SIMD; measured on MI355X for
// 4,096 reads: 1.21 ms with one read per wave, 0.79 with two, 0.85 with four,
// 1.03 with eight.  The boundary lists of the wave's reads must fit in
// 48 KB of LDS.
static size_t lds_for(int rpw, int32_t trim, int32_t keep) {
  return sizeof(double) * 2 * kEvBlock + (size_t)rpw * sizeof(int64_t) * (size_t)(trim + keep);
}

static int reads_per_wave(int32_t nreads, int32_t trim, int32_t keep) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int64_t waves_wanted = 2 * 4 * (int64_t)cus;  // two per SIMD
  int rpw = 1;
  for (int r : {2, 4})
    if ((int64_t)nreads / r >= waves_wanted && lds_for(r, trim, keep) <= 48 * 1024) rpw = r;
  return rpw;
}

hipError_t launch_detect_events(const float* raw, const int64_t* offs, int32_t stride,
                                const int32_t* trims, int32_t nreads, int32_t trim,
                                int32_t keep, int32_t prefix, float* out, int32_t* counts,
                                hipStream_t st) {
  const int rpw = reads_per_wave(nreads, trim, keep);
  const size_t lds = lds_for(rpw, trim, keep);
  const dim3 grid((unsigned)((nreads + rpw - 1) / rpw));
  if (rpw == 4)
    hipLaunchKernelGGL(k_detect_events<4>, grid, dim3(64), lds, st, raw, offs, stride, trims,
                       nreads, trim, keep, prefix, out, counts);
  else if (rpw == 2)
    hipLaunchKernelGGL(k_detect_events<2>, grid, dim3(64), lds, st, raw, offs, stride, trims,
                       nreads, trim, keep, prefix, out, counts);
  else
    hipLaunchKernelGGL(k_detect_events<1>, grid, dim3(64), lds, st, raw, offs, stride, trims,
                       nreads, trim, keep, prefix, out, counts);
  return hipGetLastError();
}

}  // namespace sdtw
