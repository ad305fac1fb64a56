// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sdtw.h"

namespace sdtw {

// Status plumbing: every C entry point reports through set_error().
int set_error(int status, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);

// Width of the widest column strip a kernel uses (64 lanes x 32 columns); the
// device copy of a reference is padded to a multiple of it plus one strip.
constexpr int kLanes = 64;
constexpr int kMaxStrip = 32;
constexpr int64_t kPadUnit = int64_t(kLanes) * kMaxStrip;

// Offset that maps int16 onto [0, 65535]; |x - y| is translation invariant.
constexpr uint32_t kI16Bias = 32768u;

// Shortest read (or row band) the continuous-skew kernel takes with K chains
// per lane: its one-step-ahead LDS prefetch needs the last sub-lane's boundary
// write two steps before lane 0's read, i.e. M >= 64K + 1.
inline int32_t skew_min_m(int chains) { return 64 * chains + 1; }

// Strip widths and chains-per-lane the skew kernel is built for: W in
// {8, 16, 32}, K in {1, 2, 4}, W / K a multiple of 4.
inline bool valid_strip_chains(int strip, int chains) {
  if (strip != 8 && strip != 16 && strip != 32) return false;
  if (chains != 1 && chains != 2 && chains != 4) return false;
  return (strip / chains) % 4 == 0;
}

// Row bands per workgroup (waves per read): 1 for every (strip, chains)
// above; 2 or 4 with strip 16 and 1 or 2 chains; 2, 3 or 4 with strip 16 or
// 32 and 1 chain; 2 with strip 32 and 2 chains.
inline bool valid_skew_config(int strip, int chains, int bands) {
  if (!valid_strip_chains(strip, chains)) return false;
  if (bands == 1) return true;
  if (bands == 3) return chains == 1 && (strip == 16 || strip == 32);
  if (bands != 2 && bands != 4) return false;
  return (strip == 16 && chains <= 2) || (strip == 32 && chains == 1) ||
         (strip == 32 && chains == 2 && bands == 2);
}

// Bands a read of M rows is cut into: as many as allowed (at most `bands`,
// each >= 64K + 1 rows) or, with a target > 0, about M / target of them
// (rounded to nearest, at least 1), so that reads of different lengths get
// bands of about the same height and finish together.
__host__ __device__ inline int32_t skew_read_bands(int32_t m, int chains, int bands,
                                                   int32_t target = 0) {
  int32_t pe = m / (64 * chains + 1);
  pe = pe < 1 ? 1 : (pe > bands ? bands : pe);
  if (target > 0) {
    int32_t t = (m + target / 2) / target;
    t = t < 1 ? 1 : t;
    pe = t < pe ? t : pe;
  }
  return pe;
}
// Rows of the tallest band of a read of M rows.
inline int32_t skew_band_rows(int32_t m, int chains, int bands, int32_t target = 0) {
  const int32_t pe = skew_read_bands(m, chains, bands, target);
  return (m + pe - 1) / pe;
}

// LDS words of the skew kernel: a shared part (zeros and a +inf cell; the
// band-to-band rings) and, per band, the finished-row stage and the
// query/boundary entries of up to band_rows rows.  Extending resident rows
// (stream), the shared part also holds the first band's copy of the
// resident row's next tile and the value left of it, and one finished-row
// stage serves every band (only a read's last band uses it), so that two
// workgroups of four bands fit on a CU.
__host__ __device__ constexpr int skew_entry_words(int chains, int band_rows) {
  return (2 * (band_rows + 64 * chains) + 3) & ~3;
}
__host__ __device__ constexpr int skew_band_words(int strip, int chains, int band_rows) {
  return (64 * strip + 2 * (band_rows + 64 * chains) + 3) & ~3;
}
inline size_t skew_lds_bytes(int strip, int chains, int bands, int band_rows,
                             bool stream = false) {
  const size_t tile = 64 * (size_t)strip;
  const size_t shared = (size_t)strip + 4 + (size_t)(bands - 1) * (2 * tile + 4);
  if (stream)
    return 4 * (shared + 2 * tile + 4 + (size_t)bands * skew_entry_words(chains, band_rows));
  return 4 * (shared + (size_t)bands * (size_t)skew_band_words(strip, chains, band_rows));
}

inline int64_t padded_length(int64_t n) {
  return ((n + kPadUnit - 1) / kPadUnit) * kPadUnit + kPadUnit;
}

// ---- launchers (prep.hip) ---------------------------------------------------
hipError_t launch_prepare_reference(const uint8_t* g, int64_t L, const float* table,
                                    int k, double scale, float* z, int16_t* codes,
                                    int64_t* nsat, double* scratch, hipStream_t st);
constexpr int kRefPartials = 2;  // doubles of scratch: the reference's mean and sd
hipError_t launch_prepare_queries(const float* raw, const int64_t* offs, int32_t nq,
                                  double scale, const double* stats_in, double* stats_out,
                                  float* z, int16_t* codes, int64_t* nsat, hipStream_t st);
hipError_t launch_layout_reference(const void* src, int64_t n, int dtype,
                                   uint32_t* dst, int64_t n_pad, int32_t* nonfinite,
                                   hipStream_t st);

// ---- launchers (align.hip) --------------------------------------------------
// One streaming work item: extend a resident row by the rows of one chunk.
struct StreamItem {
  uint32_t* acc;   // resident row gamma(m_old, 0..N) in the kernel's cost encoding
  int64_t q0;      // first chunk value in the query array
  int32_t m;       // chunk rows (>= 1)
  int32_t m_old;   // rows already folded into acc (0: acc is not read)
  int32_t out;     // output slot for (cost, end)
  int32_t pad;
};

struct AlignArgs {
  const uint32_t* ref;   // padded device layout (u32 biased int16, or f32 bits)
  int64_t n;             // true reference length
  const void* q;         // query values (int16 or float)
  const int64_t* offs;   // CSR offsets [nq+1]
  const int32_t* order;  // work list: read indices
  int32_t nwork;         // entries in the work list
  int32_t max_m;         // longest read in the work list (LDS sizing)
  int32_t max_band;      // skew kernel: rows of the tallest band of any item (LDS sizing)
  int32_t band_target;   // skew kernel: target rows per band (0: as many bands as fit)
  int32_t lds_bytes;     // skew kernel: LDS to reserve per workgroup if more than it needs
                         // (caps the workgroups a compute unit takes, spreading a short
                         // work list over every compute unit)
  int32_t* counter;      // streaming launches: persistent work counter (reset by launcher)
  uint32_t* sched;       // batch launches: kSchedWords words of pull and placement state
                         // (device, reset by launcher)
  void* cost;            // int32[nq] or float[nq]
  int32_t* end;          // int32[nq]
  int32_t single_m;      // used when offs == nullptr: one read of this length
  const StreamItem* items;  // streaming launches: work item descriptors
};
// Pull and placement state of a batch launch of the continuous-skew kernel:
// a 64-bit pull word (items taken from the front of the work list in the low
// half, from the back in the high half), then per SIMD slot (XCC, shader
// engine, shader array, CU, SIMD: 3 + 3 + 1 + 4 + 2 bits of the hardware ids)
// the number of the launch's waves that run on it, then per slot the work
// left to the first two of them.
constexpr int kSchedHead = 4;  // words before the per-SIMD counts
constexpr int kSchedSimds = 1 << 13;
constexpr int kSchedWords = kSchedHead + 3 * kSchedSimds;
// Continuous-skew persistent kernel: `bands` waves per workgroup (one read per
// workgroup, cut into row bands), `chains` chains per lane; every read in the
// list must have M >= skew_min_m(chains) and a.max_band must bound
// skew_band_rows() of every read.  `stream`: work items come from a.items and
// extend resident rows.  `blocks` workgroups pull items until none is left.
hipError_t launch_align_skew(int dtype, int strip, int chains, int bands, int blocks,
                             const AlignArgs& a, hipStream_t st, bool stream = false);
// Synchronised-tile single-wave kernel; any M >= 1; one block per work item.
hipError_t launch_align_plain(int dtype, int strip, const AlignArgs& a, hipStream_t st,
                              bool stream = false);
size_t plain_lds_bytes(int dtype, int strip, int max_m);

// ---- launchers (scores.hip) -------------------------------------------------
// Best and runner-up ends of the resident rows items[i].acc (n columns), out
// to index items[i].out.  `part` holds ns * best_two_segments(n) keys of
// scratch (per-segment minima), written and read on `st`.
constexpr int64_t kBestTwoSegment = 16384;  // columns per workgroup of the first pass
int64_t best_two_segments(int64_t n);
hipError_t launch_best_two(int dtype, const StreamItem* items, int32_t ns, int64_t n,
                           int32_t window, uint64_t* part, void* best_cost, int32_t* best_end,
                           void* second_cost, int32_t* second_end, hipStream_t st);
int max_lds_bytes();

// ---- launchers (events.hip) -------------------------------------------------
// Event values of each read's raw samples (trim + keep <= kMaxEventList).
constexpr int32_t kMaxEventList = 6144;
// Read r: raw[offs[stride r] .. offs[stride r + 1]); events trims[r] (or trim)
// onward; prefix: the samples are the start of a longer read.
hipError_t launch_detect_events(const float* raw, const int64_t* offs, int32_t stride,
                                const int32_t* trims, int32_t nreads, int32_t trim,
                                int32_t keep, int32_t prefix, float* out, int32_t* counts,
                                hipStream_t st);

// Reads received chunk by chunk: per-read detector state (event_state_bytes()
// each) kept between calls.
size_t event_state_bytes();
hipError_t launch_event_state_init(void* states, const int32_t* slots, int32_t n,
                                   hipStream_t st);
hipError_t launch_events_continue(const float* raw, const int64_t* ranges, const int32_t* slots,
                                  void* states, int32_t nreads, int32_t trim, int32_t keep,
                                  float* out, int32_t* counts, hipStream_t st);

// ---- launchers (wide.hip) ---------------------------------------------------
// One int16 query over every compute unit: row scans with look-back between
// tiles of 256 * cols columns (cols in {8, 16, 32, 64}).  `scratch` holds
// wide_scratch_words(n, m, cols) 64-bit words, used only by this launch
// (cleared by it, in order on `st`).  `row` (n values, optional): the last
// row is written there; with `row_in` the rows extend it (it holds the row
// before the first of the m rows, at most 4,096 rows in all) instead of
// starting from the free-start zeros.
int64_t wide_tiles(int64_t n, int cols);
int64_t wide_scratch_words(int64_t n, int32_t m, int cols);
int wide_pick_cols(int64_t n, int device);  // columns per thread for sdtw_align_one_wide(cols=0)
// The fixed per-device scratch of sdtw_align_one_wide_noalloc: its size in
// 64-bit words, and its device address on `device` (the current device),
// looked up once per device.
int64_t wide_noalloc_words();
hipError_t wide_noalloc_scratch(int device, uint64_t** out);
hipError_t launch_align_wide(const uint32_t* ref, int64_t n, const int16_t* q, int32_t m,
                             int cols, uint64_t* scratch, int32_t* cost, int32_t* end,
                             hipStream_t st, uint32_t* row = nullptr, bool row_in = false);

}  // namespace sdtw
