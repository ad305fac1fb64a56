// C ABI of the sDTW library: validation, object lifetimes, scheduling.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

struct sdtw_ref_s {
  int device;
  int dtype;
  int64_t n;       // true length
  int64_t n_pad;   // device layout length
  uint32_t* data;  // u32 biased int16 or float bits
  std::atomic<int> open_streams;
  std::atomic<int> stream_strip{0};  // sdtw_stream_set_config for this reference (0: automatic)
  std::atomic<int> stream_bands{0};
};

namespace sdtw {
// Completion of one sdtw_stream_extend call (one event per call, shared by
// the streams it extended); the event returns to a pool when released.
struct CallToken {
  hipEvent_t ev = nullptr;
  ~CallToken();
};
}  // namespace sdtw

struct sdtw_stream_s {
  int device;
  sdtw_ref ref;
  uint32_t* row;        // resident row gamma(rows, .), n_pad entries
  size_t bytes;
  int32_t rows;         // query rows folded in so far
  std::shared_ptr<sdtw::CallToken> last;  // last extend that used the row
};

struct sdtw_plan_s {
  int device;
  int dtype;
  int32_t nq;
  int32_t max_m;
  std::vector<int32_t> sorted_m;  // read lengths, longest first (order_dev's order)
  int64_t* offs_dev;              // [nq+1]
  int32_t* order_dev;             // [nq]: read indices, longest first
  uint32_t* sched_dev;            // [kSchedWords]: pull and placement state of a launch
  int strip;                      // columns per lane
  int chains;                     // most chains per lane (K) the long reads use
  int bands;                      // waves per read (row bands) of the skew kernel
  int32_t band_rows;              // target rows per band (0: as many bands as fit)
  int waves_per_cu;               // persistent grid density (bands x workgroups per CU)
  int cus;                        // compute units of the device
};

namespace sdtw {

static thread_local char g_err[512] = "";

int set_error(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return status;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return SDTW_OK;
  if (e == hipErrorOutOfMemory)
    return set_error(SDTW_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_error(SDTW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

static int current_device() {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess) return -1;
  return d;
}

// Kernels run on the current device; objects of another device would be
// reached through peer addresses, so every call that launches checks.
static int require_device(int dev, const char* who) {
  const int cur = current_device();
  if (cur != dev)
    return set_error(SDTW_EINVAL, "%s: objects live on device %d, current device is %d", who, dev,
                     cur);
  return SDTW_OK;
}

static int cu_count() {
  int dev = current_device(), v = 0;
  if (dev < 0 || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return v;
}

static bool valid_strip(int s) { return s == 8 || s == 16 || s == 32; }

}  // namespace sdtw

namespace sdtw {

// ---- events recycled across extend calls -----------------------------------
static std::mutex g_ev_mu;
static std::vector<hipEvent_t> g_ev_free;

static hipEvent_t event_get() {
  {
    std::lock_guard<std::mutex> g(g_ev_mu);
    if (!g_ev_free.empty()) {
      hipEvent_t e = g_ev_free.back();
      g_ev_free.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

CallToken::~CallToken() {
  if (!ev) return;
  std::lock_guard<std::mutex> g(g_ev_mu);
  g_ev_free.push_back(ev);
}

// ---- resident-row pool: a byte budget per device, rows cached by size ----
struct RowPool {
  std::mutex mu;
  int64_t budget = int64_t(16) << 30;
  int64_t in_use = 0;
  int64_t cached = 0;
  std::map<size_t, std::vector<void*>> free_rows;
};
constexpr int kMaxDevices = 64;
static RowPool g_pool[kMaxDevices];

static RowPool* pool_for(int dev) {
  return (dev >= 0 && dev < kMaxDevices) ? &g_pool[dev] : nullptr;
}

// ---- pinned descriptor slots for stream_extend -----------------------------
struct DescSlot {
  StreamItem* host = nullptr;
  StreamItem* dev = nullptr;  // cap items, then one int32 work counter
  int32_t cap = 0;
  uint64_t* part = nullptr;  // sdtw_stream_best_two: per-segment minima
  int64_t part_cap = 0;
  std::shared_ptr<CallToken> last;
};
// A call takes a slot whose previous call has completed, adding slots (up to
// kMaxDescSlots) while every slot is still in use, so that a long call on
// one HIP stream never holds back calls on other streams.
constexpr int kMaxDescSlots = 64;
struct DescRing {
  std::mutex mu;
  std::vector<std::unique_ptr<DescSlot>> slot;
  int next = 0;  // round-robin victim when all kMaxDescSlots are busy
  // long-reference stream extensions enqueued and perhaps still running, with
  // their workgroup counts
  std::vector<std::pair<std::shared_ptr<CallToken>, int>> long_inflight;
};
static DescRing g_ring[kMaxDevices];
static std::atomic<int> g_stream_bands{0};  // sdtw_stream_set_config (0: automatic)
static std::atomic<int> g_stream_strip{0};

static int ensure_slot(DescSlot& sl, int32_t n) {
  if (sl.cap >= n) return SDTW_OK;
  int32_t cap = std::max<int32_t>(n, std::max<int32_t>(2 * sl.cap, 1024));
  if (sl.host) (void)hipHostFree(sl.host);
  if (sl.dev) (void)hipFree(sl.dev);
  sl.host = nullptr;
  sl.dev = nullptr;
  sl.cap = 0;
  int rc = check_hip(hipHostMalloc((void**)&sl.host, sizeof(StreamItem) * (size_t)cap),
                     "sdtw_stream_extend: pinned descriptors");
  if (!rc)
    rc = check_hip(hipMalloc((void**)&sl.dev, sizeof(StreamItem) * (size_t)cap + 64),
                   "sdtw_stream_extend: device descriptors");
  if (rc) return rc;
  sl.cap = cap;
  return SDTW_OK;
}

// Segment minima of sdtw_stream_best_two.  The first allocation already
// holds 2^20 keys (8 MiB: e.g. 1,024 rows of 16 M columns), so that serving
// loops do not regrow it: hipFree of the old buffer would wait for all work
// on the device, including long launches on other HIP streams.
constexpr int64_t kMinPartKeys = int64_t(1) << 20;
static int ensure_part(DescSlot& sl, int64_t n) {
  if (sl.part_cap >= n) return SDTW_OK;
  const int64_t cap = std::max<int64_t>(std::max<int64_t>(n, 2 * sl.part_cap), kMinPartKeys);
  if (sl.part) (void)hipFree(sl.part);
  sl.part = nullptr;
  sl.part_cap = 0;
  int rc = check_hip(hipMalloc((void**)&sl.part, sizeof(uint64_t) * (size_t)cap),
                     "sdtw_stream_best_two: segment minima");
  if (rc) return rc;
  sl.part_cap = cap;
  return SDTW_OK;
}

// A descriptor slot for a call of n items: one whose previous call has
// completed, else a new one (up to kMaxDescSlots), else the round-robin
// victim after its call completes.  The caller holds ring.mu.
static int acquire_slot(DescRing& ring, int32_t n, DescSlot** out, const char* who) {
  DescSlot* pick = nullptr;
  for (auto& c : ring.slot) {
    if (!c->last || !c->last->ev || hipEventQuery(c->last->ev) == hipSuccess) {
      pick = c.get();
      break;
    }
  }
  if (!pick && (int)ring.slot.size() < kMaxDescSlots) {
    ring.slot.push_back(std::make_unique<DescSlot>());
    pick = ring.slot.back().get();
  }
  if (!pick) {
    pick = ring.slot[(size_t)ring.next].get();
    ring.next = (ring.next + 1) % kMaxDescSlots;
    int rc = check_hip(hipEventSynchronize(pick->last->ev), who);
    if (rc) return rc;
  }
  int rc = ensure_slot(*pick, n);
  if (rc) return rc;
  *out = pick;
  return SDTW_OK;
}

}  // namespace sdtw

using namespace sdtw;

#define SDTW_REQUIRE(cond, ...) \
  do {                          \
    if (!(cond)) return set_error(SDTW_EINVAL, __VA_ARGS__); \
  } while (0)

extern "C" {

const char* sdtw_last_error(void) { return g_err; }

int sdtw_version(void) { return 1; }

// ---------------------------------------------------------------------------
// preparation
// ---------------------------------------------------------------------------

int sdtw_prepare_reference(const uint8_t* genome_dev, int64_t L, const float* table_dev, int k,
                           double scale, float* z_dev, int16_t* codes_dev, int64_t* nsat_dev,
                           void* stream) {
  SDTW_REQUIRE(genome_dev && table_dev && z_dev, "sdtw_prepare_reference: null pointer");
  SDTW_REQUIRE(k >= 1 && k <= 12, "sdtw_prepare_reference: k=%d outside [1, 12]", k);
  SDTW_REQUIRE(L >= k, "sdtw_prepare_reference: genome length %lld < k=%d", (long long)L, k);
  SDTW_REQUIRE(L - k + 1 <= (int64_t)INT32_MAX / 2,
               "sdtw_prepare_reference: genome too long (%lld bases)", (long long)L);
  SDTW_REQUIRE(isfinite(scale) && scale > 0.0, "sdtw_prepare_reference: scale must be > 0");
  hipStream_t st = (hipStream_t)stream;
  double* scratch = nullptr;
  int rc = check_hip(hipMallocAsync((void**)&scratch, kRefPartials * sizeof(double), st),
                     "sdtw_prepare_reference: scratch");
  if (rc) return rc;
  rc = check_hip(launch_prepare_reference(genome_dev, L, table_dev, k, scale, z_dev, codes_dev,
                                          nsat_dev, scratch, st),
                 "sdtw_prepare_reference: launch");
  hipError_t e = hipFreeAsync(scratch, st);
  if (rc) return rc;
  return check_hip(e, "sdtw_prepare_reference: free");
}

int sdtw_prepare_queries(const float* raw_dev, const int64_t* offsets_dev, int32_t nq,
                         double scale, float* z_dev, int16_t* codes_dev, int64_t* nsat_dev,
                         void* stream) {
  SDTW_REQUIRE(raw_dev && offsets_dev && z_dev, "sdtw_prepare_queries: null pointer");
  SDTW_REQUIRE(nq >= 1, "sdtw_prepare_queries: nq=%d < 1", nq);
  SDTW_REQUIRE(isfinite(scale) && scale > 0.0, "sdtw_prepare_queries: scale must be > 0");
  return check_hip(launch_prepare_queries(raw_dev, offsets_dev, nq, scale, nullptr, nullptr,
                                          z_dev, codes_dev, nsat_dev, (hipStream_t)stream),
                   "sdtw_prepare_queries: launch");
}

int sdtw_prepare_queries_ex(const float* raw_dev, const int64_t* offsets_dev, int32_t nq,
                            double scale, const double* stats_in_dev, double* stats_out_dev,
                            float* z_dev, int16_t* codes_dev, int64_t* nsat_dev, void* stream) {
  SDTW_REQUIRE(raw_dev && offsets_dev && z_dev, "sdtw_prepare_queries_ex: null pointer");
  SDTW_REQUIRE(nq >= 1, "sdtw_prepare_queries_ex: nq=%d < 1", nq);
  SDTW_REQUIRE(isfinite(scale) && scale > 0.0, "sdtw_prepare_queries_ex: scale must be > 0");
  return check_hip(launch_prepare_queries(raw_dev, offsets_dev, nq, scale, stats_in_dev,
                                          stats_out_dev, z_dev, codes_dev, nsat_dev,
                                          (hipStream_t)stream),
                   "sdtw_prepare_queries_ex: launch");
}

int sdtw_detect_events(const float* raw_dev, const int64_t* offsets_dev, int32_t nreads,
                       int32_t trim, int32_t keep, float* events_dev, int32_t* counts_dev,
                       void* stream) {
  SDTW_REQUIRE(raw_dev && offsets_dev && events_dev && counts_dev,
               "sdtw_detect_events: null pointer");
  SDTW_REQUIRE(nreads >= 1, "sdtw_detect_events: nreads=%d < 1", nreads);
  SDTW_REQUIRE(trim >= 0 && keep >= 1 && keep <= SDTW_MAX_QUERY &&
                   (int64_t)trim + keep <= kMaxEventList,
               "sdtw_detect_events: trim=%d keep=%d outside trim >= 0, 1 <= keep <= %d, "
               "trim + keep <= %d", trim, keep, SDTW_MAX_QUERY, kMaxEventList);
  return check_hip(launch_detect_events(raw_dev, offsets_dev, 1, nullptr, nreads, trim, keep, 0,
                                        events_dev, counts_dev, (hipStream_t)stream),
                   "sdtw_detect_events: launch");
}

int sdtw_detect_events_prefix(const float* raw_dev, const int64_t* ranges_dev,
                              const int32_t* firsts_dev, int32_t nreads, int32_t max_first,
                              int32_t keep, float* events_dev, int32_t* counts_dev,
                              void* stream) {
  SDTW_REQUIRE(raw_dev && ranges_dev && firsts_dev && events_dev && counts_dev,
               "sdtw_detect_events_prefix: null pointer");
  SDTW_REQUIRE(nreads >= 1, "sdtw_detect_events_prefix: nreads=%d < 1", nreads);
  SDTW_REQUIRE(max_first >= 0 && keep >= 1 && keep <= SDTW_MAX_QUERY &&
                   (int64_t)max_first + keep <= kMaxEventList,
               "sdtw_detect_events_prefix: max_first=%d keep=%d outside max_first >= 0, "
               "1 <= keep <= %d, max_first + keep <= %d", max_first, keep, SDTW_MAX_QUERY,
               kMaxEventList);
  return check_hip(launch_detect_events(raw_dev, ranges_dev, 2, firsts_dev, nreads, max_first,
                                        keep, 1, events_dev, counts_dev, (hipStream_t)stream),
                   "sdtw_detect_events_prefix: launch");
}

int64_t sdtw_event_state_bytes(void) { return (int64_t)event_state_bytes(); }

int sdtw_event_state_init(void* states_dev, const int32_t* slots_dev, int32_t n, void* stream) {
  SDTW_REQUIRE(states_dev && slots_dev, "sdtw_event_state_init: null pointer");
  SDTW_REQUIRE(n >= 1, "sdtw_event_state_init: n=%d < 1", n);
  return check_hip(launch_event_state_init(states_dev, slots_dev, n, (hipStream_t)stream),
                   "sdtw_event_state_init: launch");
}

int sdtw_detect_events_continue(const float* raw_dev, const int64_t* ranges_dev,
                                const int32_t* slots_dev, void* states_dev, int32_t nreads,
                                int32_t trim, int32_t keep, float* events_dev,
                                int32_t* counts_dev, void* stream) {
  SDTW_REQUIRE(raw_dev && ranges_dev && slots_dev && states_dev && events_dev && counts_dev,
               "sdtw_detect_events_continue: null pointer");
  SDTW_REQUIRE(nreads >= 1, "sdtw_detect_events_continue: nreads=%d < 1", nreads);
  SDTW_REQUIRE(trim >= 0 && keep >= 1 && keep <= SDTW_MAX_QUERY,
               "sdtw_detect_events_continue: trim=%d keep=%d outside trim >= 0, "
               "1 <= keep <= %d", trim, keep, SDTW_MAX_QUERY);
  return check_hip(launch_events_continue(raw_dev, ranges_dev, slots_dev, states_dev, nreads,
                                          trim, keep, events_dev, counts_dev,
                                          (hipStream_t)stream),
                   "sdtw_detect_events_continue: launch");
}

// ---------------------------------------------------------------------------
// reference
// ---------------------------------------------------------------------------

int sdtw_load_reference(const void* ref, int64_t n, int dtype, int ref_is_device, void* stream,
                        sdtw_ref* out) {
  SDTW_REQUIRE(ref && out, "sdtw_load_reference: null pointer");
  SDTW_REQUIRE(dtype == SDTW_F32 || dtype == SDTW_I16, "sdtw_load_reference: bad dtype %d", dtype);
  SDTW_REQUIRE(n >= 1 && n <= (int64_t)INT32_MAX - 2 * kPadUnit,
               "sdtw_load_reference: length %lld outside [1, 2^31)", (long long)n);
  hipStream_t st = (hipStream_t)stream;
  const size_t esz = dtype == SDTW_I16 ? 2 : 4;
  const int64_t n_pad = padded_length(n);
  uint32_t* data = nullptr;
  void* tmp = nullptr;
  int32_t* nonfinite = nullptr;
  int32_t host_nonfinite = 0;
  int rc = check_hip(hipMalloc((void**)&data, (size_t)n_pad * 4), "sdtw_load_reference: alloc");
  if (!rc) rc = check_hip(hipMalloc((void**)&nonfinite, sizeof(int32_t)), "sdtw_load_reference: alloc");
  if (!rc) rc = check_hip(hipMemcpyAsync(nonfinite, &host_nonfinite, sizeof(int32_t),
                                         hipMemcpyHostToDevice, st), "sdtw_load_reference: copy");
  const void* src = ref;
  if (!rc && !ref_is_device) {
    rc = check_hip(hipMalloc(&tmp, (size_t)n * esz), "sdtw_load_reference: alloc");
    if (!rc) rc = check_hip(hipMemcpyAsync(tmp, ref, (size_t)n * esz, hipMemcpyHostToDevice, st),
                            "sdtw_load_reference: copy");
    src = tmp;
  }
  if (!rc) rc = check_hip(launch_layout_reference(src, n, dtype, data, n_pad, nonfinite, st),
                          "sdtw_load_reference: layout");
  if (!rc) rc = check_hip(hipMemcpyAsync(&host_nonfinite, nonfinite, sizeof(int32_t),
                                         hipMemcpyDeviceToHost, st), "sdtw_load_reference: copy");
  if (!rc) rc = check_hip(hipStreamSynchronize(st), "sdtw_load_reference: sync");
  if (tmp) (void)hipFree(tmp);
  if (nonfinite) (void)hipFree(nonfinite);
  if (!rc && host_nonfinite)
    rc = set_error(SDTW_EINVAL, "sdtw_load_reference: %d non-finite values", host_nonfinite);
  if (rc) {
    if (data) (void)hipFree(data);
    return rc;
  }
  sdtw_ref_s* r = new (std::nothrow) sdtw_ref_s;
  if (!r) {
    (void)hipFree(data);
    return set_error(SDTW_ENOMEM, "sdtw_load_reference: host allocation");
  }
  r->device = current_device();
  r->dtype = dtype;
  r->n = n;
  r->n_pad = n_pad;
  r->data = data;
  r->open_streams = 0;
  *out = r;
  return SDTW_OK;
}

int sdtw_reference_info(sdtw_ref ref, int64_t* n, int* dtype) {
  SDTW_REQUIRE(ref, "sdtw_reference_info: null reference");
  if (n) *n = ref->n;
  if (dtype) *dtype = ref->dtype;
  return SDTW_OK;
}

int sdtw_free_reference(sdtw_ref ref) {
  SDTW_REQUIRE(ref, "sdtw_free_reference: null reference");
  if (ref->open_streams > 0)
    return set_error(SDTW_ESTATE, "sdtw_free_reference: %d streams still open",
                     ref->open_streams.load());
  int rc = check_hip(hipFree(ref->data), "sdtw_free_reference");
  delete ref;
  return rc;
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

// One launch of the batch: reads order[first, first + count), longest first,
// run by the skew kernel with `chains` chains per lane and `bands` waves per
// read (chains == 0: the synchronised single-wave kernel).
struct LaunchGroup {
  int32_t first, count, max_m, chains, bands, max_band, band_target;
};

static std::vector<LaunchGroup> launch_groups(const sdtw_plan_s* p) {
  std::vector<LaunchGroup> g;
  int32_t pos = 0;
  const int32_t n = p->nq;
  for (int k = p->chains; k >= 1; k /= 2) {
    if (!valid_strip_chains(p->strip, k)) continue;
    const int bands = valid_skew_config(p->strip, k, p->bands) ? p->bands : 1;
    const int32_t target = bands > 1 ? p->band_rows : 0;
    const int32_t lo = skew_min_m(k);
    const int32_t start = pos;
    int32_t max_band = 0;
    while (pos < n && p->sorted_m[pos] >= lo) {
      max_band = std::max(max_band, skew_band_rows(p->sorted_m[pos], k, bands, target));
      ++pos;
    }
    if (pos > start)
      g.push_back({start, pos - start, p->sorted_m[start], k, bands, max_band, target});
  }
  if (pos < n) g.push_back({pos, n - pos, p->sorted_m[pos], 0, 1, 0, 0});
  return g;
}

// Resident waves per CU for a skew launch: whole workgroups of `bands` waves
// within the CU's 160 KiB of LDS, at most 16 waves (four per SIMD).
static int skew_waves_per_cu(int strip, int chains, int bands, int max_band,
                             bool stream = false) {
  const size_t per = skew_lds_bytes(strip, chains, bands, max_band, stream);
  const int groups = (int)std::min<size_t>(16 / bands, (160 * 1024) / std::max<size_t>(per, 1));
  return std::max(groups, 1) * bands;
}

// LDS to reserve per workgroup so that `blocks` workgroups spread evenly over
// the compute units: when there are fewer than the CUs could hold, reserve a
// 1/ceil(blocks/cus) share of a CU's 160 KiB (whole KiB) so that no CU takes
// more than its share (the dispatcher would otherwise fill some CUs up to
// their limit and leave others with less work).  `min_share` > 1 leaves room
// for that many launches at once on every CU.
static int32_t spread_lds(size_t need, int blocks, int groups_per_cu, int cus,
                          int min_share = 1) {
  constexpr size_t kCuLds = 160 * 1024;
  if ((int64_t)blocks >= (int64_t)groups_per_cu * cus) return 0;
  const int share = std::max((blocks + cus - 1) / cus, min_share);
  // 1 KiB less than the share leaves room for the kernel's static LDS (a
  // share-sized reservation would let only share - 1 workgroups in)
  const size_t cap = (size_t)max_lds_bytes() - 1024;
  const size_t want = (std::min(kCuLds / (size_t)share, cap + 1024) - 1024) & ~(size_t)1023;
  return want > need ? (int32_t)want : 0;
}

// Default launch shape.  A wave issues about one VALU instruction per 10
// cycles when its instructions depend on each other and no faster than one
// per 5 cycles however independent they are (measured on gfx950), while a
// SIMD issues one per about 4.3 cycles from two or more waves.  So every SIMD
// needs two or more waves: with four or more reads per SIMD one wave per
// read and one chain per lane; with fewer, each read is cut into two row
// bands when its rows allow (measured on 1,024 reads of 250-500 rows x 10 M
// columns: 1.73x one band, 1.23x four bands, whose 64 tile-switch steps per
// band of ~94 rows cost more than the extra waves bring), else two chains.
static void choose_config(sdtw_plan_s* p) {
  p->strip = 16;
  const int64_t simds = (int64_t)p->cus * 4;
  const int32_t median_m = p->sorted_m[(size_t)p->nq / 2];
  if (p->nq >= 4 * simds) {
    p->chains = 1;
    p->bands = 1;
  } else if (median_m >= 2 * skew_min_m(1)) {
    p->chains = 1;
    p->bands = 2;
  } else {
    p->chains = 2;
    p->bands = 1;
  }
  p->band_rows = 0;
  p->waves_per_cu = skew_waves_per_cu(p->strip, p->chains, p->bands,
                                      std::max(skew_band_rows(p->max_m, p->chains, p->bands),
                                               skew_min_m(p->chains)));
}

int sdtw_plan_create(const int64_t* offsets_host, int32_t nq, int dtype, sdtw_plan* out) {
  SDTW_REQUIRE(offsets_host && out, "sdtw_plan_create: null pointer");
  SDTW_REQUIRE(nq >= 1, "sdtw_plan_create: nq=%d < 1", nq);
  SDTW_REQUIRE(dtype == SDTW_F32 || dtype == SDTW_I16, "sdtw_plan_create: bad dtype %d", dtype);
  SDTW_REQUIRE(offsets_host[0] >= 0, "sdtw_plan_create: negative offset");
  std::vector<int32_t> order((size_t)nq);
  int32_t max_m = 0;
  for (int32_t r = 0; r < nq; ++r) {
    const int64_t m = offsets_host[r + 1] - offsets_host[r];
    SDTW_REQUIRE(m >= 1 && m <= SDTW_MAX_QUERY,
                 "sdtw_plan_create: read %d has length %lld outside [1, %d]", r, (long long)m,
                 SDTW_MAX_QUERY);
    order[(size_t)r] = r;
    max_m = std::max<int32_t>(max_m, (int32_t)m);
  }
  auto len = [&](int32_t r) { return offsets_host[r + 1] - offsets_host[r]; };
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return len(a) != len(b) ? len(a) > len(b) : a < b;
  });

  sdtw_plan_s* p = new (std::nothrow) sdtw_plan_s();
  if (!p) return set_error(SDTW_ENOMEM, "sdtw_plan_create: host allocation");
  p->device = current_device();
  p->dtype = dtype;
  p->nq = nq;
  p->max_m = max_m;
  p->sorted_m.resize((size_t)nq);
  for (int32_t i = 0; i < nq; ++i) p->sorted_m[(size_t)i] = (int32_t)len(order[(size_t)i]);
  p->cus = cu_count();
  if (p->cus <= 0) p->cus = 256;
  choose_config(p);
  int rc = check_hip(hipMalloc((void**)&p->offs_dev, sizeof(int64_t) * (size_t)(nq + 1)),
                     "sdtw_plan_create: alloc");
  if (!rc) rc = check_hip(hipMalloc((void**)&p->order_dev, sizeof(int32_t) * (size_t)nq),
                          "sdtw_plan_create: alloc");
  if (!rc) rc = check_hip(hipMalloc((void**)&p->sched_dev, sizeof(uint32_t) * kSchedWords),
                          "sdtw_plan_create: alloc");
  if (!rc) rc = check_hip(hipMemcpy(p->offs_dev, offsets_host, sizeof(int64_t) * (size_t)(nq + 1),
                                    hipMemcpyHostToDevice), "sdtw_plan_create: copy");
  if (!rc) rc = check_hip(hipMemcpy(p->order_dev, order.data(), sizeof(int32_t) * (size_t)nq,
                                    hipMemcpyHostToDevice), "sdtw_plan_create: copy");
  if (rc) {
    (void)hipFree(p->offs_dev);
    (void)hipFree(p->order_dev);
    (void)hipFree(p->sched_dev);
    delete p;
    return rc;
  }
  *out = p;
  return SDTW_OK;
}

int sdtw_plan_info(sdtw_plan plan, int32_t* nq, int* dtype, int32_t* max_m) {
  SDTW_REQUIRE(plan, "sdtw_plan_info: null plan");
  if (nq) *nq = plan->nq;
  if (dtype) *dtype = plan->dtype;
  if (max_m) *max_m = plan->max_m;
  return SDTW_OK;
}

int sdtw_plan_set_config(sdtw_plan plan, int strip, int chains, int bands, int waves_per_cu,
                         int32_t band_rows) {
  SDTW_REQUIRE(plan, "sdtw_plan_set_config: null plan");
  SDTW_REQUIRE(band_rows == -1 || band_rows == 0 || band_rows >= skew_min_m(1),
               "sdtw_plan_set_config: band_rows %d is not -1, 0 or >= %d", band_rows,
               skew_min_m(1));
  SDTW_REQUIRE(strip == 0 || valid_strip(strip), "sdtw_plan_set_config: strip %d not in {8,16,32}",
               strip);
  SDTW_REQUIRE(chains == 0 || chains == 1 || chains == 2 || chains == 4,
               "sdtw_plan_set_config: chains %d not in {1,2,4}", chains);
  SDTW_REQUIRE(bands >= 0 && bands <= 4, "sdtw_plan_set_config: bands %d not in {1,2,3,4}",
               bands);
  SDTW_REQUIRE(waves_per_cu >= 0 && waves_per_cu <= 32,
               "sdtw_plan_set_config: waves_per_cu %d outside [0, 32]", waves_per_cu);
  const int s2 = strip ? strip : plan->strip;
  const int k2 = chains ? chains : plan->chains;
  const int w2 = waves_per_cu ? waves_per_cu : plan->waves_per_cu;
  SDTW_REQUIRE(valid_strip_chains(s2, k2),
               "sdtw_plan_set_config: strip %d with %d chains (strip/chains must be a multiple "
               "of 4)", s2, k2);
  int b2 = bands;
  if (b2 == 0) {  // keep the plan's bands where they fit the rest, else one wave per read
    b2 = plan->bands;
    if (!valid_skew_config(s2, k2, b2) || w2 % b2 != 0) b2 = 1;
  }
  SDTW_REQUIRE(valid_skew_config(s2, k2, b2),
               "sdtw_plan_set_config: strip %d with %d chains and %d bands is not built "
               "(bands > 1: strip 16 with at most 2 chains, strip 32 with 1 chain, or strip "
               "32 with 2 chains and 2 bands)", s2, k2, b2);
  SDTW_REQUIRE(w2 % b2 == 0, "sdtw_plan_set_config: waves_per_cu %d is not a multiple of %d bands",
               w2, b2);
  plan->strip = s2;
  plan->chains = k2;
  plan->bands = b2;
  plan->waves_per_cu = w2;
  if (band_rows >= 0) plan->band_rows = band_rows;
  return SDTW_OK;
}

int sdtw_plan_get_config(sdtw_plan plan, int* strip, int* chains, int* bands, int* waves_per_cu,
                         int32_t* band_rows) {
  SDTW_REQUIRE(plan, "sdtw_plan_get_config: null plan");
  if (strip) *strip = plan->strip;
  if (chains) *chains = plan->chains;
  if (bands) *bands = plan->bands;
  if (waves_per_cu) *waves_per_cu = plan->waves_per_cu;
  if (band_rows) *band_rows = plan->band_rows;
  return SDTW_OK;
}

int sdtw_plan_destroy(sdtw_plan plan) {
  SDTW_REQUIRE(plan, "sdtw_plan_destroy: null plan");
  hipError_t e1 = hipFree(plan->offs_dev);
  hipError_t e2 = hipFree(plan->order_dev);
  hipError_t e3 = hipFree(plan->sched_dev);
  delete plan;
  if (e1 != hipSuccess) return check_hip(e1, "sdtw_plan_destroy");
  if (e2 != hipSuccess) return check_hip(e2, "sdtw_plan_destroy");
  return check_hip(e3, "sdtw_plan_destroy");
}

// ---------------------------------------------------------------------------
// alignment
// ---------------------------------------------------------------------------

// Enqueue the batch's launches; `n` reference columns (the autotuner times a
// prefix of the reference).
static int align_batch_impl(sdtw_ref ref, sdtw_plan plan, const void* q_dev, void* cost_dev,
                            int32_t* end_dev, hipStream_t st, int64_t n);

int sdtw_align_batch(sdtw_ref ref, sdtw_plan plan, const void* q_dev, void* cost_dev,
                     int32_t* end_dev, void* stream) {
  SDTW_REQUIRE(ref && plan, "sdtw_align_batch: null reference or plan");
  SDTW_REQUIRE(q_dev && cost_dev && end_dev, "sdtw_align_batch: null device pointer");
  SDTW_REQUIRE(ref->dtype == plan->dtype, "sdtw_align_batch: reference dtype %d != plan dtype %d",
               ref->dtype, plan->dtype);
  SDTW_REQUIRE(ref->device == plan->device, "sdtw_align_batch: reference and plan on devices %d, %d",
               ref->device, plan->device);
  if (int rc = require_device(ref->device, "sdtw_align_batch")) return rc;
  return align_batch_impl(ref, plan, q_dev, cost_dev, end_dev, (hipStream_t)stream, ref->n);
}

static int align_batch_impl(sdtw_ref ref, sdtw_plan plan, const void* q_dev, void* cost_dev,
                            int32_t* end_dev, hipStream_t st, int64_t n) {
  SDTW_REQUIRE(valid_strip(plan->strip), "sdtw_align_batch: bad strip");
  const std::vector<LaunchGroup> groups = launch_groups(plan);
  const size_t lds_max = (size_t)max_lds_bytes();
  for (const LaunchGroup& g : groups) {
    const size_t lds = g.chains ? skew_lds_bytes(plan->strip, g.chains, g.bands, g.max_band)
                                : plain_lds_bytes(plan->dtype, plan->strip, g.max_m);
    SDTW_REQUIRE(lds <= lds_max, "sdtw_align_batch: %zu bytes of LDS needed, %zu available", lds,
                 lds_max);
  }
  AlignArgs a{};
  a.ref = ref->data;
  a.n = n;
  a.q = q_dev;
  a.offs = plan->offs_dev;
  a.sched = plan->sched_dev;
  a.cost = cost_dev;
  a.end = end_dev;
  for (const LaunchGroup& g : groups) {
    a.order = plan->order_dev + g.first;
    a.nwork = g.count;
    a.max_m = g.max_m;
    a.max_band = g.max_band;
    a.band_target = g.band_target;
    int rc;
    if (g.chains) {
      const int groups_per_cu = std::max(plan->waves_per_cu / g.bands, 1);
      const int blocks = (int)std::min<int64_t>((int64_t)plan->cus * groups_per_cu, g.count);
      a.lds_bytes = spread_lds(skew_lds_bytes(plan->strip, g.chains, g.bands, g.max_band),
                               blocks, groups_per_cu, plan->cus);
      rc = check_hip(launch_align_skew(plan->dtype, plan->strip, g.chains, g.bands, blocks, a, st),
                     "sdtw_align_batch: launch");
    } else {
      rc = check_hip(launch_align_plain(plan->dtype, plan->strip, a, st),
                     "sdtw_align_batch: launch");
    }
    if (rc) return rc;
  }
  return SDTW_OK;
}

int sdtw_align_one(sdtw_ref ref, const void* q_dev, int32_t M, void* cost_dev, int32_t* end_dev,
                   void* stream) {
  SDTW_REQUIRE(ref, "sdtw_align_one: null reference");
  SDTW_REQUIRE(q_dev && cost_dev && end_dev, "sdtw_align_one: null device pointer");
  SDTW_REQUIRE(M >= 1 && M <= SDTW_MAX_QUERY, "sdtw_align_one: M=%d outside [1, %d]", M,
               SDTW_MAX_QUERY);
  if (int rc = require_device(ref->device, "sdtw_align_one")) return rc;
  AlignArgs a{};
  a.ref = ref->data;
  a.n = ref->n;
  a.q = q_dev;
  a.offs = nullptr;
  a.order = nullptr;
  a.nwork = 1;
  a.max_m = M;
  a.single_m = M;
  a.cost = cost_dev;
  a.end = end_dev;
  return check_hip(launch_align_plain(ref->dtype, 16, a, (hipStream_t)stream),
                   "sdtw_align_one: launch");
}

int sdtw_align_one_wide(sdtw_ref ref, const void* q_dev, int32_t M, int cols, void* cost_dev,
                        int32_t* end_dev, void* stream) {
  SDTW_REQUIRE(ref, "sdtw_align_one_wide: null reference");
  SDTW_REQUIRE(q_dev && cost_dev && end_dev, "sdtw_align_one_wide: null device pointer");
  SDTW_REQUIRE(ref->dtype == SDTW_I16, "sdtw_align_one_wide: int16 references only");
  SDTW_REQUIRE(M >= 1 && M <= SDTW_MAX_QUERY, "sdtw_align_one_wide: M=%d outside [1, %d]", M,
               SDTW_MAX_QUERY);
  SDTW_REQUIRE(cols == 0 || cols == 8 || cols == 16 || cols == 32 || cols == 64,
               "sdtw_align_one_wide: cols=%d not in {0, 8, 16, 32, 64}", cols);
  if (int rc = require_device(ref->device, "sdtw_align_one_wide")) return rc;
  if (cols == 0) cols = wide_pick_cols(ref->n, ref->device);
  SDTW_REQUIRE(wide_tiles(ref->n, cols) <= (int64_t)INT32_MAX,
               "sdtw_align_one_wide: reference too long for %d columns per thread", cols);
  const int dev = ref->device;
  DescRing& ring = g_ring[dev >= 0 && dev < kMaxDevices ? dev : 0];
  std::lock_guard<std::mutex> g(ring.mu);
  DescSlot* pick = nullptr;
  int rc = acquire_slot(ring, 1, &pick, "sdtw_align_one_wide");
  if (rc) return rc;
  DescSlot& sl = *pick;
  rc = ensure_part(sl, wide_scratch_words(ref->n, M, cols));
  if (rc) return rc;
  auto tok = std::make_shared<CallToken>();
  tok->ev = event_get();
  if (!tok->ev) return set_error(SDTW_EDEVICE, "sdtw_align_one_wide: event creation failed");
  hipStream_t st = (hipStream_t)stream;
  rc = check_hip(launch_align_wide(ref->data, ref->n, (const int16_t*)q_dev, M, cols, sl.part,
                                   (int32_t*)cost_dev, end_dev, st),
                 "sdtw_align_one_wide: launch");
  const int rc_ev = check_hip(hipEventRecord(tok->ev, st), "sdtw_align_one_wide: record");
  if (!rc_ev) sl.last = tok;
  return rc ? rc : rc_ev;
}

int sdtw_align_one_wide_noalloc(sdtw_ref ref, const void* q_dev, int32_t M, int cols,
                                void* cost_dev, int32_t* end_dev, void* stream) {
  SDTW_REQUIRE(ref, "sdtw_align_one_wide_noalloc: null reference");
  SDTW_REQUIRE(q_dev && cost_dev && end_dev, "sdtw_align_one_wide_noalloc: null device pointer");
  SDTW_REQUIRE(ref->dtype == SDTW_I16, "sdtw_align_one_wide_noalloc: int16 references only");
  SDTW_REQUIRE(M >= 1 && M <= SDTW_MAX_QUERY, "sdtw_align_one_wide_noalloc: M=%d outside [1, %d]",
               M, SDTW_MAX_QUERY);
  SDTW_REQUIRE(cols == 0 || cols == 8 || cols == 16 || cols == 32 || cols == 64,
               "sdtw_align_one_wide_noalloc: cols=%d not in {0, 8, 16, 32, 64}", cols);
  if (int rc = require_device(ref->device, "sdtw_align_one_wide_noalloc")) return rc;
  if (cols == 0) cols = wide_pick_cols(ref->n, ref->device);
  SDTW_REQUIRE(wide_tiles(ref->n, cols) <= (int64_t)INT32_MAX,
               "sdtw_align_one_wide_noalloc: reference too long for %d columns per thread", cols);
  const int64_t need = wide_scratch_words(ref->n, M, cols);
  SDTW_REQUIRE(need <= wide_noalloc_words(),
               "sdtw_align_one_wide_noalloc: %d rows x %lld columns at %d columns per thread "
               "need %lld words of scratch, the fixed array holds %lld", M, (long long)ref->n,
               cols, (long long)need, (long long)wide_noalloc_words());
  uint64_t* scratch = nullptr;
  int rc = check_hip(wide_noalloc_scratch(ref->device, &scratch),
                     "sdtw_align_one_wide_noalloc: scratch address");
  if (rc) return rc;
  return check_hip(launch_align_wide(ref->data, ref->n, (const int16_t*)q_dev, M, cols, scratch,
                                     (int32_t*)cost_dev, end_dev, (hipStream_t)stream),
                   "sdtw_align_one_wide_noalloc: launch");
}

// ---------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {
// Tuned launch shapes are remembered per (architecture and compute units,
// dtype, reference length, batch shape class); the batch shape class puts
// the number of reads, the median and the longest read length each into
// quarter-octave buckets, so batches of about the same shape (a serving
// loop's ragged batches, a workload drawn again) share a tuned shape.
struct TuneKey {
  std::string arch;
  int cus, dtype;
  int64_t n;
  int nq_b, med_b, max_b;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, cus, dtype, n, nq_b, med_b, max_b) <
           std::tie(o.arch, o.cus, o.dtype, o.n, o.nq_b, o.med_b, o.max_b);
  }
};
struct TuneVal {
  int strip, chains, bands, waves_per_cu;
  int32_t band_rows;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tuned;  // best configuration per key
bool g_tune_file_read = false;

int quarter_octave(int64_t v) { return (int)lround(4.0 * log2((double)std::max<int64_t>(v, 1))); }

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  for (char& c : a)
    if (c == ' ') c = '_';
  return a;
}

TuneKey tune_key(const sdtw_plan_s* p, int64_t n) {
  return {device_arch(p->device), p->cus, p->dtype, n, quarter_octave(p->nq),
          quarter_octave(p->sorted_m[p->sorted_m.size() / 2]), quarter_octave(p->max_m)};
}

// Optional persistence: SDTW_TUNE_CACHE names a text file with one tuned
// shape per line ("arch cus dtype n nq_b med_b max_b strip chains bands
// waves_per_cu band_rows"), read once per process and rewritten after every
// autotune.  Unset or empty: the cache lives in this process only.
const char* tune_file() {
  const char* f = getenv("SDTW_TUNE_CACHE");
  return (f && *f) ? f : nullptr;
}

void tune_file_read_locked() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = tune_file();
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char arch[256];
  TuneKey k;
  TuneVal v;
  long long n;
  while (fscanf(f, "%255s %d %d %lld %d %d %d %d %d %d %d %d", arch, &k.cus, &k.dtype, &n,
                &k.nq_b, &k.med_b, &k.max_b, &v.strip, &v.chains, &v.bands, &v.waves_per_cu,
                &v.band_rows) == 12) {
    k.arch = arch;
    k.n = n;
    if (valid_skew_config(v.strip, v.chains, v.bands) && v.waves_per_cu >= v.bands &&
        v.waves_per_cu <= 32 && v.waves_per_cu % v.bands == 0)
      g_tuned[k] = v;
  }
  fclose(f);
}

void tune_file_write_locked() {
  const char* path = tune_file();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto& kv : g_tuned) {
    const TuneKey& k = kv.first;
    const TuneVal& v = kv.second;
    fprintf(f, "%s %d %d %lld %d %d %d %d %d %d %d %d\n", k.arch.c_str(), k.cus, k.dtype,
            (long long)k.n, k.nq_b, k.med_b, k.max_b, v.strip, v.chains, v.bands,
            v.waves_per_cu, (int)v.band_rows);
  }
  if (fclose(f) == 0) rename(tmp.c_str(), path);
}
}  // namespace

extern "C" {

int sdtw_plan_autotune(sdtw_ref ref, sdtw_plan plan, const void* q_dev, void* cost_dev,
                       int32_t* end_dev, int64_t max_columns, void* stream) {
  SDTW_REQUIRE(ref && plan, "sdtw_plan_autotune: null reference or plan");
  SDTW_REQUIRE(q_dev && cost_dev && end_dev, "sdtw_plan_autotune: null device pointer");
  SDTW_REQUIRE(ref->dtype == plan->dtype,
               "sdtw_plan_autotune: reference dtype %d != plan dtype %d", ref->dtype,
               plan->dtype);
  SDTW_REQUIRE(max_columns >= 0, "sdtw_plan_autotune: negative max_columns");
  SDTW_REQUIRE(ref->device == plan->device,
               "sdtw_plan_autotune: reference and plan on devices %d, %d", ref->device,
               plan->device);
  if (int rc = require_device(ref->device, "sdtw_plan_autotune")) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = max_columns ? std::min<int64_t>(ref->n, max_columns) : ref->n;
  // candidates: every strip / chains / bands the kernel is built for with
  // strip >= 16 and at most 2 chains, each at the resident waves per CU its
  // LDS allows and at half that
  // and, with 3 or 4 bands, targets of a half and a third of the median read
  // (equal band heights for reads of different lengths)
  std::vector<TuneVal> cand;
  const int32_t median_m = plan->sorted_m[plan->sorted_m.size() / 2];
  for (int strip : {16, 32})
    for (int chains : {1, 2})
      for (int bands : {1, 2, 3, 4}) {
        if (!valid_skew_config(strip, chains, bands)) continue;
        if (bands > 1 && plan->max_m < bands * skew_min_m(chains)) continue;
        std::vector<int32_t> targets = {0};
        if (bands > 2)
          for (int32_t t : {(median_m + 1) / 2, (median_m + 2) / 3})
            if (t >= skew_min_m(chains)) targets.push_back(t);
        for (int32_t target : targets) {
          const int band_rows = std::max(skew_band_rows(plan->max_m, chains, bands, target),
                                         skew_min_m(chains));
          const int w = skew_waves_per_cu(strip, chains, bands, band_rows);
          cand.push_back({strip, chains, bands, w, target});
          if (w / 2 >= bands && (w / 2) % bands == 0)
            cand.push_back({strip, chains, bands, w / 2, target});
        }
      }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_error(SDTW_EDEVICE, "sdtw_plan_autotune: event creation failed");
  }
  const TuneVal keep = {plan->strip, plan->chains, plan->bands, plan->waves_per_cu,
                        plan->band_rows};
  TuneVal best = keep;
  int rc = SDTW_OK;
  // two passes over the candidates, the second in reverse order, each
  // candidate timed once per pass after a warm-up launch, keeping its faster
  // time: the first pass also brings the clock up (the first launches of a
  // cold device run slower), a single timing can misorder shapes a few
  // percent apart, and a clock that drifts during the passes favours no
  // position in the list
  std::vector<float> cand_ms(cand.size(), 0.f);
  for (int pass = 0; pass < 2 && !rc; ++pass) {
    for (size_t j = 0; j < cand.size(); ++j) {
      const size_t i = pass == 0 ? j : cand.size() - 1 - j;
      const TuneVal& c = cand[i];
      plan->strip = c.strip;
      plan->chains = c.chains;
      plan->bands = c.bands;
      plan->waves_per_cu = c.waves_per_cu;
      plan->band_rows = c.band_rows;
      rc = align_batch_impl(ref, plan, q_dev, cost_dev, end_dev, st, n);  // warm-up
      if (!rc) rc = check_hip(hipEventRecord(e0, st), "sdtw_plan_autotune: record");
      if (!rc) rc = align_batch_impl(ref, plan, q_dev, cost_dev, end_dev, st, n);
      if (!rc) rc = check_hip(hipEventRecord(e1, st), "sdtw_plan_autotune: record");
      if (!rc) rc = check_hip(hipEventSynchronize(e1), "sdtw_plan_autotune: wait");
      float ms = 0.f;
      if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "sdtw_plan_autotune: time");
      if (rc) break;
      if (cand_ms[i] == 0.f || ms < cand_ms[i]) cand_ms[i] = ms;
    }
  }
  float best_ms = 0.f;
  for (size_t i = 0; i < cand.size() && !rc; ++i) {
    if (best_ms == 0.f || cand_ms[i] < best_ms) {
      best_ms = cand_ms[i];
      best = cand[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->strip = best.strip;
  plan->chains = best.chains;
  plan->bands = best.bands;
  plan->waves_per_cu = best.waves_per_cu;
  plan->band_rows = best.band_rows;
  if (rc) return rc;
  const TuneKey key = tune_key(plan, ref->n);
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_file_read_locked();
  g_tuned[key] = best;
  tune_file_write_locked();
  return SDTW_OK;
}

int sdtw_plan_use_tuned(sdtw_ref ref, sdtw_plan plan, int* found) {
  SDTW_REQUIRE(ref && plan, "sdtw_plan_use_tuned: null reference or plan");
  const TuneKey key = tune_key(plan, ref->n);
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_file_read_locked();
  auto it = g_tuned.find(key);
  if (found) *found = it != g_tuned.end();
  if (it != g_tuned.end()) {
    plan->strip = it->second.strip;
    plan->chains = it->second.chains;
    plan->bands = it->second.bands;
    plan->waves_per_cu = it->second.waves_per_cu;
    plan->band_rows = it->second.band_rows;
  }
  return SDTW_OK;
}

// ---------------------------------------------------------------------------
// streaming extension
// ---------------------------------------------------------------------------

int sdtw_set_row_budget(int64_t bytes) {
  SDTW_REQUIRE(bytes >= 0, "sdtw_set_row_budget: negative budget");
  RowPool* pl = pool_for(current_device());
  SDTW_REQUIRE(pl, "sdtw_set_row_budget: no current device");
  std::lock_guard<std::mutex> g(pl->mu);
  pl->budget = bytes;
  return SDTW_OK;
}

int sdtw_row_pool_trim(void) {
  const int dev = current_device();
  RowPool* pl = pool_for(dev);
  SDTW_REQUIRE(pl, "sdtw_row_pool_trim: no current device");
  std::lock_guard<std::mutex> g(pl->mu);
  hipError_t first = hipSuccess;
  for (auto& kv : pl->free_rows) {
    for (void* row : kv.second) {
      const hipError_t e = hipFree(row);
      if (first == hipSuccess) first = e;
      pl->cached -= (int64_t)kv.first;
    }
  }
  pl->free_rows.clear();
  return check_hip(first, "sdtw_row_pool_trim");
}

int sdtw_row_budget_info(int64_t* budget, int64_t* in_use, int64_t* cached) {
  RowPool* pl = pool_for(current_device());
  SDTW_REQUIRE(pl, "sdtw_row_budget_info: no current device");
  std::lock_guard<std::mutex> g(pl->mu);
  if (budget) *budget = pl->budget;
  if (in_use) *in_use = pl->in_use;
  if (cached) *cached = pl->cached;
  return SDTW_OK;
}

int sdtw_stream_open(sdtw_ref ref, sdtw_stream* out) {
  SDTW_REQUIRE(ref && out, "sdtw_stream_open: null pointer");
  if (int rc = require_device(ref->device, "sdtw_stream_open")) return rc;
  RowPool* pl = pool_for(ref->device);
  SDTW_REQUIRE(pl, "sdtw_stream_open: bad device");
  const size_t bytes = sizeof(uint32_t) * (size_t)ref->n_pad;
  void* row = nullptr;
  {
    std::lock_guard<std::mutex> g(pl->mu);
    if (pl->in_use + (int64_t)bytes > pl->budget)
      return set_error(SDTW_EBUDGET, "sdtw_stream_open: %zu more bytes exceed the row budget "
                       "(%lld in use of %lld)", bytes, (long long)pl->in_use,
                       (long long)pl->budget);
    auto it = pl->free_rows.find(bytes);
    if (it != pl->free_rows.end() && !it->second.empty()) {
      row = it->second.back();
      it->second.pop_back();
      pl->cached -= (int64_t)bytes;
    } else {
      // make room in the budget by releasing cached rows of other sizes
      for (auto& kv : pl->free_rows) {
        while (pl->in_use + pl->cached + (int64_t)bytes > pl->budget && !kv.second.empty()) {
          (void)hipFree(kv.second.back());
          kv.second.pop_back();
          pl->cached -= (int64_t)kv.first;
        }
      }
      if (hipMalloc(&row, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(SDTW_ENOMEM, "sdtw_stream_open: device allocation of %zu bytes", bytes);
      }
    }
    pl->in_use += (int64_t)bytes;
  }
  sdtw_stream_s* s = new (std::nothrow) sdtw_stream_s();
  if (!s) {
    std::lock_guard<std::mutex> g(pl->mu);
    pl->free_rows[bytes].push_back(row);
    pl->in_use -= (int64_t)bytes;
    pl->cached += (int64_t)bytes;
    return set_error(SDTW_ENOMEM, "sdtw_stream_open: host allocation");
  }
  s->device = ref->device;
  s->ref = ref;
  s->row = (uint32_t*)row;
  s->bytes = bytes;
  s->rows = 0;
  ref->open_streams++;
  *out = s;
  return SDTW_OK;
}

int sdtw_stream_info(sdtw_stream s, int32_t* rows, int64_t* n) {
  SDTW_REQUIRE(s, "sdtw_stream_info: null stream");
  if (rows) *rows = s->rows;
  if (n) *n = s->ref->n;
  return SDTW_OK;
}

int sdtw_stream_close(sdtw_stream s) {
  SDTW_REQUIRE(s, "sdtw_stream_close: null stream");
  // the row may still be read or written by enqueued work
  if (s->last && s->last->ev) {
    int rc = check_hip(hipEventSynchronize(s->last->ev), "sdtw_stream_close: wait");
    if (rc) return rc;
  }
  RowPool* pl = pool_for(s->device);
  {
    std::lock_guard<std::mutex> g(pl->mu);
    pl->free_rows[s->bytes].push_back(s->row);
    pl->in_use -= (int64_t)s->bytes;
    pl->cached += (int64_t)s->bytes;
  }
  s->ref->open_streams--;
  delete s;
  return SDTW_OK;
}

int sdtw_stream_copy_row(sdtw_stream s, void* dst_dev, void* stream) {
  SDTW_REQUIRE(s && dst_dev, "sdtw_stream_copy_row: null pointer");
  if (int rc = require_device(s->device, "sdtw_stream_copy_row")) return rc;
  if (s->rows == 0)
    return set_error(SDTW_ESTATE, "sdtw_stream_copy_row: the stream has no rows yet");
  return check_hip(hipMemcpyAsync(dst_dev, s->row, sizeof(uint32_t) * (size_t)s->ref->n,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream),
                   "sdtw_stream_copy_row");
}

int sdtw_stream_set_config(sdtw_ref ref, int strip, int bands) {
  SDTW_REQUIRE(strip == 0 || strip == 16 || strip == 32,
               "sdtw_stream_set_config: strip %d not in {0,16,32}", strip);
  SDTW_REQUIRE(bands >= 0 && bands <= 4, "sdtw_stream_set_config: bands %d not in {0,1,2,3,4}",
               bands);
  if (ref) {
    ref->stream_strip.store(strip);
    ref->stream_bands.store(bands);
  } else {
    g_stream_strip.store(strip);
    g_stream_bands.store(bands);
  }
  return SDTW_OK;
}

int sdtw_stream_extend(const sdtw_stream* streams, int32_t ns, const void* chunk_dev,
                       const int64_t* chunk_offsets_host, void* cost_dev, int32_t* end_dev,
                       void* stream) {
  SDTW_REQUIRE(streams && chunk_dev && chunk_offsets_host && cost_dev && end_dev,
               "sdtw_stream_extend: null pointer");
  SDTW_REQUIRE(ns >= 1, "sdtw_stream_extend: ns=%d < 1", ns);
  SDTW_REQUIRE(streams[0], "sdtw_stream_extend: stream 0 is null");
  const sdtw_ref ref = streams[0]->ref;
  const int dtype = ref->dtype;
  if (int rc = require_device(ref->device, "sdtw_stream_extend")) return rc;
  const int32_t row_cap = dtype == SDTW_I16 ? 32767 : INT32_MAX;
  std::set<const sdtw_stream_s*> seen;
  std::vector<int32_t> order((size_t)ns);
  int32_t max_m = 0;
  for (int32_t i = 0; i < ns; ++i) {
    const sdtw_stream s = streams[i];
    SDTW_REQUIRE(s, "sdtw_stream_extend: stream %d is null", i);
    SDTW_REQUIRE(s->ref == ref, "sdtw_stream_extend: stream %d uses another reference", i);
    SDTW_REQUIRE(seen.insert(s).second, "sdtw_stream_extend: stream %d appears twice", i);
    const int64_t m = chunk_offsets_host[i + 1] - chunk_offsets_host[i];
    SDTW_REQUIRE(chunk_offsets_host[i] >= 0 && m >= 1 && m <= SDTW_MAX_QUERY,
                 "sdtw_stream_extend: chunk %d has length %lld outside [1, %d]", i,
                 (long long)m, SDTW_MAX_QUERY);
    SDTW_REQUIRE((int64_t)s->rows + m <= row_cap,
                 "sdtw_stream_extend: stream %d would exceed %d rows", i, row_cap);
    order[(size_t)i] = i;
    max_m = std::max<int32_t>(max_m, (int32_t)m);
  }
  auto len = [&](int32_t i) { return chunk_offsets_host[i + 1] - chunk_offsets_host[i]; };
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return len(a) != len(b) ? len(a) > len(b) : a < b;
  });
  // One chain per lane.  Automatic shape: more waves per chunk the fewer
  // chunks there are (a chunk's latency shrinks with its bands while the
  // device is not full): four bands up to two chunks per compute unit (two
  // workgroups of four bands fit on a CU, two waves per SIMD), two up to
  // four, then one; strip 32 for references of 2^20 columns and more (half
  // the tiles per chunk), else 16, whose workgroups need a third of strip
  // 32's LDS, so that short-reference calls find room beside long-reference
  // ones.
  constexpr int kChains = 1;
  const int cus = std::max(cu_count(), 1);
  int bands = ref->stream_bands.load();
  if (bands == 0) bands = g_stream_bands.load();
  if (bands == 0) bands = ns <= 2 * cus ? 4 : (ns <= 4 * cus ? 2 : 1);
  int kStrip = ref->stream_strip.load();
  if (kStrip == 0) kStrip = g_stream_strip.load();
  if (kStrip == 0) kStrip = ref->n >= (int64_t(1) << 20) ? 32 : 16;
  int32_t nbig = 0, max_band = 0;
  while (nbig < ns && len(order[(size_t)nbig]) >= skew_min_m(kChains)) {
    max_band = std::max(max_band, skew_band_rows((int32_t)len(order[(size_t)nbig]), kChains, bands));
    ++nbig;
  }
  const size_t lds_max = (size_t)max_lds_bytes();
  SDTW_REQUIRE(skew_lds_bytes(kStrip, kChains, bands, max_band, true) <= lds_max &&
                   plain_lds_bytes(dtype, kStrip, max_m) <= lds_max,
               "sdtw_stream_extend: chunk of %d rows needs more LDS than available", max_m);

  const int dev = ref->device;
  DescRing& ring = g_ring[dev >= 0 && dev < kMaxDevices ? dev : 0];
  std::lock_guard<std::mutex> g(ring.mu);
  DescSlot* pick = nullptr;
  int rc = acquire_slot(ring, ns, &pick, "sdtw_stream_extend");
  if (rc) return rc;
  DescSlot& sl = *pick;
  for (int32_t t = 0; t < ns; ++t) {
    const int32_t i = order[(size_t)t];
    StreamItem& it = sl.host[t];
    it.acc = streams[i]->row;
    it.q0 = chunk_offsets_host[i];
    it.m = (int32_t)len(i);
    it.m_old = streams[i]->rows;
    it.out = i;
    it.pad = 0;
  }
  auto tok = std::make_shared<CallToken>();
  tok->ev = event_get();
  if (!tok->ev) return set_error(SDTW_EDEVICE, "sdtw_stream_extend: event creation failed");
  hipStream_t st = (hipStream_t)stream;
  rc = check_hip(hipMemcpyAsync(sl.dev, sl.host, sizeof(StreamItem) * (size_t)ns,
                                hipMemcpyHostToDevice, st),
                 "sdtw_stream_extend: descriptors");
  AlignArgs a{};
  a.ref = ref->data;
  a.n = ref->n;
  a.q = chunk_dev;
  a.counter = (int32_t*)(sl.dev + sl.cap);
  a.cost = cost_dev;
  a.end = end_dev;
  int long_blocks = 0;
  if (!rc && nbig) {
    a.items = sl.dev;
    a.nwork = nbig;
    a.max_m = (int32_t)len(order[0]);
    a.max_band = max_band;
    // No LDS reservation (spread_lds): calls in flight on other HIP streams
    // (other targets, the next batch) must find room on every CU.  Except
    // for long references while this launch and the long-reference launches
    // still running have at most one workgroup per CU between them: two
    // long-reference workgroups fit on a CU (two waves per SIMD), which pays
    // once the device is full, but with CUs idle the dispatcher would also
    // put the next batch's workgroups beside this one's, each then slower
    // than alone on a CU of its own.  Such a launch reserves enough LDS that
    // no second long-reference workgroup joins one of its CUs (short-
    // reference ones, a third of the size, still do).
    const int wpc = skew_waves_per_cu(kStrip, kChains, bands, max_band, true);
    const int blocks = (int)std::min<int64_t>((int64_t)cus * (wpc / bands), nbig);
    int64_t running = 0;
    if (kStrip == 32) {
      auto& v = ring.long_inflight;
      v.erase(std::remove_if(v.begin(), v.end(),
                             [](const std::pair<std::shared_ptr<CallToken>, int>& e) {
                               if (!e.first->ev) return true;
                               if (hipEventQuery(e.first->ev) != hipErrorNotReady) return true;
                               (void)hipGetLastError();  // "not ready" is no error here
                               return false;
                             }),
              v.end());
      for (const auto& e : v) running += e.second;
    }
    a.lds_bytes = 0;
    if (kStrip == 32 && 2 * (blocks + running) <= cus) {
      const size_t need = skew_lds_bytes(kStrip, kChains, bands, max_band, true);
      const size_t alone = ((160 * 1024 - need + 1024 + 1023) & ~(size_t)1023);
      if (alone > need && alone <= lds_max) a.lds_bytes = (int32_t)alone;
    }
    rc = check_hip(launch_align_skew(dtype, kStrip, kChains, bands, blocks, a, st, true),
                   "sdtw_stream_extend: launch");
    if (kStrip == 32) long_blocks = blocks;
  }
  if (!rc && nbig < ns) {
    a.items = sl.dev + nbig;
    a.nwork = ns - nbig;
    a.max_m = (int32_t)len(order[(size_t)nbig]);
    rc = check_hip(launch_align_plain(dtype, kStrip, a, st, true), "sdtw_stream_extend: launch");
  }
  // the slot is busy until this point of the stream, whatever was enqueued
  const int rc_ev = check_hip(hipEventRecord(tok->ev, st), "sdtw_stream_extend: record");
  if (!rc_ev) sl.last = tok;
  if (!rc) rc = rc_ev;
  if (rc) return rc;
  if (long_blocks) ring.long_inflight.emplace_back(tok, long_blocks);
  for (int32_t i = 0; i < ns; ++i) {
    streams[i]->rows += (int32_t)len(i);
    streams[i]->last = tok;
  }
  return SDTW_OK;
}

int sdtw_stream_extend_wide(sdtw_stream s, const void* chunk_dev, int32_t M, int cols,
                            void* cost_dev, int32_t* end_dev, void* stream) {
  SDTW_REQUIRE(s && chunk_dev && cost_dev && end_dev, "sdtw_stream_extend_wide: null pointer");
  const sdtw_ref ref = s->ref;
  SDTW_REQUIRE(ref->dtype == SDTW_I16, "sdtw_stream_extend_wide: int16 references only");
  SDTW_REQUIRE(M >= 1 && (int64_t)s->rows + M <= SDTW_MAX_QUERY,
               "sdtw_stream_extend_wide: %d rows folded in plus a chunk of %d exceed %d", s->rows,
               M, SDTW_MAX_QUERY);
  SDTW_REQUIRE(cols == 0 || cols == 8 || cols == 16 || cols == 32 || cols == 64,
               "sdtw_stream_extend_wide: cols=%d not in {0, 8, 16, 32, 64}", cols);
  if (int rc = require_device(ref->device, "sdtw_stream_extend_wide")) return rc;
  if (cols == 0) cols = wide_pick_cols(ref->n, ref->device);
  SDTW_REQUIRE(wide_tiles(ref->n, cols) <= (int64_t)INT32_MAX,
               "sdtw_stream_extend_wide: reference too long for %d columns per thread", cols);
  const int dev = ref->device;
  DescRing& ring = g_ring[dev >= 0 && dev < kMaxDevices ? dev : 0];
  std::lock_guard<std::mutex> g(ring.mu);
  DescSlot* pick = nullptr;
  int rc = acquire_slot(ring, 1, &pick, "sdtw_stream_extend_wide");
  if (rc) return rc;
  DescSlot& sl = *pick;
  rc = ensure_part(sl, wide_scratch_words(ref->n, M, cols));
  if (rc) return rc;
  auto tok = std::make_shared<CallToken>();
  tok->ev = event_get();
  if (!tok->ev) return set_error(SDTW_EDEVICE, "sdtw_stream_extend_wide: event creation failed");
  hipStream_t st = (hipStream_t)stream;
  rc = check_hip(launch_align_wide(ref->data, ref->n, (const int16_t*)chunk_dev, M, cols, sl.part,
                                   (int32_t*)cost_dev, end_dev, st, s->row, s->rows > 0),
                 "sdtw_stream_extend_wide: launch");
  const int rc_ev = check_hip(hipEventRecord(tok->ev, st), "sdtw_stream_extend_wide: record");
  if (!rc_ev) sl.last = tok;
  if (!rc) rc = rc_ev;
  if (rc) return rc;
  s->rows += M;
  s->last = tok;
  return SDTW_OK;
}

int sdtw_stream_best_two(const sdtw_stream* streams, int32_t ns, int32_t window,
                         void* best_cost_dev, int32_t* best_end_dev, void* second_cost_dev,
                         int32_t* second_end_dev, void* stream) {
  SDTW_REQUIRE(streams && best_cost_dev && best_end_dev && second_cost_dev && second_end_dev,
               "sdtw_stream_best_two: null pointer");
  SDTW_REQUIRE(ns >= 1, "sdtw_stream_best_two: ns=%d < 1", ns);
  SDTW_REQUIRE(window >= 0, "sdtw_stream_best_two: negative window");
  SDTW_REQUIRE(streams[0], "sdtw_stream_best_two: stream 0 is null");
  const sdtw_ref ref = streams[0]->ref;
  if (int rc = require_device(ref->device, "sdtw_stream_best_two")) return rc;
  for (int32_t i = 0; i < ns; ++i) {
    SDTW_REQUIRE(streams[i], "sdtw_stream_best_two: stream %d is null", i);
    SDTW_REQUIRE(streams[i]->ref == ref, "sdtw_stream_best_two: stream %d uses another reference",
                 i);
    if (streams[i]->rows == 0)
      return set_error(SDTW_ESTATE, "sdtw_stream_best_two: stream %d has no rows yet", i);
  }
  const int dev = ref->device;
  DescRing& ring = g_ring[dev >= 0 && dev < kMaxDevices ? dev : 0];
  std::lock_guard<std::mutex> g(ring.mu);
  DescSlot* pick = nullptr;
  int rc = acquire_slot(ring, ns, &pick, "sdtw_stream_best_two");
  if (rc) return rc;
  DescSlot& sl = *pick;
  const int64_t nseg = best_two_segments(ref->n);
  SDTW_REQUIRE((int64_t)ns * nseg <= (int64_t)INT32_MAX,
               "sdtw_stream_best_two: %d rows of %lld columns exceed one launch", ns,
               (long long)ref->n);
  rc = ensure_part(sl, (int64_t)ns * nseg);
  if (rc) return rc;
  for (int32_t i = 0; i < ns; ++i) {
    StreamItem& it = sl.host[i];
    it = StreamItem{};
    it.acc = streams[i]->row;
    it.out = i;
  }
  auto tok = std::make_shared<CallToken>();
  tok->ev = event_get();
  if (!tok->ev) return set_error(SDTW_EDEVICE, "sdtw_stream_best_two: event creation failed");
  hipStream_t st = (hipStream_t)stream;
  rc = check_hip(hipMemcpyAsync(sl.dev, sl.host, sizeof(StreamItem) * (size_t)ns,
                                hipMemcpyHostToDevice, st),
                 "sdtw_stream_best_two: descriptors");
  if (!rc)
    rc = check_hip(launch_best_two(ref->dtype, sl.dev, ns, ref->n, window, sl.part, best_cost_dev,
                                   best_end_dev, second_cost_dev, second_end_dev, st),
                   "sdtw_stream_best_two: launch");
  const int rc_ev = check_hip(hipEventRecord(tok->ev, st), "sdtw_stream_best_two: record");
  if (!rc_ev) sl.last = tok;
  if (!rc) rc = rc_ev;
  if (rc) return rc;
  for (int32_t i = 0; i < ns; ++i) streams[i]->last = tok;  // close waits for the read
  return SDTW_OK;
}

}  // extern "C"

