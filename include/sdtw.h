/*
 * sdtw.h -- C ABI of the MI355X (gfx950) subsequence-DTW library.
 *
 * What it computes.  For a query X[1..M] (a read's normalised events) and a
 * reference Y[1..N] (the expected current of a genome, forward strand
 * followed by the reverse-complement strand), the sDTW cost
 *
 *     gamma(i,j) = |X[i] - Y[j]| + min(gamma(i-1,j), gamma(i-1,j-1), gamma(i,j-1))
 *     gamma(0,j) = 0,  gamma(i,0) = +inf
 *
 * (section 2.3, Eq. 1 and its boundary conditions: free start and free end
 * in the reference, Manhattan distance), and returns per read
 *
 *     cost = min_j gamma(M,j)     end = (first j attaining it) - 1   (0-based)
 *
 * which is the (score, position) pair that Algorithms 1 and 2 return
 * (sections 2.3 and 4.3); the start position / warp path is not computed,
 * as in section 4.3 (only two cost columns are kept).
 *
 * Number formats.  SDTW_I16: int16 inputs (the fixed-point scaling of
 * section 4.1 / section 4.3), exact 32-bit accumulation, int32 costs in
 * input units.  SDTW_F32: float32 inputs, each cell rounded as
 * fl(|fl(x - y)| + min(...)), float32 costs.  Results never depend on launch
 * configuration, batch composition or tiling: they are bit-identical to a
 * sequential evaluation of Eq. 1 in the same number format.
 *
 * Conventions.
 *   - Every call returns an sdtw_status.  On a non-OK return nothing was
 *     launched and no output was written; sdtw_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread).
 *   - "*_dev" pointers are device memory owned by the caller (for example
 *     torch tensors).  They must stay valid until the enqueued work on
 *     `stream` has completed.  "*_host" pointers are host memory read
 *     synchronously before the call returns.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call that launches work is asynchronous on that stream.
 *   - Device faults surface as SDTW_EDEVICE from the call that observes them.
 *   - Objects (sdtw_ref, sdtw_plan, sdtw_stream) belong to the device that
 *     was current when they were created; use them with that device current.
 */
#ifndef SDTW_H
#define SDTW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdtw_ref_s* sdtw_ref;       /* device copy of a reference signal */
typedef struct sdtw_plan_s* sdtw_plan;     /* validated, scheduled batch layout */
typedef struct sdtw_stream_s* sdtw_stream; /* one read extended chunk by chunk  */

enum sdtw_dtype {
  SDTW_F32 = 0, /* float32 inputs, float32 costs                     */
  SDTW_I16 = 1  /* int16 inputs, 32-bit accumulation, int32 costs    */
};

enum sdtw_status {
  SDTW_OK = 0,
  SDTW_EINVAL = 1,  /* bad argument (null pointer, size, dtype, ...)      */
  SDTW_ENOMEM = 2,  /* device allocation failed                           */
  SDTW_EBUDGET = 3, /* resident-row pool budget exhausted                 */
  SDTW_EDEVICE = 4, /* HIP runtime / kernel error                         */
  SDTW_ESTATE = 5   /* object in the wrong state (closed, still in use)   */
};

/* Largest query length accepted by sdtw_plan_create (rows per read). */
#define SDTW_MAX_QUERY 4096

/* Message for the last non-OK status returned on this thread. */
const char* sdtw_last_error(void);

/* Library ABI version (increments on incompatible changes). */
int sdtw_version(void);

/* ------------------------------------------------------------------------ */
/* Preparation (section 4.1; section 2.2 k-mer model)                        */
/* ------------------------------------------------------------------------ */

/*
 * Reference preparation, once per reference (section 4.1: the k-mer model
 * turns the base reference into a synthetic signal for the forward and the
 * reverse strand, which is z-score normalised and scaled to fixed point;
 * section 2.2: a window of k bases slides over the sequence and each k-mer is
 * looked up in the model).
 *
 *   genome_dev  uint8[L], bases coded A=0 C=1 G=2 T=3 (the low two bits of
 *               each byte are used; other bits are ignored, not checked).
 *   L           genome length, L >= k.
 *   table_dev   float32[4^k] expected current per k-mer; k-mer index is
 *               sum_m b[m] 4^(k-1-m), first base most significant.
 *   k           1 <= k <= 12.
 *   scale       fixed-point scaling factor (> 0), e.g. 64.
 *   z_dev       out float32[2(L-k+1)]: forward strand k-mers 0..L-k, then
 *               the reverse-complement strand read 5'->3', jointly z-scored
 *               (mean and population standard deviation of the whole
 *               concatenation, each sum accumulated in double in index
 *               order, so the statistics equal a plain sequential loop's
 *               bit for bit; sd == 0 gives zeros).
 *   codes_dev   out int16[2(L-k+1)] or NULL: saturate(rint(z * scale)), the
 *               product and rounding in double, round-half-even.
 *   nsat_dev    out int64[1] or NULL: number of saturated codes.
 */
int sdtw_prepare_reference(const uint8_t* genome_dev, int64_t L,
                           const float* table_dev, int k, double scale,
                           float* z_dev, int16_t* codes_dev, int64_t* nsat_dev,
                           void* stream);

/*
 * Query preparation, per read (section 4.1: each read's events are
 * normalised and scaled with the same factor as the reference).
 *
 *   raw_dev       float32 events of all reads, concatenated (CSR).
 *   offsets_dev   int64[nq+1] on the device, read r is
 *                 raw[offsets[r] .. offsets[r+1]).  A read whose end is not
 *                 after its start is empty and produces nothing (the offsets
 *                 are not otherwise checked: they must lie inside raw/z).
 *   nq            >= 1.
 *   z_dev         out float32, same layout: (v - mean_r) / sd_r with the
 *                 read's own mean and population sd, both accumulated in
 *                 double in index order (sd == 0 gives zeros).
 *   codes_dev     out int16 or NULL: saturate(rint(z * scale)) as above.
 *   nsat_dev      out int64[1] or NULL: number of saturated codes (all reads).
 */
int sdtw_prepare_queries(const float* raw_dev, const int64_t* offsets_dev,
                         int32_t nq, double scale, float* z_dev,
                         int16_t* codes_dev, int64_t* nsat_dev, void* stream);

/*
 * sdtw_prepare_queries with explicit statistics, for reads that arrive in
 * chunks: every chunk of a read must be scaled like its first one so that
 * extending a resident row equals aligning the concatenated read.
 *   stats_in_dev   double[2 nq] (mean, sd) per read to apply, or NULL to
 *                  use each read's own statistics as sdtw_prepare_queries.
 *   stats_out_dev  double[2 nq] receiving the (mean, sd) applied, or NULL.
 */
int sdtw_prepare_queries_ex(const float* raw_dev, const int64_t* offsets_dev, int32_t nq,
                            double scale, const double* stats_in_dev, double* stats_out_dev,
                            float* z_dev, int16_t* codes_dev, int64_t* nsat_dev, void* stream);

/*
 * Event detection (section 4.1: raw samples are cut into events before
 * normalisation; section 5.2: the R9.4 parameters of the f5c / nanopolish
 * two-window t-test detector).  Per read: t statistics over windows of 3
 * and 6 samples, a short (threshold 1.4) and a long (threshold 9.0) peak
 * detector with peak height 0.2 give the event boundaries; an event's value
 * is the float32 rounding of the float64 mean of its samples.  The first
 * `trim` events (the adaptor) are dropped and the next `keep` written.
 *   raw_dev      float32 samples in pA (device), reads concatenated.
 *   offsets_dev  int64[nreads + 1] (device): read r is
 *                raw_dev[offsets[r] .. offsets[r+1]).
 *   trim, keep   trim >= 0, 1 <= keep <= SDTW_MAX_QUERY, trim + keep <= 6144.
 *   events_dev   out float32[nreads * keep]: row r holds read r's events
 *                trim .. trim+counts[r]-1, then zeros.
 *   counts_dev   out int32[nreads]: events written (fewer than keep when
 *                the read has fewer than trim + keep events).
 * A read is scanned only until its first trim + keep boundaries are final.
 * Only a kernel is enqueued (no allocation), so the call may be captured in
 * a hipGraph.  The query for sdtw_prepare_queries is then
 * events_dev with offsets r * keep .. r * keep + counts[r].
 */
int sdtw_detect_events(const float* raw_dev, const int64_t* offsets_dev, int32_t nreads,
                       int32_t trim, int32_t keep, float* events_dev, int32_t* counts_dev,
                       void* stream);

/*
 * Event detection on the samples received so far of reads still being
 * sequenced (Read Until: events are cut from the start of a read while it
 * passes through the pore).  Same detector as sdtw_detect_events; only
 * events that more samples cannot change are written: the scan stops 5
 * samples before the end (the t statistics there still depend on samples
 * to come) and an event is written only if its end boundary is final.
 * Events written for a prefix are the same as those of the whole read.
 *   ranges_dev   int64[2 * nreads] (device): read r's samples so far are
 *                raw_dev[ranges[2r] .. ranges[2r+1]).
 *   firsts_dev   int32[nreads] (device): index of the first event wanted
 *                (adaptor events plus events already taken), 0 <= first <=
 *                max_first; a read outside that range gets count -1.
 *   max_first, keep   0 <= max_first, 1 <= keep <= SDTW_MAX_QUERY,
 *                max_first + keep <= 6144.
 *   events_dev   out float32[nreads * keep]: read r's events first ..
 *                first + counts[r] - 1, then zeros.
 *   counts_dev   out int32[nreads]: events written (0 .. keep).
 * Only a kernel is enqueued (no allocation).
 */
int sdtw_detect_events_prefix(const float* raw_dev, const int64_t* ranges_dev,
                              const int32_t* firsts_dev, int32_t nreads, int32_t max_first,
                              int32_t keep, float* events_dev, int32_t* counts_dev,
                              void* stream);

/*
 * Event detection for reads received chunk by chunk, scanning each sample
 * once: the detectors' state of every read is kept between calls in
 * caller-owned device memory (sdtw_event_state_bytes() per read).  Events
 * are delivered in order as soon as they are final (later samples cannot
 * change them), and are the same as sdtw_detect_events on the whole read.
 *   sdtw_event_state_init: resets states_dev slots slots_dev[0 .. n) (a
 *     kernel; call it when a read starts on a slot, in order on `stream`).
 *   sdtw_detect_events_continue:
 *     ranges_dev  int64[2 * nreads]: read r's samples so far are
 *                 raw_dev[ranges[2r] .. ranges[2r+1]); the start stays the
 *                 same from call to call, the end only grows.
 *     slots_dev   int32[nreads]: read r's state is slot slots[r] of
 *                 states_dev; distinct within a call.
 *     trim        the read's first `trim` events (the adaptor) are consumed
 *                 and not written.
 *     keep        at most keep events written per read and call (1 <= keep
 *                 <= SDTW_MAX_QUERY); the rest stay for the next call.
 *     events_dev  out float32[nreads * keep]: the read's next counts[r]
 *                 events, then zeros.
 *     counts_dev  out int32[nreads]; -1 if more than 32 boundaries were
 *                 waiting to be delivered (keep too small for the samples
 *                 given): the read's state is then unusable.
 * Only kernels are enqueued (no allocation).
 */
int64_t sdtw_event_state_bytes(void);
int sdtw_event_state_init(void* states_dev, const int32_t* slots_dev, int32_t n, void* stream);
int sdtw_detect_events_continue(const float* raw_dev, const int64_t* ranges_dev,
                                const int32_t* slots_dev, void* states_dev, int32_t nreads,
                                int32_t trim, int32_t keep, float* events_dev,
                                int32_t* counts_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Reference handle                                                          */
/* ------------------------------------------------------------------------ */

/*
 * Copy a prepared reference signal into library-owned device memory, laid
 * out for the alignment kernels (section 4.3 keeps the reference resident
 * and streams it past the processing elements; here it stays in HBM).
 *
 *   ref        int16[n] (SDTW_I16) or float32[n] (SDTW_F32) values.
 *   ref_is_device  1 if `ref` is device memory, 0 if host memory.
 *   n          >= 1.  Float values must be finite (checked; EINVAL).
 *   out        receives the handle.  The call synchronises `stream`; the
 *              caller may free `ref` when it returns.
 */
int sdtw_load_reference(const void* ref, int64_t n, int dtype,
                        int ref_is_device, void* stream, sdtw_ref* out);

/* Length and dtype of a loaded reference. */
int sdtw_reference_info(sdtw_ref ref, int64_t* n, int* dtype);

/* Release a reference.  ESTATE while streams opened on it are still open. */
int sdtw_free_reference(sdtw_ref ref);

/* ------------------------------------------------------------------------ */
/* Batched alignment (sections 2.3 / 4.3; many query processors, section 7)  */
/* ------------------------------------------------------------------------ */

/*
 * Validate and schedule a batch layout once; reuse it for every batch with
 * the same read lengths.  Reads are ordered longest first and pulled by a
 * persistent grid (one launch per group of reads that share a kernel
 * configuration); reads of 64 rows or fewer go to the one-wave kernel.
 *
 *   offsets_host  int64[nq+1] CSR offsets of the query values, read r is
 *                 q[offsets[r] .. offsets[r+1]); every read 1 <= M <=
 *                 SDTW_MAX_QUERY (EINVAL otherwise).
 *   nq            >= 1.
 *   dtype         SDTW_F32 or SDTW_I16 (the query dtype of later calls).
 *   out           receives the plan (device memory is allocated here).
 */
int sdtw_plan_create(const int64_t* offsets_host, int32_t nq, int dtype,
                     sdtw_plan* out);

/* Number of reads and dtype of a plan. */
int sdtw_plan_info(sdtw_plan plan, int32_t* nq, int* dtype, int32_t* max_m);

/*
 * Override the kernel configuration chosen for a plan (autotuning).  Results
 * never depend on it.
 *   strip   columns per lane: 8, 16 or 32 (0 = keep).
 *   chains  independent dependency chains per lane for long reads: 1, 2 or
 *           4 (0 = keep); strip / chains must be a multiple of 4.  Reads
 *           with M >= 64 * chains + 1 use that many; shorter reads fall back
 *           to fewer chains, and reads with M <= 64 to the one-wave kernel.
 *   bands   waves per read: 1 to 4 (0 = keep the plan's where they fit the
 *           other settings, else 1); 2 or 4 need strip 16 with at most 2
 *           chains or strip 32 with 1 chain (2 also strip 32 with 2
 *           chains), 3 needs strip 16 or 32 with 1 chain.  A read's rows are
 *           cut into
 *           up to `bands` row bands of at least 64 * chains + 1 rows each
 *           (Eq. 1: a row depends on the rows above only through the
 *           previous row), one wave per band, pipelined over the
 *           reference tiles.
 *   waves_per_cu  resident waves per compute unit for the persistent grid,
 *           1..32 (0 = keep); a multiple of bands.
 *   band_rows  target rows per band: each read gets about M / band_rows
 *           bands (rounded to nearest, at least 1, at most `bands` and at
 *           most M / (64 * chains + 1)), so that reads of different lengths
 *           finish together; 0 = as many bands as fit; -1 = keep.  Otherwise
 *           >= 65.
 * EINVAL for values outside these sets.
 */
int sdtw_plan_set_config(sdtw_plan plan, int strip, int chains, int bands, int waves_per_cu,
                         int32_t band_rows);
int sdtw_plan_get_config(sdtw_plan plan, int* strip, int* chains, int* bands,
                         int* waves_per_cu, int32_t* band_rows);

/*
 * Autotune the plan's kernel configuration on this batch: run every
 * candidate (strip 16 or 32, 1 or 2 chains, 1 to 4 bands where valid,
 * with 3 or 4 bands also band_rows targets of a half and a third of the
 * median read, each at the waves per CU its LDS allows and at half that)
 * in two passes (the second in reverse order), each a warm-up launch and one
 * timed with HIP events on `stream`; keep the candidate with the fastest of
 * its two times on the plan
 * and remember it for sdtw_plan_use_tuned, keyed by the device's
 * architecture and compute units, the dtype, the reference length and the
 * batch's shape class (number of reads, median and longest read length,
 * each in quarter-octave buckets: round(4 log2 v)).  If the environment
 * variable SDTW_TUNE_CACHE names a file, tuned shapes are also written there
 * (one per line, the file rewritten after every autotune) and read back by
 * the first sdtw_plan_autotune or sdtw_plan_use_tuned of a process.
 *   max_columns  time the candidates on the first min(n, max_columns)
 *                reference columns (0 = all); the ranking does not depend on
 *                the reference length beyond the first few tiles.
 * cost_dev / end_dev receive intermediate results (scratch).  Synchronises
 * `stream`; allocates nothing on the device.  Results of later calls never
 * depend on the configuration chosen.
 */
int sdtw_plan_autotune(sdtw_ref ref, sdtw_plan plan, const void* q_dev, void* cost_dev,
                       int32_t* end_dev, int64_t max_columns, void* stream);

/*
 * Apply a configuration sdtw_plan_autotune found earlier (in this process,
 * or in the SDTW_TUNE_CACHE file) for a batch of the same shape class against
 * a reference of the same length on the same kind of device; *found
 * (optional) is set to 1 if there was one, else 0 and the plan is unchanged.
 */
int sdtw_plan_use_tuned(sdtw_ref ref, sdtw_plan plan, int* found);

/* Release a plan (synchronise the streams that used it first). */
int sdtw_plan_destroy(sdtw_plan plan);

/*
 * Align every read of the plan against the reference.
 *
 *   q_dev     query values in the plan's layout: int16 (SDTW_I16) or float32
 *             (SDTW_F32); the plan's dtype must equal the reference's.
 *   cost_dev  out int32[nq] (SDTW_I16) or float32[nq] (SDTW_F32).
 *   end_dev   out int32[nq], 0-based end column in the reference.
 *
 * Only kernels are enqueued (no allocation, no host synchronisation), so the
 * call may be captured in a hipGraph.  Two calls with the same plan must not
 * overlap in time (the plan holds the work-pull and placement words the
 * launch clears and uses).  Where the launch runs (which SIMD a workgroup
 * lands on) decides which reads share a SIMD and their issue priority, never
 * the results.
 */
int sdtw_align_batch(sdtw_ref ref, sdtw_plan plan, const void* q_dev,
                     void* cost_dev, int32_t* end_dev, void* stream);

/*
 * One read per launch with the single-wave kernel (the plain baseline the
 * batched engine is measured against).  Same semantics as a one-read batch.
 *   q_dev  M values; 1 <= M <= SDTW_MAX_QUERY.
 */
int sdtw_align_one(sdtw_ref ref, const void* q_dev, int32_t M, void* cost_dev,
                   int32_t* end_dev, void* stream);

/*
 * One read spread over every compute unit (int16 references only): each of
 * the M rows of Eq. 1 is computed as a prefix scan over the N columns (a row
 * of the recurrence is a composition of maps x -> min(a, x + d), section 4.3
 * computes the same cells as an oblique wavefront), with tiles of 256 x
 * `cols` columns that pass their boundary values to the right through
 * device-memory flags.  Results equal sdtw_align_one's bit for bit; the
 * latency no longer grows with N / (columns of one workgroup).
 *   q_dev  M int16 values; 1 <= M <= SDTW_MAX_QUERY.
 *   cols   columns per thread, 8, 16, 32 or 64; 0 = the fewest that cut the
 *          reference into at most 64 tiles, else into at most 256, else 32
 *          (the fastest choice measured for each reference length).
 *   cost_dev  out int32[1]; end_dev out int32[1] (0-based column).
 * Enqueues three kernels and records an event that tracks the reuse of its
 * library-owned scratch (8 bytes per tile per row: 8 MiB per call in flight
 * unless more is needed), so the call is not for graph capture.  If a
 * tile waits for its left neighbour for about a second (a defect; never in
 * normal operation) every wait ends and cost and end are -1.
 * EINVAL for a float32 reference.
 */
int sdtw_align_one_wide(sdtw_ref ref, const void* q_dev, int32_t M, int cols, void* cost_dev,
                        int32_t* end_dev, void* stream);

/*
 * sdtw_align_one_wide for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, arguments and results, but the scratch is a
 * fixed array of 2^20 64-bit words (8 MiB) that the library holds on every
 * device it runs on until the process ends, and the call records no event.
 * It calls no hipMalloc, hipFree or allocating routine; the first call on a
 * device looks the array's address up once.
 *   Limit: wide scratch words = 2 M t + M ceil(t / 64) + t + 1 for t =
 *   ceil(N / (256 cols)) tiles must not exceed 2^20 (EINVAL otherwise, with
 *   the sizes in the message; nothing is launched).  For example M = 250
 *   fits up to about 16 M columns at cols = 32.
 *   Every call on a device shares that device's array, which keeps the last
 *   call's contents (each call clears what it needs itself, with a kernel):
 *   calls that overlap in time on one device race and must be ordered by
 *   the caller (one stream, or events).
 */
int sdtw_align_one_wide_noalloc(sdtw_ref ref, const void* q_dev, int32_t M, int cols,
                                void* cost_dev, int32_t* end_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Streaming extension (Read Until: section 2.2 rejection before most of a   */
/* read is sequenced; section 4.1 reads arrive as the sequencer produces     */
/* them)                                                                     */
/* ------------------------------------------------------------------------ */
/*
 * A stream holds one read's resident DP row gamma(m, 0..N-1) for the m query
 * rows folded in so far (row i depends only on X[1..i], section 2.3 Eq. 1),
 * so extending it by a chunk of k new events computes rows m+1..m+k only,
 * with results identical to aligning the concatenated m+k events from
 * scratch.  Normalisation is the caller's: a read's chunks must be scaled
 * with statistics fixed by its first chunk (see sdtw_prepare_queries_ex).
 *
 * Rows come from a per-device pool with a byte budget; a row is N padded x
 * 4 bytes.  Closed rows are cached for reuse and released when a row of
 * another size needs their room.
 */

/* Byte budget of resident rows on the current device (default 16 GiB). */
int sdtw_set_row_budget(int64_t bytes);
int sdtw_row_budget_info(int64_t* budget, int64_t* in_use, int64_t* cached);

/*
 * Free the rows closed streams left cached on the current device (they are
 * kept for reuse by later sdtw_stream_open calls of the same size and do not
 * count against the budget).  Open streams are not touched.
 */
int sdtw_row_pool_trim(void);

/*
 * Open a stream on `ref` (its dtype applies).  SDTW_EBUDGET when the row
 * would exceed the budget (nothing allocated; retry after closing others),
 * SDTW_ENOMEM when the device allocation fails.  The reference cannot be
 * freed while streams are open on it.
 */
int sdtw_stream_open(sdtw_ref ref, sdtw_stream* out);

/* Rows folded in so far and the reference length. */
int sdtw_stream_info(sdtw_stream s, int32_t* rows, int64_t* n);

/*
 * Close a stream and return its row to the pool.  Waits for enqueued work
 * that uses the row.  The handle is invalid afterwards.
 */
int sdtw_stream_close(sdtw_stream s);

/*
 * Copy the resident row (N values: int32 costs for SDTW_I16, float32 for
 * SDTW_F32) to device memory `dst_dev`, asynchronously on `stream`.
 * SDTW_ESTATE when the stream has no rows yet.
 */
int sdtw_stream_copy_row(sdtw_stream s, void* dst_dev, void* stream);

/*
 * Extend `ns` distinct streams by one chunk each in one launch (continuous
 * batching).  Chunk i is chunk_dev[offsets[i] .. offsets[i+1]) (int16 or
 * float32 values of the reference's dtype), 1 <= length <= SDTW_MAX_QUERY;
 * a stream's total rows stay <= 32,767 on the int16 path.  All streams
 * must share one reference.  Outputs, per stream in call order: the cost
 * and 0-based end of the new last row (as sdtw_align_batch).  A stream's
 * row count advances when the call returns; calls on the same streams must
 * be issued in order on one HIP stream (or ordered by the caller).  Calls
 * on other streams may run at once on other HIP streams: against
 * references of 2^20 columns or more two calls' workgroups share a CU once
 * the calls in flight (the library counts its own) cover more than half
 * the CUs, and take CUs of their own below that.  Placement never changes
 * results.
 */
int sdtw_stream_extend(const sdtw_stream* streams, int32_t ns, const void* chunk_dev,
                       const int64_t* chunk_offsets_host, void* cost_dev, int32_t* end_dev,
                       void* stream);

/*
 * Extend one stream by one chunk over the whole device (section 2.2's
 * per-chunk decision, Eq. 1 continued from the resident row): the chunk's
 * rows as row scans across tiles of 256 x cols columns, as
 * sdtw_align_one_wide does for a whole read, starting from the stream's
 * resident row and writing the new last row back over it.  For a few
 * chunks against a long reference, whose batched extension is bounded by
 * one chunk's four waves, this answers in milliseconds; it uses the whole
 * device per chunk, so batches of many chunks belong to sdtw_stream_extend.
 * The two may extend the same stream in turn (one resident row format).
 *   chunk_dev  M int16 values (device); the stream's rows plus M must stay
 *              <= SDTW_MAX_QUERY (EINVAL otherwise; sdtw_stream_extend
 *              takes longer streams).
 *   cols       columns per thread: 0 (automatic), 8, 16, 32 or 64.
 *   cost_dev, end_dev  one int32 each (device): the new last row's cost and
 *              0-based end, as sdtw_align_batch; -1 and -1 if a wait in the
 *              launch ran out (a defect), the resident row then undefined.
 * int16 references only (EINVAL otherwise).  The stream's row count
 * advances when the call returns; calls on one stream are ordered as for
 * sdtw_stream_extend.
 */
int sdtw_stream_extend_wide(sdtw_stream s, const void* chunk_dev, int32_t M, int cols,
                            void* cost_dev, int32_t* end_dev, void* stream);

/*
 * Best and runner-up ends of the resident rows of `ns` streams on one
 * reference: the two mapped positions and scores a mapping quality is
 * computed from (section 5.1).  best = the first column with the row's
 * minimum (the end the last sdtw_stream_extend returned); second = the first
 * column with the minimum among the columns farther than `window` from best.
 *   window           >= 0 columns.
 *   best_cost_dev, second_cost_dev   out [ns]: int32 (SDTW_I16) or float32
 *                    (SDTW_F32), in stream order.
 *   best_end_dev, second_end_dev     out int32 [ns], 0-based columns.
 * When no column lies outside the window, second is INT32_MAX (int16 path)
 * or +inf, at column -1.  Enqueued on `stream`; order it after the extends
 * that wrote the rows (same stream).  Closing a stream waits for this call.
 * SDTW_ESTATE if a stream has no rows yet; EINVAL if ns times
 * ceil(n / 16384) exceeds INT32_MAX.  Uses library-owned device scratch of
 * 8 bytes per 16,384 columns per row: 8 MiB per call in flight, allocated
 * by the first such call; a call that needs more reallocates, which waits
 * for all work on the device.
 */
int sdtw_stream_best_two(const sdtw_stream* streams, int32_t ns, int32_t window,
                         void* best_cost_dev, int32_t* best_end_dev, void* second_cost_dev,
                         int32_t* second_end_dev, void* stream);

/*
 * Launch shape of later sdtw_stream_extend calls on streams of `ref` (one
 * chain per lane); ref = NULL sets the process default that references
 * without their own setting use.
 *   strip  columns per lane, 16 or 32; 0 (default) = 32 for references of
 *          2^20 columns or more, else 16.
 *   bands  waves per chunk (the row bands of sdtw_plan_set_config), 1 to 4;
 *          0 (default) = 4 for at most two chunks per compute unit, 2 for
 *          at most four, else 1 (a chunk of M rows uses at most M / 65).
 * Results never depend on it.  EINVAL for other values.
 */
int sdtw_stream_set_config(sdtw_ref ref, int strip, int bands);

#ifdef __cplusplus
}
#endif

#endif /* SDTW_H */
