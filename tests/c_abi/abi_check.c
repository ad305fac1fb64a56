/*
 * Plain C client of the library's C ABI (include/sdtw.h): no Python, no
 * torch.  Used by tests/test_c_abi.py.
 *
 *   abi_check --version
 *   abi_check DIR   reads DIR/ref.i16 (int16 reference codes), DIR/q.i16
 *                   (int16 query codes, CSR) and DIR/offs.i64 (nq + 1
 *                   offsets); writes DIR/batch.i32 (cost, end per read:
 *                   sdtw_align_batch after sdtw_plan_autotune),
 *                   DIR/stream.i32 (cost, end after each of two chunks of
 *                   read 0: sdtw_stream_open / extend / close) and
 *                   DIR/wide.i32 (cost, end of read 0 over the whole device:
 *                   sdtw_align_one_wide).  With DIR/raw.f32 and
 *                   DIR/raw_offs.i64 present it also writes DIR/events.f32
 *                   and DIR/event_counts.i32 (sdtw_detect_events, trim 50,
 *                   keep 250).
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sdtw.h"

static void* slurp(const char* dir, const char* name, size_t* bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    exit(2);
  }
  fseek(f, 0, SEEK_END);
  long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  void* buf = malloc((size_t)n);
  if (!buf || fread(buf, 1, (size_t)n, f) != (size_t)n) {
    fprintf(stderr, "cannot read %s\n", path);
    exit(2);
  }
  fclose(f);
  *bytes = (size_t)n;
  return buf;
}

static void dump(const char* dir, const char* name, const void* buf, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "wb");
  if (!f || fwrite(buf, 1, bytes, f) != bytes) {
    fprintf(stderr, "cannot write %s\n", path);
    exit(2);
  }
  fclose(f);
}

#define SDTW(call)                                                            \
  do {                                                                        \
    int rc_ = (call);                                                         \
    if (rc_ != SDTW_OK) {                                                     \
      fprintf(stderr, "%s -> %d: %s\n", #call, rc_, sdtw_last_error());      \
      return 1;                                                               \
    }                                                                         \
  } while (0)
#define HIP(call)                                                             \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s -> %s\n", #call, hipGetErrorString(e_));            \
      return 1;                                                               \
    }                                                                         \
  } while (0)

int main(int argc, char** argv) {
  if (argc == 2 && strcmp(argv[1], "--version") == 0) {
    printf("%d\n", sdtw_version());
    return 0;
  }
  if (argc != 2) {
    fprintf(stderr, "usage: abi_check --version | DIR\n");
    return 2;
  }
  const char* dir = argv[1];
  size_t rb, qb, ob;
  int16_t* ref = (int16_t*)slurp(dir, "ref.i16", &rb);
  int16_t* q = (int16_t*)slurp(dir, "q.i16", &qb);
  int64_t* offs = (int64_t*)slurp(dir, "offs.i64", &ob);
  const int64_t n = (int64_t)(rb / 2);
  const int32_t nq = (int32_t)(ob / 8) - 1;

  hipStream_t st;
  HIP(hipStreamCreate(&st));
  sdtw_ref r;
  SDTW(sdtw_load_reference(ref, n, SDTW_I16, 0, st, &r));  /* host input, copied */

  /* batch */
  void* q_dev;
  int32_t *cost_dev, *end_dev;
  HIP(hipMalloc(&q_dev, qb));
  HIP(hipMalloc((void**)&cost_dev, sizeof(int32_t) * (size_t)nq));
  HIP(hipMalloc((void**)&end_dev, sizeof(int32_t) * (size_t)nq));
  HIP(hipMemcpy(q_dev, q, qb, hipMemcpyHostToDevice));
  sdtw_plan plan;
  SDTW(sdtw_plan_create(offs, nq, SDTW_I16, &plan));
  SDTW(sdtw_plan_autotune(r, plan, q_dev, cost_dev, end_dev, 0, st));
  SDTW(sdtw_align_batch(r, plan, q_dev, cost_dev, end_dev, st));
  HIP(hipStreamSynchronize(st));
  int32_t* out = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)nq);
  HIP(hipMemcpy(out, cost_dev, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost));
  HIP(hipMemcpy(out + nq, end_dev, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost));
  dump(dir, "batch.i32", out, sizeof(int32_t) * 2 * (size_t)nq);

  /* stream: read 0 in two chunks */
  sdtw_stream s;
  SDTW(sdtw_stream_open(r, &s));
  const int64_t m0 = offs[1] - offs[0];
  const int64_t cut = m0 / 3 > 0 ? m0 / 3 : 1;
  int32_t res[4];
  const int64_t chunks[2][2] = {{0, cut}, {cut, m0}};
  for (int k = 0; k < 2; ++k) {
    const int64_t len = chunks[k][1] - chunks[k][0];
    if (len <= 0) {
      res[2 * k] = res[2 * k + 1] = -1;
      continue;
    }
    const int64_t co[2] = {0, len};
    SDTW(sdtw_stream_extend(&s, 1, (const int16_t*)q_dev + offs[0] + chunks[k][0], co, cost_dev,
                            end_dev, st));
    HIP(hipStreamSynchronize(st));
    HIP(hipMemcpy(&res[2 * k], cost_dev, sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP(hipMemcpy(&res[2 * k + 1], end_dev, sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  SDTW(sdtw_stream_close(s));
  dump(dir, "stream.i32", res, sizeof res);

  /* read 0 over the whole device */
  int32_t wide[2];
  SDTW(sdtw_align_one_wide(r, q_dev, (int32_t)m0, 0, cost_dev, end_dev, st));
  HIP(hipStreamSynchronize(st));
  HIP(hipMemcpy(&wide[0], cost_dev, sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP(hipMemcpy(&wide[1], end_dev, sizeof(int32_t), hipMemcpyDeviceToHost));
  dump(dir, "wide.i32", wide, sizeof wide);

  /* event detection on raw samples, when given */
  char rawpath[4096];
  snprintf(rawpath, sizeof rawpath, "%s/raw.f32", dir);
  FILE* probe = fopen(rawpath, "rb");
  if (probe) {
    fclose(probe);
    size_t xb, xob;
    float* x = (float*)slurp(dir, "raw.f32", &xb);
    int64_t* xo = (int64_t*)slurp(dir, "raw_offs.i64", &xob);
    const int32_t nr = (int32_t)(xob / 8) - 1;
    const int32_t keep = 250;
    void *x_dev, *xo_dev, *ev_dev, *cnt_dev;
    HIP(hipMalloc(&x_dev, xb));
    HIP(hipMalloc(&xo_dev, xob));
    HIP(hipMalloc(&ev_dev, sizeof(float) * (size_t)nr * keep));
    HIP(hipMalloc(&cnt_dev, sizeof(int32_t) * (size_t)nr));
    HIP(hipMemcpy(x_dev, x, xb, hipMemcpyHostToDevice));
    HIP(hipMemcpy(xo_dev, xo, xob, hipMemcpyHostToDevice));
    SDTW(sdtw_detect_events((const float*)x_dev, (const int64_t*)xo_dev, nr, 50, keep,
                            (float*)ev_dev, (int32_t*)cnt_dev, st));
    HIP(hipStreamSynchronize(st));
    float* ev = (float*)malloc(sizeof(float) * (size_t)nr * keep);
    int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)nr);
    HIP(hipMemcpy(ev, ev_dev, sizeof(float) * (size_t)nr * keep, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(cnt, cnt_dev, sizeof(int32_t) * (size_t)nr, hipMemcpyDeviceToHost));
    dump(dir, "events.f32", ev, sizeof(float) * (size_t)nr * keep);
    dump(dir, "event_counts.i32", cnt, sizeof(int32_t) * (size_t)nr);
    HIP(hipFree(x_dev));
    HIP(hipFree(xo_dev));
    HIP(hipFree(ev_dev));
    HIP(hipFree(cnt_dev));
    free(ev);
    free(cnt);
    free(x);
    free(xo);
  }

  SDTW(sdtw_plan_destroy(plan));
  SDTW(sdtw_free_reference(r));
  HIP(hipFree(q_dev));
  HIP(hipFree(cost_dev));
  HIP(hipFree(end_dev));
  HIP(hipStreamDestroy(st));
  free(out);
  free(ref);
  free(q);
  free(offs);
  printf("ok %d reads\n", nq);
  return 0;
}
