/*
 * CPU oracle for subsequence DTW (sDTW) as used by signal-level Read Until
 * (HARU, arXiv 2211.07340).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * Everything here is plain, sequential and slow on purpose: one loop nest
 * per definition, no blocking, no vectorisation, no reordering.  Build with
 * -O2 -ffp-contract=off and without -ffast-math (x86-64 SSE arithmetic, one
 * IEEE rounding per operation).
 *
 * Contents
 *   reference preparation   section 4.1 (k-mer model, both strands, z-score,
 *                           fixed-point scaling) and section 2.2 (k-mer model
 *                           lookup over a sliding window of k bases)
 *   query preparation       section 4.1 (z-score per read, same scaling factor
 *                           as the reference)
 *   sDTW                    section 2.3, Eq. 1 with its boundary conditions,
 *                           evaluated column by column with an (M+1) cost
 *                           array as in Algorithm 2 (section 4.3); the three
 *                           neighbour reads of Algorithm 2 are taken in their
 *                           Eq. 1 meaning (see the note above oracle_sdtw_*)
 *   batch drivers           one read per task, dynamic scheduling over
 *                           POSIX threads; used to time the oracle
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Reference preparation (section 4.1, section 2.2)                          */
/* ------------------------------------------------------------------------ */

/*
 * k-mer model conversion of a base sequence into an expected-current signal.
 * Bases are coded A=0, C=1, G=2, T=3.  The k-mer starting at base p has index
 * sum_{m<k} b[p+m] * 4^(k-1-m) (first base most significant) and current
 * table[index].  Both strands are produced, since the molecule is double
 * stranded (section 4.1): out[0 .. L-k] is the forward strand, and
 * out[L-k+1 .. 2(L-k+1)-1] is the reverse-complement strand read 5'->3',
 * i.e. the k-mer model applied to revcomp(g).  Output length 2(L-k+1).
 * Returns the output length, or -1 if L < k.
 */
int64_t oracle_kmer_signal(const uint8_t* g, int64_t L, int k,
                           const float* table, float* out) {
  if (L < k || k < 1) return -1;
  int64_t nk = L - k + 1;
  /* forward strand */
  for (int64_t p = 0; p < nk; ++p) {
    int64_t idx = 0;
    for (int m = 0; m < k; ++m) idx = idx * 4 + g[p + m];
    out[p] = table[idx];
  }
  /* reverse complement: rc[q] = 3 - g[L-1-q] */
  for (int64_t p = 0; p < nk; ++p) {
    int64_t idx = 0;
    for (int m = 0; m < k; ++m) {
      int64_t q = p + m;                 /* position in revcomp(g) */
      int base = 3 - (int)g[L - 1 - q];  /* complement of the mirrored base */
      idx = idx * 4 + base;
    }
    out[nk + p] = table[idx];
  }
  return 2 * nk;
}

/*
 * z-score normalisation (sections 4.1): z = (v - mean) / sd with the
 * population standard deviation, statistics accumulated in double in index
 * order, each output rounded once to float.  sd == 0 gives all zeros.
 */
void oracle_znorm(const float* v, int64_t n, float* out) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += (double)v[i];
  double mean = s / (double)n;
  double ss = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double d = (double)v[i] - mean;
    ss += d * d;
  }
  double sd = sqrt(ss / (double)n);
  for (int64_t i = 0; i < n; ++i)
    out[i] = (sd > 0.0) ? (float)(((double)v[i] - mean) / sd) : 0.0f;
}

/*
 * The same z-score split in two: the statistics of v (mean and population
 * sd, accumulated in double in index order), and their application to any
 * values (used for a read that arrives in chunks: every chunk is scaled with
 * the statistics of the read's first chunk).
 */
void oracle_zstats(const float* v, int64_t n, double* mean_sd) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += (double)v[i];
  double mean = s / (double)n;
  double ss = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double d = (double)v[i] - mean;
    ss += d * d;
  }
  mean_sd[0] = mean;
  mean_sd[1] = sqrt(ss / (double)n);
}

void oracle_zapply(const float* v, int64_t n, double mean, double sd, float* out) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = (sd > 0.0) ? (float)(((double)v[i] - mean) / sd) : 0.0f;
}

/*
 * Fixed-point scaling (section 4.1, section 4.3 "fixed-point data
 * representation"): code = saturate_int16(round_half_even(z * scale)), the
 * product taken in double.  Returns the number of saturated values.
 */
int64_t oracle_quantize(const float* z, int64_t n, double scale, int16_t* out) {
  int64_t nsat = 0;
  for (int64_t i = 0; i < n; ++i) {
    double r = nearbyint((double)z[i] * scale); /* default mode: half-even */
    if (r > 32767.0) { r = 32767.0; ++nsat; }
    if (r < -32768.0) { r = -32768.0; ++nsat; }
    out[i] = (int16_t)r;
  }
  return nsat;
}

/* ------------------------------------------------------------------------ */
/* sDTW (section 2.3 Eq. 1; Algorithm 2 of section 4.3)                      */
/* ------------------------------------------------------------------------ */
/*
 * gamma(i,j) = |X[i] - Y[j]| + min(gamma(i-1,j), gamma(i-1,j-1), gamma(i,j-1))
 * for 1<=i<=M, 1<=j<=N, with gamma(0,j) = 0 (free start anywhere in Y) and
 * gamma(i,0) = +inf.  The result is score = min_j gamma(M,j) and the first
 * (smallest) j attaining it (strict '<' scan, as in Algorithms 1 and 2).
 *
 * Evaluation order: column j = 1..N outer, row i = 1..M inner, keeping the
 * single cost array C[0..M] with C[0] = gamma(0, .) = 0 and C[i] holding
 * gamma(i, j-1) before the update of row i and gamma(i, j) after it.  Inside
 * the update: "up" is C[i-1] (already gamma(i-1, j)), "diag" is the value of
 * C[i-1] before its own update in this column (gamma(i-1, j-1); for i=1 it
 * is gamma(0, j-1) = 0), and "left" is C[i] before the update.
 *
 * Returned end index is 0-based: end = j - 1.  `lastrow`, if non-NULL,
 * receives gamma(M, 1..N) (N values).  M >= 1 and N >= 1 are required.
 */

/* exact integer variant on int16 inputs (the paper's fixed-point path,
 * accumulated here in 64 bits so that no overflow is possible) */
void oracle_sdtw_i64(const int16_t* x, int64_t M, const int16_t* y, int64_t N,
                     int64_t* cost, int64_t* end, int64_t* lastrow) {
  const int64_t INF = INT64_MAX;
  int64_t* C = (int64_t*)malloc((size_t)(M + 1) * sizeof(int64_t));
  C[0] = 0;
  for (int64_t i = 1; i <= M; ++i) C[i] = INF;
  int64_t score = INF, pos = -1;
  for (int64_t j = 1; j <= N; ++j) {
    int64_t diag = 0; /* gamma(0, j-1) */
    for (int64_t i = 1; i <= M; ++i) {
      int64_t up = C[i - 1];
      int64_t left = C[i];
      int64_t m = up;
      if (diag < m) m = diag;
      if (left < m) m = left;
      int64_t d = (int64_t)x[i - 1] - (int64_t)y[j - 1];
      if (d < 0) d = -d;
      C[i] = d + m; /* m is finite: up is always finite */
      diag = left;
    }
    if (lastrow) lastrow[j - 1] = C[M];
    if (C[M] < score) { score = C[M]; pos = j; }
  }
  *cost = score;
  *end = pos - 1;
  free(C);
}

/* float variant: every cell rounded as fl(fl(|fl(x - y)|) + min(...)) */
void oracle_sdtw_f32(const float* x, int64_t M, const float* y, int64_t N,
                     float* cost, int64_t* end, float* lastrow) {
  float* C = (float*)malloc((size_t)(M + 1) * sizeof(float));
  C[0] = 0.0f;
  for (int64_t i = 1; i <= M; ++i) C[i] = INFINITY;
  float score = INFINITY;
  int64_t pos = -1;
  for (int64_t j = 1; j <= N; ++j) {
    float diag = 0.0f;
    for (int64_t i = 1; i <= M; ++i) {
      float up = C[i - 1];
      float left = C[i];
      float m = up;
      if (diag < m) m = diag;
      if (left < m) m = left;
      float d = x[i - 1] - y[j - 1];
      d = fabsf(d);
      C[i] = d + m;
      diag = left;
    }
    if (lastrow) lastrow[j - 1] = C[M];
    if (C[M] < score) { score = C[M]; pos = j; }
  }
  *cost = score;
  *end = pos - 1;
  free(C);
}

/* double variant on the same float inputs: the accuracy reference */
void oracle_sdtw_f64(const float* x, int64_t M, const float* y, int64_t N,
                     double* cost, int64_t* end, double* lastrow) {
  double* C = (double*)malloc((size_t)(M + 1) * sizeof(double));
  C[0] = 0.0;
  for (int64_t i = 1; i <= M; ++i) C[i] = INFINITY;
  double score = INFINITY;
  int64_t pos = -1;
  for (int64_t j = 1; j <= N; ++j) {
    double diag = 0.0;
    for (int64_t i = 1; i <= M; ++i) {
      double up = C[i - 1];
      double left = C[i];
      double m = up;
      if (diag < m) m = diag;
      if (left < m) m = left;
      double d = fabs((double)x[i - 1] - (double)y[j - 1]);
      C[i] = d + m;
      diag = left;
    }
    if (lastrow) lastrow[j - 1] = C[M];
    if (C[M] < score) { score = C[M]; pos = j; }
  }
  *cost = score;
  *end = pos - 1;
  free(C);
}

/* ------------------------------------------------------------------------ */
/* Batch drivers: reads are independent; one read per task                   */
/* ------------------------------------------------------------------------ */

enum { ORACLE_I64 = 0, ORACLE_F32 = 1, ORACLE_F64 = 2 };

typedef struct {
  int kind;
  const void* q;          /* int16 or float values, CSR */
  const int64_t* offs;    /* nq + 1 offsets */
  const int64_t* index;   /* optional subset of reads to run (NULL: all) */
  int64_t nrun;
  const void* ref;
  int64_t N;
  double* cost;           /* per read (as double; exact for i64 < 2^53) */
  int64_t* end;
  int64_t next;           /* shared work counter */
  pthread_mutex_t mu;
} batch_job;

static void* batch_worker(void* arg) {
  batch_job* jb = (batch_job*)arg;
  for (;;) {
    pthread_mutex_lock(&jb->mu);
    int64_t t = jb->next++;
    pthread_mutex_unlock(&jb->mu);
    if (t >= jb->nrun) break;
    int64_t r = jb->index ? jb->index[t] : t;
    int64_t a = jb->offs[r], M = jb->offs[r + 1] - jb->offs[r];
    if (jb->kind == ORACLE_I64) {
      int64_t c, e;
      oracle_sdtw_i64((const int16_t*)jb->q + a, M, (const int16_t*)jb->ref,
                      jb->N, &c, &e, NULL);
      jb->cost[t] = (double)c;
      jb->end[t] = e;
    } else if (jb->kind == ORACLE_F32) {
      float c;
      int64_t e;
      oracle_sdtw_f32((const float*)jb->q + a, M, (const float*)jb->ref, jb->N,
                      &c, &e, NULL);
      jb->cost[t] = (double)c;
      jb->end[t] = e;
    } else {
      double c;
      int64_t e;
      oracle_sdtw_f64((const float*)jb->q + a, M, (const float*)jb->ref, jb->N,
                      &c, &e, NULL);
      jb->cost[t] = c;
      jb->end[t] = e;
    }
  }
  return NULL;
}

/*
 * Run `kind` over reads index[0..nrun) (or 0..nrun if index is NULL) with
 * `nthreads` POSIX threads.  Results land in cost[t], end[t] for task t.
 * Returns the number of threads actually started.
 */
int oracle_batch(int kind, const void* q, const int64_t* offs,
                 const int64_t* index, int64_t nrun, const void* ref,
                 int64_t N, int nthreads, double* cost, int64_t* end) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  batch_job jb;
  jb.kind = kind;
  jb.q = q;
  jb.offs = offs;
  jb.index = index;
  jb.nrun = nrun;
  jb.ref = ref;
  jb.N = N;
  jb.cost = cost;
  jb.end = end;
  jb.next = 0;
  pthread_mutex_init(&jb.mu, NULL);
  pthread_t th[256];
  int started = 0;
  for (int t = 0; t < nthreads; ++t)
    if (pthread_create(&th[t], NULL, batch_worker, &jb) == 0) ++started;
  if (started == 0) batch_worker(&jb);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&jb.mu);
  return started ? started : 1;
}
