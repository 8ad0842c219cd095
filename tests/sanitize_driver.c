/*
 * Host memory-safety check of the CPU oracle and the input generator: a small
 * end-to-end run (generate, seed, assign, update, k-means++, topic corpus)
 * built together with oracle.c and synth.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Exit status 0
 * and no sanitizer report is a pass.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t synth_indptr(int64_t n_docs, int32_t n_terms, double nnz_mean, double nnz_sigma,
                     int64_t nnz_min, int64_t nnz_max, uint64_t seed, int64_t *indptr,
                     int32_t nthreads);
int synth_fill(int64_t n_docs, int32_t n_terms, double zipf_s, double tf_p, uint64_t seed,
               const int64_t *indptr, int32_t *indices, float *values, int32_t nthreads);
int synth_topic_fill(int64_t n_docs, int32_t n_terms, int32_t n_topics, int32_t n_shared,
                     double shared_frac, double zipf_s, double tf_p, uint64_t seed,
                     const int64_t *indptr, int32_t *indices, float *values, int32_t nthreads);
int synth_seed_rows(int64_t n_docs, int32_t k, uint64_t seed, int32_t *out);
void synth_stream_u64(uint64_t seed, uint64_t purpose, uint64_t item, int64_t n, uint64_t *out);
int orc_seed(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
             const float *values, int32_t k, const int32_t *rows, double *C);
int orc_assign(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
               const float *values, int32_t k, const double *C, const int64_t *docs,
               int64_t n_list, int32_t *a, double *s1, double *s2, int32_t nthreads);
int orc_assign_seeds(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
                     const float *values, int32_t k, const int32_t *rows, const int64_t *docs,
                     int64_t n_list, int32_t *a, double *s1, double *s2, int32_t nthreads);
int orc_update(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
               const float *values, int32_t k, const int32_t *a, const double *C_old,
               double *C_new, int64_t *counts, double *snorm, double *shift_sq,
               double *dot_old);
int orc_kmeanspp(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
                 const float *values, int32_t k, const uint64_t *draws, int32_t *rows_out);

#define CHECK(x)                                          \
  do {                                                    \
    if (!(x)) {                                           \
      fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
      return 1;                                           \
    }                                                     \
  } while (0)

int main(void) {
  const int64_t n = 700;
  const int32_t D = 3000, k = 23;
  int64_t *ip = malloc(sizeof(int64_t) * (n + 1));
  CHECK(ip);
  const int64_t z = synth_indptr(n, D, 25.0, 0.6, 1, 200, 11, ip, 2);
  CHECK(z > 0);
  int32_t *ix = malloc(sizeof(int32_t) * z);
  float *v = malloc(sizeof(float) * z);
  CHECK(ix && v);
  CHECK(synth_fill(n, D, 1.1, 0.6, 11, ip, ix, v, 2) == 0);

  int32_t *rows = malloc(sizeof(int32_t) * k);
  CHECK(synth_seed_rows(n, k, 3, rows) == 0);
  double *C = malloc(sizeof(double) * k * D), *C2 = malloc(sizeof(double) * k * D);
  int32_t *a = malloc(sizeof(int32_t) * n);
  double *s1 = malloc(sizeof(double) * n), *s2 = malloc(sizeof(double) * n);
  int64_t *counts = malloc(sizeof(int64_t) * k);
  double *snorm = malloc(sizeof(double) * k), *shift = malloc(sizeof(double) * k),
         *dot_old = malloc(sizeof(double) * k);
  CHECK(C && C2 && a && s1 && s2 && counts && snorm && shift && dot_old);
  CHECK(orc_seed(n, D, ip, ix, v, k, rows, C) == 0);
  CHECK(orc_assign_seeds(n, D, ip, ix, v, k, rows, NULL, 0, a, s1, s2, 2) == 0);
  for (int it = 0; it < 4; ++it) {
    CHECK(orc_assign(n, D, ip, ix, v, k, C, NULL, 0, a, s1, s2, 2) == 0);
    CHECK(orc_update(n, D, ip, ix, v, k, a, C, C2, counts, snorm, shift, dot_old) == 0);
    double *t = C;
    C = C2;
    C2 = t;
  }
  uint64_t *draws = malloc(sizeof(uint64_t) * n);
  int32_t *seeds = malloc(sizeof(int32_t) * n);
  CHECK(draws && seeds);
  synth_stream_u64(5, 7, 0, n, draws);
  CHECK(orc_kmeanspp(n, D, ip, ix, v, k, draws, seeds) == 0);
  CHECK(orc_kmeanspp(n, D, ip, ix, v, (int32_t)n, draws, seeds) == 0);   /* every row */
  CHECK(orc_kmeanspp(n, D, ip, ix, v, (int32_t)n + 1, draws, seeds) == -1);

  /* topic-structured rows */
  const int64_t z2 = synth_indptr(n, D, 20.0, 0.5, 1, 100, 12, ip, 1);
  CHECK(z2 > 0);
  int32_t *ix2 = malloc(sizeof(int32_t) * z2);
  float *v2 = malloc(sizeof(float) * z2);
  CHECK(ix2 && v2);
  CHECK(synth_topic_fill(n, D, 6, 300, 0.3, 1.1, 0.6, 12, ip, ix2, v2, 1) == 0);

  free(ix2); free(v2); free(draws); free(seeds); free(ip); free(ix); free(v); free(rows);
  free(C); free(C2); free(a); free(s1); free(s2); free(counts); free(snorm); free(shift);
  free(dot_old);
  puts("sanitized run ok");
  return 0;
}
