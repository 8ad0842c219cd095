/*
 * Seeded synthetic sparse tf-idf corpora: the workload generator.
 *
 * This module only produces INPUTS (documents and seed rows).  It holds none of
 * the clustering arithmetic, and both the GPU library and the CPU oracle consume
 * what it writes.  The corpora stand in for the paper's tweet and arXiv-abstract
 * collections (Sec. 4.1), which are not available: documents are bags of
 * Zipf-distributed terms weighted by tf-idf and L2-normalised, as in Sec. 4.1.
 *
 * Recipe (one document d, all randomness from a counter-based stream keyed by
 * (seed, d), so the output does not depend on the thread count):
 *   nnz_d  = clip(round(exp(mu + sigma * Z)), nnz_min, nnz_max), Z ~ N(0,1) by
 *            Box-Muller, mu = ln(nnz_mean) - sigma^2 / 2 (so the unclipped mean
 *            is nnz_mean);
 *   terms  = nnz_d distinct ranks drawn from Zipf(s) over ranks 1..D by inverse
 *            CDF, duplicates rejected and redrawn; term id = rank - 1;
 *   tf     ~ Geometric(p) on {1, 2, ...} per term;
 *   value  = ln(1 + tf) * idf_t,  idf_t = ln((1 + N) / (1 + df_t)) + 1 (> 0);
 *   row    = value / ||value||_2, the norm taken in double, stored as float,
 *            indices ascending within the row.
 *
 * The random stream is SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used in counter mode: the
 * i-th draw of stream `key` is mix64(key + i * 0x9E3779B97F4A7C15).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t key;
  uint64_t ctr;
} stream_t;

static inline stream_t stream_for(uint64_t seed, uint64_t purpose, uint64_t item) {
  stream_t s;
  s.key = mix64(mix64(seed ^ (purpose * GOLDEN)) + item * GOLDEN);
  s.ctr = 0;
  return s;
}

static inline uint64_t next_u64(stream_t *s) {
  s->ctr += 1;
  return mix64(s->key + s->ctr * GOLDEN);
}

/* uniform in the open interval (0, 1), 53 random bits */
static inline double next_u01(stream_t *s) {
  return ((double)(next_u64(s) >> 11) + 0.5) * 0x1.0p-53;
}

enum { PURPOSE_NNZ = 1, PURPOSE_TERMS = 2, PURPOSE_TF = 3, PURPOSE_SEEDROWS = 4 };

static int64_t doc_nnz(uint64_t seed, int64_t d, double mu, double sigma, int64_t lo, int64_t hi) {
  stream_t s = stream_for(seed, PURPOSE_NNZ, (uint64_t)d);
  double u1 = next_u01(&s), u2 = next_u01(&s);
  double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  double v = exp(mu + sigma * z);
  int64_t n = (int64_t)llround(v);
  if (n < lo) n = lo;
  if (n > hi) n = hi;
  return n;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Pass 1: row lengths.  indptr has n_docs + 1 entries.  Returns total nnz. */
int64_t synth_indptr(int64_t n_docs, int32_t n_terms, double nnz_mean, double nnz_sigma,
                     int64_t nnz_min, int64_t nnz_max, uint64_t seed, int64_t *indptr,
                     int32_t nthreads) {
  if (n_docs < 0 || n_terms <= 0 || nnz_min < 1 || nnz_max < nnz_min || nnz_max > n_terms)
    return -1;
  double mu = log(nnz_mean) - 0.5 * nnz_sigma * nnz_sigma;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
  for (int64_t d = 0; d < n_docs; ++d)
    indptr[d + 1] = doc_nnz(seed, d, mu, nnz_sigma, nnz_min, nnz_max);
  indptr[0] = 0;
  for (int64_t d = 0; d < n_docs; ++d) indptr[d + 1] += indptr[d];
  return indptr[n_docs];
}

/* Pass 2: terms and tf-idf values for the rows laid out by synth_indptr. */
int synth_fill(int64_t n_docs, int32_t n_terms, double zipf_s, double tf_p, uint64_t seed,
               const int64_t *indptr, int32_t *indices, float *values, int32_t nthreads) {
  if (n_docs < 0 || n_terms <= 0 || !(tf_p > 0.0 && tf_p < 1.0)) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  /* Zipf CDF over ranks 1..D (unnormalised, monotone). */
  double *cdf = (double *)malloc(sizeof(double) * (size_t)n_terms);
  if (!cdf) return -2;
  double acc = 0.0;
  for (int32_t r = 0; r < n_terms; ++r) {
    acc += pow((double)(r + 1), -zipf_s);
    cdf[r] = acc;
  }
  const double total = acc;
  const double log_q = log(1.0 - tf_p);
  int64_t nnz = indptr[n_docs];
  /* tf is kept temporarily as ln(1 + tf) in values[]. */
  int err = 0;
#pragma omp parallel
  {
    uint8_t *seen = (uint8_t *)calloc((size_t)n_terms, 1);
    if (!seen) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for schedule(dynamic, 256)
    for (int64_t d = 0; d < n_docs; ++d) {
      if (!seen) continue;
      int64_t b = indptr[d], n = indptr[d + 1] - b;
      stream_t st = stream_for(seed, PURPOSE_TERMS, (uint64_t)d);
      int64_t got = 0;
      while (got < n) {
        double u = next_u01(&st) * total;
        /* first rank whose cumulative weight reaches u */
        int32_t lo = 0, hi = n_terms - 1;
        while (lo < hi) {
          int32_t mid = lo + (hi - lo) / 2;
          if (cdf[mid] >= u) hi = mid; else lo = mid + 1;
        }
        if (seen[lo]) continue;
        seen[lo] = 1;
        indices[b + got] = lo;
        ++got;
      }
      qsort(indices + b, (size_t)n, sizeof(int32_t), cmp_i32);
      stream_t tfs = stream_for(seed, PURPOSE_TF, (uint64_t)d);
      for (int64_t q = 0; q < n; ++q) {
        seen[indices[b + q]] = 0;
        double u = next_u01(&tfs);
        double tf = 1.0 + floor(log(u) / log_q);
        values[b + q] = (float)log1p(tf);
      }
    }
    free(seen);
  }
  if (err) { free(cdf); return -2; }
  /* document frequencies (integer, so independent of the thread split) */
  int64_t *df = (int64_t *)calloc((size_t)n_terms, sizeof(int64_t));
  if (!df) { free(cdf); return -2; }
  for (int64_t q = 0; q < nnz; ++q) df[indices[q]] += 1;
  double *idf = (double *)malloc(sizeof(double) * (size_t)n_terms);
  if (!idf) { free(cdf); free(df); return -2; }
  for (int32_t t = 0; t < n_terms; ++t)
    idf[t] = log((1.0 + (double)n_docs) / (1.0 + (double)df[t])) + 1.0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t d = 0; d < n_docs; ++d) {
    int64_t b = indptr[d], e = indptr[d + 1];
    double ss = 0.0;
    for (int64_t q = b; q < e; ++q) {
      double v = (double)values[q] * idf[indices[q]];
      ss += v * v;
    }
    double inv = 1.0 / sqrt(ss);
    for (int64_t q = b; q < e; ++q) {
      double v = (double)values[q] * idf[indices[q]];
      values[q] = (float)(v * inv);
    }
  }
  free(cdf);
  free(df);
  free(idf);
  return 0;
}

/*
 * Topic-structured variant (the paper's collections have topical structure that
 * iid Zipf draws lack).  Terms [0, n_shared) are a shared vocabulary; the rest
 * is split into n_topics equal blocks.  Row d picks a topic uniformly; each of
 * its terms is drawn, with probability shared_frac, from Zipf(s) over the
 * shared vocabulary, otherwise from Zipf(s) over its topic's block.  Weights,
 * idf and normalisation as in synth_fill.
 */
int synth_topic_fill(int64_t n_docs, int32_t n_terms, int32_t n_topics, int32_t n_shared,
                     double shared_frac, double zipf_s, double tf_p, uint64_t seed,
                     const int64_t *indptr, int32_t *indices, float *values, int32_t nthreads) {
  if (n_docs < 0 || n_topics < 1 || n_shared < 1 || n_shared >= n_terms) return -1;
  const int32_t block = (n_terms - n_shared) / n_topics;
  if (block < 1) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  const int32_t nmax = n_shared > block ? n_shared : block;
  double *cdf = (double *)malloc(sizeof(double) * (size_t)nmax);
  if (!cdf) return -2;
  double acc = 0.0;
  for (int32_t r = 0; r < nmax; ++r) {
    acc += pow((double)(r + 1), -zipf_s);
    cdf[r] = acc;
  }
  const double log_q = log(1.0 - tf_p);
  int err = 0;
#pragma omp parallel
  {
    uint8_t *seen = (uint8_t *)calloc((size_t)n_terms, 1);
    if (!seen) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for schedule(dynamic, 256)
    for (int64_t d = 0; d < n_docs; ++d) {
      if (!seen) continue;
      int64_t b = indptr[d], n = indptr[d + 1] - b;
      stream_t st = stream_for(seed, PURPOSE_TERMS, (uint64_t)d);
      const int32_t topic = (int32_t)(next_u01(&st) * n_topics) % n_topics;
      int64_t got = 0, tries = 0;
      while (got < n) {
        const double us = next_u01(&st);
        /* after many rejections alternate between the two pools so both can fill */
        const int shared = tries > 64 * n ? (int)(tries & 1) : us < shared_frac;
        const int32_t size = shared ? n_shared : block;
        const double u = next_u01(&st) * cdf[size - 1];
        int32_t lo = 0, hi = size - 1;
        while (lo < hi) {
          int32_t mid = lo + (hi - lo) / 2;
          if (cdf[mid] >= u) hi = mid; else lo = mid + 1;
        }
        const int32_t t = shared ? lo : n_shared + topic * block + lo;
        ++tries;
        if (seen[t]) continue;
        seen[t] = 1;
        indices[b + got] = t;
        ++got;
      }
      qsort(indices + b, (size_t)n, sizeof(int32_t), cmp_i32);
      stream_t tfs = stream_for(seed, PURPOSE_TF, (uint64_t)d);
      for (int64_t q = 0; q < n; ++q) {
        seen[indices[b + q]] = 0;
        double u = next_u01(&tfs);
        double tf = 1.0 + floor(log(u) / log_q);
        values[b + q] = (float)log1p(tf);
      }
    }
    free(seen);
  }
  free(cdf);
  if (err) return -2;
  int64_t nnz = indptr[n_docs];
  int64_t *df = (int64_t *)calloc((size_t)n_terms, sizeof(int64_t));
  double *idf = (double *)malloc(sizeof(double) * (size_t)n_terms);
  if (!df || !idf) { free(df); free(idf); return -2; }
  for (int64_t q = 0; q < nnz; ++q) df[indices[q]] += 1;
  for (int32_t t = 0; t < n_terms; ++t)
    idf[t] = log((1.0 + (double)n_docs) / (1.0 + (double)df[t])) + 1.0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t d = 0; d < n_docs; ++d) {
    int64_t b = indptr[d], e = indptr[d + 1];
    double ss = 0.0;
    for (int64_t q = b; q < e; ++q) {
      double v = (double)values[q] * idf[indices[q]];
      ss += v * v;
    }
    double inv = 1.0 / sqrt(ss);
    for (int64_t q = b; q < e; ++q) values[q] = (float)((double)values[q] * idf[indices[q]] * inv);
  }
  free(df);
  free(idf);
  return 0;
}

/* k distinct document ids, uniform, in draw order. */
int synth_seed_rows(int64_t n_docs, int32_t k, uint64_t seed, int32_t *out) {
  if (k < 0 || (int64_t)k > n_docs) return -1;
  uint8_t *taken = (uint8_t *)calloc((size_t)(n_docs > 0 ? n_docs : 1), 1);
  if (!taken) return -2;
  stream_t s = stream_for(seed, PURPOSE_SEEDROWS, 0);
  int32_t got = 0;
  while (got < k) {
    int64_t d = (int64_t)(next_u01(&s) * (double)n_docs);
    if (d >= n_docs) d = n_docs - 1;
    if (taken[d]) continue;
    taken[d] = 1;
    out[got++] = (int32_t)d;
  }
  free(taken);
  return 0;
}

/* Raw access to the stream, for tests of the generator itself. */
void synth_stream_u64(uint64_t seed, uint64_t purpose, uint64_t item, int64_t n, uint64_t *out) {
  stream_t s = stream_for(seed, purpose, item);
  for (int64_t i = 0; i < n; ++i) out[i] = next_u64(&s);
}
