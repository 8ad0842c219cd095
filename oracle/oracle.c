/*
 * CPU FP64 oracle for spherical k-means: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow and direct.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library; the product path
 * never does, and this file shares no code with the GPU library.
 *
 * What it computes (paper Sec. 2):
 *   - every input row is treated as given (stored float values widened exactly
 *     to double; rows are not renormalised);
 *   - a centroid is the sum of its members divided by that sum's length, so it
 *     has unit length;
 *   - each row is assigned to the centroid of highest cosine similarity, which
 *     for unit vectors is the plain dot product.
 * Readings where the paper is silent:
 *   - ties in the argmax go to the lowest centroid index;
 *   - an empty cluster keeps its previous centroid;
 *   - sums run in ascending term order (dot products) and ascending row order
 *     (centroid sums).
 * Centroids are dense k x D row-major arrays of double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Initial centroids: c_j = x_r / ||x_r|| for the given rows r = rows[j]. */
int orc_seed(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
             const float *values, int32_t k, const int32_t *rows, double *C) {
  for (int32_t j = 0; j < k; ++j) {
    int64_t r = rows[j];
    if (r < 0 || r >= n_docs) return -1;
    double *c = C + (size_t)j * (size_t)D;
    memset(c, 0, sizeof(double) * (size_t)D);
    double ss = 0.0;
    for (int64_t q = indptr[r]; q < indptr[r + 1]; ++q) ss += (double)values[q] * (double)values[q];
    double nrm = sqrt(ss);
    for (int64_t q = indptr[r]; q < indptr[r + 1]; ++q) c[indices[q]] = (double)values[q] / nrm;
  }
  return 0;
}

/* Similarity of row i with centroid j: sum over the row's terms, ascending. */
static double dot_row(const int64_t *indptr, const int32_t *indices, const float *values,
                      int64_t i, const double *c) {
  double s = 0.0;
  for (int64_t q = indptr[i]; q < indptr[i + 1]; ++q) s += (double)values[q] * c[indices[q]];
  return s;
}

/*
 * Assignment step.  For each listed row (all rows when docs == NULL):
 *   a[o]  = lowest j attaining max_j s_ij,
 *   s1[o] = that maximum, s2[o] = max over j != a[o] (or -inf when k == 1).
 */
int orc_assign(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
               const float *values, int32_t k, const double *C, const int64_t *docs,
               int64_t n_list, int32_t *a, double *s1, double *s2, int32_t nthreads) {
  (void)D;
  if (k < 1) return -1;
  int64_t n = docs ? n_list : n_docs;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t o = 0; o < n; ++o) {
    int64_t i = docs ? docs[o] : o;
    if (i < 0 || i >= n_docs) { bad = 1; continue; }
    int32_t best = 0;
    double b1 = -INFINITY, b2 = -INFINITY;
    for (int32_t j = 0; j < k; ++j) {
      double s = dot_row(indptr, indices, values, i, C + (size_t)j * (size_t)D);
      if (s > b1) {
        b2 = b1;
        b1 = s;
        best = j;
      } else if (s > b2) {
        b2 = s;
      }
    }
    a[o] = best;
    s1[o] = b1;
    s2[o] = b2;
  }
  return bad ? -1 : 0;
}

/* Dot product of two rows of the CSR by merging their ascending term lists. */
static double dot_rows(const int64_t *indptr, const int32_t *indices, const float *values,
                       int64_t i, int64_t r) {
  int64_t p = indptr[i], pe = indptr[i + 1], q = indptr[r], qe = indptr[r + 1];
  double s = 0.0;
  while (p < pe && q < qe) {
    if (indices[p] < indices[q]) ++p;
    else if (indices[p] > indices[q]) ++q;
    else {
      s += (double)values[p] * (double)values[q];
      ++p;
      ++q;
    }
  }
  return s;
}

/*
 * Assignment against the initial centroids c_j = x_{rows[j]} / ||x_{rows[j]}||
 * without forming them densely (for sampled checks at full size):
 * s_ij = (x_i . x_{rows[j]}) / ||x_{rows[j]}||.  Same outputs as orc_assign.
 */
int orc_assign_seeds(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
                     const float *values, int32_t k, const int32_t *rows, const int64_t *docs,
                     int64_t n_list, int32_t *a, double *s1, double *s2, int32_t nthreads) {
  (void)D;
  if (k < 1) return -1;
  double *nrm = (double *)malloc(sizeof(double) * (size_t)k);
  if (!nrm) return -2;
  for (int32_t j = 0; j < k; ++j) {
    if (rows[j] < 0 || rows[j] >= n_docs) { free(nrm); return -1; }
    nrm[j] = sqrt(dot_rows(indptr, indices, values, rows[j], rows[j]));
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t o = 0; o < n_list; ++o) {
    int64_t i = docs[o];
    if (i < 0 || i >= n_docs) { bad = 1; continue; }
    int32_t best = 0;
    double b1 = -INFINITY, b2 = -INFINITY;
    for (int32_t j = 0; j < k; ++j) {
      double s = dot_rows(indptr, indices, values, i, rows[j]) / nrm[j];
      if (s > b1) {
        b2 = b1;
        b1 = s;
        best = j;
      } else if (s > b2) {
        b2 = s;
      }
    }
    a[o] = best;
    s1[o] = b1;
    s2[o] = b2;
  }
  free(nrm);
  return bad ? -1 : 0;
}

/* Dense similarity matrix S[o][j] for listed rows (small inputs only). */
int orc_scores(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
               const float *values, int32_t k, const double *C, const int64_t *docs,
               int64_t n_list, double *S) {
  int64_t n = docs ? n_list : n_docs;
  for (int64_t o = 0; o < n; ++o) {
    int64_t i = docs ? docs[o] : o;
    if (i < 0 || i >= n_docs) return -1;
    for (int32_t j = 0; j < k; ++j)
      S[o * k + j] = dot_row(indptr, indices, values, i, C + (size_t)j * (size_t)D);
  }
  return 0;
}

/*
 * Update step.  S_j = sum of member rows (ascending row id); for non-empty j,
 * C_new[j] = S_j / ||S_j||, otherwise C_new[j] = C_old[j].
 * Per cluster outputs: counts, snorm = ||S_j||, shift_sq = ||C_new[j] - C_old[j]||^2,
 * dot_old = S_j . C_old[j] (the assignment-step objective of cluster j).
 * C_new must not alias C_old.
 */
int orc_update(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
               const float *values, int32_t k, const int32_t *a, const double *C_old,
               double *C_new, int64_t *counts, double *snorm, double *shift_sq,
               double *dot_old) {
  memset(C_new, 0, sizeof(double) * (size_t)k * (size_t)D);
  memset(counts, 0, sizeof(int64_t) * (size_t)k);
  for (int64_t i = 0; i < n_docs; ++i) {
    int32_t j = a[i];
    if (j < 0 || j >= k) return -1;
    counts[j] += 1;
    double *s = C_new + (size_t)j * (size_t)D;
    for (int64_t q = indptr[i]; q < indptr[i + 1]; ++q) s[indices[q]] += (double)values[q];
  }
  for (int32_t j = 0; j < k; ++j) {
    double *c = C_new + (size_t)j * (size_t)D;
    const double *o = C_old + (size_t)j * (size_t)D;
    double ss = 0.0, dd = 0.0;
    for (int32_t t = 0; t < D; ++t) {
      ss += c[t] * c[t];
      dd += c[t] * o[t];
    }
    dot_old[j] = dd;
    if (counts[j] == 0) {
      memcpy(c, o, sizeof(double) * (size_t)D);
      snorm[j] = 0.0;
      shift_sq[j] = 0.0;
      continue;
    }
    double nrm = sqrt(ss);
    snorm[j] = nrm;
    double sh = 0.0;
    for (int32_t t = 0; t < D; ++t) {
      c[t] = c[t] / nrm;
      double d = c[t] - o[t];
      sh += d * d;
    }
    shift_sq[j] = sh;
  }
  return 0;
}

/*
 * Centroids of selected clusters only, from an assignment: out[o] = S_j / ||S_j||
 * for j = clusters[o] (all-zero row and snorm 0 when the cluster is empty).
 * Used for sampled checks where the full dense k x D array is too large.
 */
int orc_centroid_rows(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
                      const float *values, int32_t k, const int32_t *a,
                      const int32_t *clusters, int32_t n_sel, double *out, double *snorm) {
  int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
  if (!slot) return -2;
  for (int32_t j = 0; j < k; ++j) slot[j] = -1;
  for (int32_t o = 0; o < n_sel; ++o) {
    if (clusters[o] < 0 || clusters[o] >= k) { free(slot); return -1; }
    slot[clusters[o]] = o;
  }
  memset(out, 0, sizeof(double) * (size_t)n_sel * (size_t)D);
  for (int64_t i = 0; i < n_docs; ++i) {
    int32_t j = a[i];
    if (j < 0 || j >= k) { free(slot); return -1; }
    int32_t o = slot[j];
    if (o < 0) continue;
    double *s = out + (size_t)o * (size_t)D;
    for (int64_t q = indptr[i]; q < indptr[i + 1]; ++q) s[indices[q]] += (double)values[q];
  }
  for (int32_t o = 0; o < n_sel; ++o) {
    double *c = out + (size_t)o * (size_t)D;
    double ss = 0.0;
    for (int32_t t = 0; t < D; ++t) ss += c[t] * c[t];
    double nrm = sqrt(ss);
    snorm[o] = nrm;
    if (nrm > 0.0)
      for (int32_t t = 0; t < D; ++t) c[t] = c[t] / nrm;
  }
  free(slot);
  return 0;
}

/*
 * k-means++ seeding (the initialisation named in Sec. 2; D^2 sampling of
 * Arthur and Vassilvitskii, 2007).  For unit vectors the squared Euclidean
 * distance to the nearest chosen seed is 2 (1 - s) with s the highest cosine,
 * so a row is drawn with probability proportional to 1 - s.  Readings:
 *   - the caller supplies one 64-bit uniform draw per seed; the first seed is
 *     row draws[0] mod n;
 *   - s_i = max over chosen seeds r of (x_i . x_r) / ||x_r||: the dot runs over
 *     the row's terms in ascending order as a chain of fused multiply-adds, the
 *     squared norm likewise over the seed's terms, then one sqrt and one divide;
 *   - the weight is the integer floor(2^32 max(0, 1 - s_i)), 0 for rows already
 *     chosen, so the draw is decided in exact integer arithmetic: with
 *     W = sum of weights > 0, seed m is the row whose cumulative weight
 *     interval [prefix, prefix + w_i) holds draws[m] mod W; with W = 0 (every
 *     row left points exactly like a seed) it is the lowest row not chosen.
 * Needs 1 <= k <= n_docs.  rows_out[k].
 */
int orc_kmeanspp(int64_t n_docs, int32_t D, const int64_t *indptr, const int32_t *indices,
                 const float *values, int32_t k, const uint64_t *draws, int32_t *rows_out) {
  if (k < 1 || (int64_t)k > n_docs) return -1;
  double *best = (double *)malloc(sizeof(double) * (size_t)n_docs);
  double *seed_row = (double *)calloc((size_t)D, sizeof(double));
  uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n_docs);
  unsigned char *chosen = (unsigned char *)calloc((size_t)n_docs, 1);
  if (!best || !seed_row || !w || !chosen) {
    free(best); free(seed_row); free(w); free(chosen);
    return -2;
  }
  for (int64_t i = 0; i < n_docs; ++i) best[i] = 0.0;
  int64_t r = (int64_t)(draws[0] % (uint64_t)n_docs);
  rows_out[0] = (int32_t)r;
  chosen[r] = 1;
  for (int32_t m = 1; m < k; ++m) {
    /* the previous seed as a dense row, and its length */
    double ss = 0.0;
    for (int64_t q = indptr[r]; q < indptr[r + 1]; ++q) {
      const double v = (double)values[q];
      seed_row[indices[q]] = v;
      ss = fma(v, v, ss);
    }
    const double nrm = sqrt(ss);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_docs; ++i) {
      double acc = 0.0;
      for (int64_t q = indptr[i]; q < indptr[i + 1]; ++q)
        acc = fma((double)values[q], seed_row[indices[q]], acc);
      const double s = acc / nrm;
      if (s > best[i]) best[i] = s;
      const double gap = 1.0 - best[i];
      w[i] = chosen[i] ? 0 : (uint64_t)floor(ldexp(gap > 0.0 ? gap : 0.0, 32));
    }
    for (int64_t q = indptr[r]; q < indptr[r + 1]; ++q) seed_row[indices[q]] = 0.0;
    uint64_t W = 0;
    for (int64_t i = 0; i < n_docs; ++i) W += w[i];
    int64_t pick = -1;
    if (W == 0) {
      for (int64_t i = 0; i < n_docs && pick < 0; ++i)
        if (!chosen[i]) pick = i;
    } else {
      const uint64_t t = draws[m] % W;
      uint64_t prefix = 0;
      for (int64_t i = 0; i < n_docs; ++i) {
        if (t < prefix + w[i]) {
          pick = i;
          break;
        }
        prefix += w[i];
      }
    }
    r = pick;
    rows_out[m] = (int32_t)r;
    chosen[r] = 1;
  }
  free(best); free(seed_row); free(w); free(chosen);
  return 0;
}
