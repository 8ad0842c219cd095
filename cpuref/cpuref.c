/*
 * cpuref.c — the paper's own method on CPU cores (OpenMP, FP64): spherical
 * k-means over sparse rows with map-like sparse centroids (Sec. 2: a dot
 * product costs O(min(p, k)) lookups), optionally skipping unchanged centroids
 * (Sec. 3.1, NCC) and pruning candidates with the dot-product index (Sec. 3.2,
 * Lemma 3.1, INDEX), combined as the end of Sec. 3.2 describes.  It is a
 * like-for-like CPU figure for the paper's ablation (baseline / NCC /
 * NCC + INDEX), written from the paper's description; it shares no code with
 * the GPU library or with the FP64 oracle.
 *
 * Readings (the same ones the GPU library takes):
 *   - one iteration = assignment then update, starting from seed rows;
 *   - argmax ties go to the lowest centroid index; an empty cluster keeps its
 *     centroid;
 *   - "unchanged" (Sec. 3.1) means an unchanged member set; member sums are
 *     taken in ascending row order, so such a centroid is bit-identical;
 *   - the index keeps, per centroid, its entries sorted by value (descending),
 *     their prefix sums of squares, the map G (term -> centroids with a
 *     non-zero there) and, per threshold, P (term -> (centroid, minimum
 *     overlap count)); a row's threshold is the highest one with
 *     lambda ||x|| <= (baseline - its FP64 error); candidate tests compare
 *     against lambda^2 less a bound on the prefix sums' rounding, so rounding
 *     can only add candidates;
 *   - stop after an assignment that moved no row (from the second one on), or
 *     after an update whose largest squared centroid shift is below the
 *     threshold (Sec. 4.1), or after max_iter iterations.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CR_NCC 1
#define CR_INDEX 2
#define CR_MAXLAM 8

/* A sparse centroid: terms ascending, values, and an open-addressing map
 * term -> position for O(1) lookups. */
typedef struct {
  int64_t n;
  int32_t *term;
  double *val;
  int32_t *slot;   /* [cap] position + 1, 0 = empty */
  int64_t cap;     /* power of two >= 2n */
} cent_t;

static inline uint32_t hash32(uint32_t t) {
  t ^= t >> 16;
  t *= 0x7feb352du;
  t ^= t >> 15;
  t *= 0x846ca68bu;
  t ^= t >> 16;
  return t;
}

static void cent_free(cent_t *c) {
  free(c->term);
  free(c->val);
  free(c->slot);
  memset(c, 0, sizeof(*c));
}

/* Builds c from the n listed terms (ascending) of a dense row r. */
static int cent_from_terms(cent_t *c, const double *r, const int32_t *terms, int64_t n) {
  cent_t z = {0};
  z.n = n;
  z.term = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  z.val = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  z.cap = 1;
  while (z.cap < 2 * n + 2) z.cap <<= 1;
  z.slot = (int32_t *)calloc((size_t)z.cap, sizeof(int32_t));
  if (!z.term || !z.val || !z.slot) {
    cent_free(&z);
    return -1;
  }
  for (int64_t q = 0; q < n; ++q) {
    const int32_t t = terms[q];
    z.term[q] = t;
    z.val[q] = r[t];
    uint64_t h = hash32((uint32_t)t) & (uint64_t)(z.cap - 1);
    while (z.slot[h]) h = (h + 1) & (uint64_t)(z.cap - 1);
    z.slot[h] = (int32_t)(q + 1);
  }
  cent_free(c);
  *c = z;
  return 0;
}

static inline double cent_get(const cent_t *c, int32_t t) {
  uint64_t h = hash32((uint32_t)t) & (uint64_t)(c->cap - 1);
  for (;;) {
    const int32_t s = c->slot[h];
    if (!s) return 0.0;
    if (c->term[s - 1] == t) return c->val[s - 1];
    h = (h + 1) & (uint64_t)(c->cap - 1);
  }
}

/* x . c: one lookup per row term, ascending terms (Sec. 2's map-based dot). */
static inline double dot_row(const int64_t *ip, const int32_t *ix, const float *v, int64_t i,
                             const cent_t *c) {
  double s = 0.0;
  for (int64_t q = ip[i]; q < ip[i + 1]; ++q) s += (double)v[q] * cent_get(c, ix[q]);
  return s;
}

/* (s, j) beats (bs, bj): higher score, then lower index. */
static inline int better(double s, int32_t j, double bs, int32_t bj) {
  return s > bs || (s == bs && j < bj);
}

/* ------------------------------------------------------------ the index */

typedef struct {
  int32_t c, m;
} pent_t;

typedef struct {
  int n_lam;
  double lam[CR_MAXLAM];
  int64_t *goff;    /* [D + 1] */
  int32_t *G;       /* centroid ids per term */
  int64_t *poff[CR_MAXLAM];
  pent_t *P[CR_MAXLAM];
} index_t;

static void index_free(index_t *x) {
  free(x->goff);
  free(x->G);
  for (int l = 0; l < CR_MAXLAM; ++l) {
    free(x->poff[l]);
    free(x->P[l]);
  }
  memset(x, 0, sizeof(*x));
}

typedef struct {
  double v;
  int32_t t;
} vt_t;

static int cmp_i32(const void *a, const void *b) {
  const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return x < y ? -1 : (x > y);
}

static int cmp_desc(const void *a, const void *b) {
  const vt_t *x = (const vt_t *)a, *y = (const vt_t *)b;
  if (x->v != y->v) return x->v > y->v ? -1 : 1;
  return x->t < y->t ? -1 : (x->t > y->t);
}

/* lambda^2 less a bound on the rounding of differences of sequential FP64
 * prefix sums of n squares with total q (each prefix off by at most
 * g_{n+1} q, the difference adds one rounding). */
static double lam_thr(double lam, int64_t n, double q) {
  const double u = 0x1p-53, m = (double)n + 2.0;
  const double g = m * u / (1.0 - m * u);
  return lam * lam - ((2.0 * g + 2.0 * u) * q / (1.0 - g) + 4.0 * u) * (1.0 + 0x1p-20);
}

/* G and P for every threshold, from the sparse centroids (Sec. 3.2). */
static int index_build(index_t *x, const cent_t *C, int32_t k, int64_t D, int n_lam,
                       const double *lam) {
  index_free(x);
  x->n_lam = n_lam;
  for (int l = 0; l < n_lam; ++l) x->lam[l] = lam[l];
  x->goff = (int64_t *)calloc((size_t)D + 1, sizeof(int64_t));
  if (!x->goff) return -1;
  int64_t total = 0;
  for (int32_t j = 0; j < k; ++j) {
    total += C[j].n;
    for (int64_t q = 0; q < C[j].n; ++q) x->goff[C[j].term[q] + 1] += 1;
  }
  for (int64_t t = 0; t < D; ++t) x->goff[t + 1] += x->goff[t];
  x->G = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(D + 1));
  if (!x->G || !fill) {
    free(fill);
    return -1;
  }
  memcpy(fill, x->goff, sizeof(int64_t) * (size_t)(D + 1));
  for (int32_t j = 0; j < k; ++j)   /* ascending centroid ids per term */
    for (int64_t q = 0; q < C[j].n; ++q) x->G[fill[C[j].term[q]]++] = j;
  /* P: per centroid, sorted entries and prefix sums; m_p = least m with
   * Q[p + m] - Q[p] >= lambda^2 (entries at p with no such m stop the
   * centroid's insertion, Sec. 3.2 step 3) */
  int32_t *pm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1) * n_lam);
  int64_t *pcnt = (int64_t *)calloc((size_t)(D + 1) * n_lam, sizeof(int64_t));
  int64_t *coff = (int64_t *)malloc(sizeof(int64_t) * ((size_t)k + 1));
  if (!pm || !pcnt || !coff) {
    free(fill);
    free(pm);
    free(pcnt);
    free(coff);
    return -1;
  }
  coff[0] = 0;
  for (int32_t j = 0; j < k; ++j) coff[j + 1] = coff[j] + C[j].n;
  int32_t *sorted_t = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  int fail = !sorted_t;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t j = 0; j < k; ++j) {
    const int64_t n = C[j].n;
    if (fail || n == 0) continue;
    vt_t *e = (vt_t *)malloc(sizeof(vt_t) * (size_t)n);
    double *Q = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!e || !Q) {
      fail = 1;
      free(e);
      free(Q);
      continue;
    }
    for (int64_t q = 0; q < n; ++q) {
      e[q].v = C[j].val[q];
      e[q].t = C[j].term[q];
    }
    qsort(e, (size_t)n, sizeof(vt_t), cmp_desc);
    Q[0] = 0.0;
    for (int64_t q = 0; q < n; ++q) Q[q + 1] = Q[q] + e[q].v * e[q].v;
    for (int64_t q = 0; q < n; ++q) sorted_t[coff[j] + q] = e[q].t;
    for (int l = 0; l < n_lam; ++l) {
      const double thr = lam_thr(lam[l], n, Q[n]);
      int64_t h = 0;   /* window end: Q[h] - Q[p] >= thr, two pointers */
      for (int64_t p = 0; p < n; ++p) {
        if (h < p + 1) h = p + 1;
        while (h < n && Q[h] - Q[p] < thr) ++h;
        int32_t m = -1;
        if (Q[h] - Q[p] >= thr) m = (int32_t)(h - p);
        pm[(coff[j] + p) * n_lam + l] = m;
      }
    }
    free(e);
    free(Q);
  }
  if (fail) {
    free(fill);
    free(pm);
    free(pcnt);
    free(coff);
    free(sorted_t);
    return -1;
  }
  for (int l = 0; l < n_lam; ++l) {
    int64_t *cnt = pcnt + (size_t)(D + 1) * l;
    int64_t np = 0;
    for (int32_t j = 0; j < k; ++j)
      for (int64_t p = 0; p < C[j].n; ++p) {
        if (pm[(coff[j] + p) * n_lam + l] < 0) break;   /* insertion stops */
        cnt[sorted_t[coff[j] + p] + 1] += 1;
        ++np;
      }
    for (int64_t t = 0; t < D; ++t) cnt[t + 1] += cnt[t];
    x->poff[l] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(D + 1));
    x->P[l] = (pent_t *)malloc(sizeof(pent_t) * (size_t)(np > 0 ? np : 1));
    if (!x->poff[l] || !x->P[l]) {
      fail = 1;
      break;
    }
    memcpy(x->poff[l], cnt, sizeof(int64_t) * (size_t)(D + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(D + 1));
    for (int32_t j = 0; j < k; ++j)
      for (int64_t p = 0; p < C[j].n; ++p) {
        const int32_t m = pm[(coff[j] + p) * n_lam + l];
        if (m < 0) break;
        pent_t pe = {j, m};
        x->P[l][fill[sorted_t[coff[j] + p]]++] = pe;
      }
  }
  free(fill);
  free(pm);
  free(pcnt);
  free(coff);
  free(sorted_t);
  return fail ? -1 : 0;
}

/* ------------------------------------------------------------ the loop */

typedef struct {
  int32_t iterations;
  int32_t converged;
  double seconds_assign, seconds_update, seconds_index;
  int64_t dots;        /* dot products computed (row, centroid) */
  int64_t index_rows;  /* rows whose candidates came from the index */
} cr_stats;

/* Runs the clustering; a_out [N] receives the final assignment (the one that
 * produced the final centroids, or the last one when the loop stopped after
 * an assignment), moved [max_iter] the rows moved per iteration (N at the
 * first).  max_seconds > 0 ends the run after the first iteration that
 * finishes later than that (converged stays 0).  Returns 0, or -1 when memory
 * runs out. */
int cr_run(int64_t N, int64_t D, const int64_t *ip, const int32_t *ix, const float *v, int32_t k,
           const int32_t *seeds, uint32_t flags, int n_lam, const double *lam, int32_t max_iter,
           double max_shift_sq, double max_seconds, int32_t nthreads, int32_t *a_out,
           int64_t *moved, cr_stats *st) {
  const double t_start = omp_get_wtime();
  if (nthreads > 0) omp_set_num_threads(nthreads);
  memset(st, 0, sizeof(*st));
  cent_t *C = (cent_t *)calloc((size_t)k, sizeof(cent_t));
  int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int32_t *ap = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  uint8_t *changed = (uint8_t *)malloc((size_t)k);
  int64_t *cnt = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
  int64_t *members = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  double *xn = (double *)malloc(sizeof(double) * (size_t)N);
  index_t X;
  memset(&X, 0, sizeof(X));
  int rc = 0;
  if (!C || !a || !ap || !changed || !cnt || !members || !xn) {
    rc = -1;
    goto out;
  }
  /* seeds: c_j = x_r / ||x_r|| (Sec. 2: unit centroids) */
  {
    double *row = (double *)calloc((size_t)D, sizeof(double));
    if (!row) {
      rc = -1;
      goto out;
    }
    for (int32_t j = 0; j < k && !rc; ++j) {
      const int64_t r = seeds[j];
      double ss = 0.0;
      for (int64_t q = ip[r]; q < ip[r + 1]; ++q) ss += (double)v[q] * (double)v[q];
      const double nrm = sqrt(ss);
      for (int64_t q = ip[r]; q < ip[r + 1]; ++q) row[ix[q]] = (double)v[q] / nrm;
      if (cent_from_terms(&C[j], row, ix + ip[r], ip[r + 1] - ip[r])) rc = -1;
      for (int64_t q = ip[r]; q < ip[r + 1]; ++q) row[ix[q]] = 0.0;
    }
    free(row);
    if (rc) goto out;
  }
  for (int64_t i = 0; i < N; ++i) {
    double ss = 0.0;
    for (int64_t q = ip[i]; q < ip[i + 1]; ++q) ss += (double)v[q] * (double)v[q];
    xn[i] = sqrt(ss);
  }
  memset(changed, 1, (size_t)k);
  int have_prev = 0;
  for (int32_t t = 0; t < max_iter; ++t) {
    const int use_ncc = (flags & CR_NCC) && have_prev;
    const int use_index = (flags & CR_INDEX) && have_prev;
    double t0 = omp_get_wtime();
    if (use_index && index_build(&X, C, k, D, n_lam, lam)) {
      rc = -1;
      goto out;
    }
    st->seconds_index += omp_get_wtime() - t0;
    t0 = omp_get_wtime();
    int64_t n_moved = 0, n_dots = 0, n_idx = 0;
    int fail = 0;
    int32_t n_ch = 0;
    int32_t *ch_list = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    if (!ch_list) {
      rc = -1;
      goto out;
    }
    for (int32_t j = 0; j < k; ++j)
      if (changed[j]) ch_list[n_ch++] = j;
#pragma omp parallel reduction(+ : n_moved, n_dots, n_idx)
    {
      uint16_t *count = use_index ? (uint16_t *)calloc((size_t)k, sizeof(uint16_t)) : NULL;
      int32_t *touched = use_index ? (int32_t *)malloc(sizeof(int32_t) * (size_t)k) : NULL;
      uint8_t *cand = use_index ? (uint8_t *)calloc((size_t)k, 1) : NULL;
      int32_t *clist = use_index ? (int32_t *)malloc(sizeof(int32_t) * (size_t)k) : NULL;
      if (use_index && (!count || !touched || !cand || !clist)) fail = 1;
#pragma omp for schedule(dynamic, 256)
      for (int64_t i = 0; i < N; ++i) {
        if (fail) continue;
        const int32_t prev = have_prev ? ap[i] : -1;
        const int keep = use_ncc && !changed[prev];   /* Sec. 3.1 */
        double bs = -INFINITY;
        int32_t bj = INT32_MAX;
        int done = 0;
        if (use_index) {
          /* Sec. 3.2: baseline from the previous centroid, highest threshold
           * not above it, candidates from G / P */
          const double b = dot_row(ip, ix, v, i, &C[prev]);
          ++n_dots;
          const int64_t nx = ip[i + 1] - ip[i];
          const double blo = b - ((double)nx + 2.0) * 0x1p-52 * fabs(b);
          int lv = -1;
          for (int l = 0; l < n_lam; ++l)
            if (lam[l] * xn[i] * (1.0 + 0x1p-40) <= blo) lv = l;
          if (lv >= 0) {
            int32_t nt = 0, nc = 0;
            for (int64_t q = ip[i]; q < ip[i + 1]; ++q) {
              const int32_t tt = ix[q];
              for (int64_t g = X.goff[tt]; g < X.goff[tt + 1]; ++g) {
                const int32_t j = X.G[g];
                if (count[j]++ == 0) touched[nt++] = j;
              }
            }
            for (int64_t q = ip[i]; q < ip[i + 1]; ++q) {
              const int32_t tt = ix[q];
              for (int64_t g = X.poff[lv][tt]; g < X.poff[lv][tt + 1]; ++g) {
                const pent_t pe = X.P[lv][g];
                if (!cand[pe.c] && count[pe.c] >= pe.m && (!keep || changed[pe.c])) {
                  cand[pe.c] = 1;
                  clist[nc++] = pe.c;
                }
              }
            }
            bs = b;
            bj = prev;
            for (int32_t q = 0; q < nc; ++q) {
              const int32_t j = clist[q];
              cand[j] = 0;
              if (j == prev) continue;
              const double s = dot_row(ip, ix, v, i, &C[j]);
              ++n_dots;
              if (better(s, j, bs, bj)) {
                bs = s;
                bj = j;
              }
            }
            for (int32_t q = 0; q < nt; ++q) count[touched[q]] = 0;
            done = 1;
            ++n_idx;
          }
        }
        if (!done) {
          if (keep) {
            /* the previous centroid is the best unchanged one (Sec. 3.1) */
            bs = dot_row(ip, ix, v, i, &C[prev]);
            bj = prev;
            ++n_dots;
            for (int32_t q = 0; q < n_ch; ++q) {
              const int32_t j = ch_list[q];
              const double s = dot_row(ip, ix, v, i, &C[j]);
              ++n_dots;
              if (better(s, j, bs, bj)) {
                bs = s;
                bj = j;
              }
            }
          } else {
            for (int32_t j = 0; j < k; ++j) {
              const double s = dot_row(ip, ix, v, i, &C[j]);
              ++n_dots;
              if (better(s, j, bs, bj)) {
                bs = s;
                bj = j;
              }
            }
          }
        }
        a[i] = bj;
        if (!have_prev || bj != prev) ++n_moved;
      }
      free(count);
      free(touched);
      free(cand);
      free(clist);
    }
    free(ch_list);
    if (fail) {
      rc = -1;
      goto out;
    }
    st->seconds_assign += omp_get_wtime() - t0;
    st->dots += n_dots;
    st->index_rows += n_idx;
    moved[t] = n_moved;
    st->iterations = t + 1;
    if (have_prev && n_moved == 0) {
      st->converged = 1;
      memcpy(a_out, a, sizeof(int32_t) * (size_t)N);
      goto out;
    }
    /* update: changed = clusters whose member set changed; their sums in
     * ascending row order, normalised (Sec. 2); empty clusters keep theirs */
    t0 = omp_get_wtime();
    if (!have_prev) {
      memset(changed, 1, (size_t)k);
    } else {
      memset(changed, 0, (size_t)k);
      for (int64_t i = 0; i < N; ++i)
        if (a[i] != ap[i]) changed[a[i]] = changed[ap[i]] = 1;
    }
    memset(cnt, 0, sizeof(int64_t) * ((size_t)k + 1));
    for (int64_t i = 0; i < N; ++i) cnt[a[i] + 1] += 1;
    for (int32_t j = 0; j < k; ++j) cnt[j + 1] += cnt[j];
    {
      int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)k + 1));
      if (!fill) {
        rc = -1;
        goto out;
      }
      memcpy(fill, cnt, sizeof(int64_t) * ((size_t)k + 1));
      for (int64_t i = 0; i < N; ++i) members[fill[a[i]]++] = i;
      free(fill);
    }
    double max_shift = 0.0;
#pragma omp parallel reduction(max : max_shift)
    {
      double *S = (double *)calloc((size_t)D, sizeof(double));
      int32_t *terms = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
      if (!S || !terms) fail = 1;
#pragma omp for schedule(dynamic, 4)
      for (int32_t j = 0; j < k; ++j) {
        if (fail || !changed[j] || cnt[j + 1] == cnt[j]) continue;
        /* the members' sum in ascending row order, its support listed */
        int64_t nt = 0;
        for (int64_t m = cnt[j]; m < cnt[j + 1]; ++m) {
          const int64_t i = members[m];
          for (int64_t q = ip[i]; q < ip[i + 1]; ++q) {
            if (S[ix[q]] == 0.0) terms[nt++] = ix[q];
            S[ix[q]] += (double)v[q];
          }
        }
        qsort(terms, (size_t)nt, sizeof(int32_t), cmp_i32);
        double ss = 0.0;
        for (int64_t q = 0; q < nt; ++q) ss += S[terms[q]] * S[terms[q]];
        const double nrm = sqrt(ss);
        /* shift ||c_new - c_old||^2 over both supports */
        double sh = 0.0;
        for (int64_t q = 0; q < nt; ++q) {
          const int32_t t2 = terms[q];
          S[t2] /= nrm;
          const double d = S[t2] - cent_get(&C[j], t2);
          sh += d * d;
        }
        for (int64_t q = 0; q < C[j].n; ++q)
          if (S[C[j].term[q]] == 0.0) sh += C[j].val[q] * C[j].val[q];
        if (sh > max_shift) max_shift = sh;
        if (cent_from_terms(&C[j], S, terms, nt)) fail = 1;
        for (int64_t q = 0; q < nt; ++q) S[terms[q]] = 0.0;
      }
      free(S);
      free(terms);
    }
    if (fail) {
      rc = -1;
      goto out;
    }
    st->seconds_update += omp_get_wtime() - t0;
    memcpy(ap, a, sizeof(int32_t) * (size_t)N);
    memcpy(a_out, a, sizeof(int32_t) * (size_t)N);
    have_prev = 1;
    if (max_shift < max_shift_sq) {
      st->converged = 1;
      goto out;
    }
    if (max_seconds > 0 && omp_get_wtime() - t_start > max_seconds) goto out;
  }
out:
  index_free(&X);
  if (C)
    for (int32_t j = 0; j < k; ++j) cent_free(&C[j]);
  free(C);
  free(a);
  free(ap);
  free(changed);
  free(cnt);
  free(members);
  free(xn);
  return rc;
}
