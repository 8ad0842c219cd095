/*
 * skm.h — exact sparse spherical k-means on AMD MI355X (gfx950).
 *
 * Implements the method of Knittel, Koch & Ertl, "Efficient Sparse Spherical
 * k-Means for Document Clustering" (DocEng 2021):
 *   - Sec. 2: rows are unit-length sparse vectors; a centroid is the sum of its
 *     members divided by that sum's length; each row goes to the centroid with
 *     the highest dot product; the loop alternates update and assignment and
 *     stops when assignments no longer change or when the largest squared
 *     centroid shift falls below a threshold (Sec. 4.1 uses 1e-4).
 *   - Sec. 3.1 (NCC): a row whose previous centroid did not change only has to
 *     be compared with the centroids that did change.
 *   - Sec. 3.2 (INDEX): an index over the centroids' sorted entries that, given
 *     a baseline similarity, returns a superset of the centroids that can reach
 *     it (Lemma 3.1); several thresholds {0.1, 0.25, 0.4, 0.6}; the highest one
 *     not above the baseline is used.
 *
 * Results are those of a plain FP64 run: ties in the argmax go to the lowest
 * centroid index, an empty cluster keeps its centroid.  Scores may be computed
 * from FP32, BF16 or FP8-E4M3 copies of the centroids with FP32 accumulation;
 * every row whose best centroid is not certified by a bound derived from the
 * format's rounding and the accumulation error is decided again in FP64 against
 * the FP64 centroids.
 *
 * Conventions for every call:
 *   - Returns an skm_status; no C++ exception crosses this interface.
 *   - On SKM_E_INVALID / SKM_E_STATE nothing was modified.  On SKM_E_NOMEM
 *     the clustering state (assignments, centroids, counters) is unchanged
 *     and the call may be repeated; derived scratch such as the changed
 *     flags may have been recomputed.
 *   - On SKM_E_DEVICE the context is unusable; only skm_destroy is valid.
 *   - skm_last_error() returns a thread-local message for the last failure.
 *   - A context is used by one thread at a time.  Work is enqueued on the
 *     context's stream; every call below returns after its results are
 *     complete (it synchronises that stream), except where stated.
 *   - "device pointer" means HIP device memory of the context's device;
 *     "host pointer" means ordinary process memory.
 */
#ifndef SKM_H
#define SKM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct skm_ctx skm_ctx;

typedef enum {
  SKM_OK = 0,
  SKM_E_INVALID = 1,     /* malformed arguments or input */
  SKM_E_NOMEM = 2,       /* the HBM budget or the device is out of memory */
  SKM_E_DEVICE = 3,      /* a HIP call failed; the context is poisoned */
  SKM_E_STATE = 4,       /* call made in the wrong order */
  SKM_E_UNSUPPORTED = 5, /* valid but outside what this build supports */
  SKM_E_BUSY = 6,        /* a request server is attached to the context */
  SKM_E_TIMEOUT = 7,     /* skm_server_wait ran out of time (request still queued) */
  SKM_E_CANCELLED = 8    /* the request or job was cancelled (skm_server_cancel, or
                            a job still pending when its server stopped) */
} skm_status;

typedef enum {
  SKM_FP32 = 0,      /* centroids scored from float copies */
  SKM_BF16 = 1,      /* bfloat16 copies, round to nearest even */
  SKM_FP8_E4M3 = 2   /* OCP E4M3 copies times a power-of-two scale per centroid */
} skm_precision;

enum {
  SKM_NCC = 1u << 0,       /* Sec. 3.1: skip centroids that did not change */
  SKM_INDEX = 1u << 1,     /* Sec. 3.2: dot-product index on rows whose previous
                              centroid changed */
  SKM_NO_EXACT = 1u << 2,  /* skip the exact tier: the argmax is taken on the
                              low-precision scores alone (timing comparator only;
                              results are then NOT those of an FP64 run) */
  SKM_DENSE_ONLY = 1u << 3, /* score every term from the dense code slabs (no
                              per-term lists of non-zero codes) */
  SKM_BORROW_DEVICE = 1u << 4 /* skm_init / skm_load with device rows: use the
                              caller's three arrays in place instead of copying
                              them; the caller keeps them alive and unchanged
                              until skm_destroy (host rows are still copied) */
};

typedef enum {
  SKM_STOP_PAPER = 0,  /* stop after an assignment that moved nothing (or fewer
                          than min_moved_frac * n_rows rows), or after an update
                          whose largest squared centroid shift is < max_shift_sq */
  SKM_STOP_FIXED = 1   /* run exactly max_iter iterations */
} skm_stop_rule;

/*
 * A CSR matrix of rows (documents).  Borrowed for the duration of the call
 * (for the context's lifetime with SKM_BORROW_DEVICE).
 *   indptr  [n_rows + 1], indptr[0] = 0, non-decreasing, indptr[n_rows] = nnz
 *   indices [nnz], strictly ascending within a row, in [0, n_cols)
 *   values  [nnz], finite and > 0; each row's L2 norm within 1e-5 of 1
 * on_device = 1: the three arrays are device pointers; 0: host pointers.
 */
typedef struct {
  int64_t n_rows;
  int64_t n_cols;
  int64_t nnz;
  const int64_t *indptr;
  const int32_t *indices;
  const float *values;
  int32_t on_device;
} skm_csr;

typedef struct {
  int32_t k;                  /* number of clusters, 1 <= k <= 65535 */
  int32_t precision;          /* skm_precision */
  uint32_t flags;             /* SKM_NCC | SKM_INDEX | SKM_NO_EXACT */
  int32_t n_lambda;           /* index thresholds, ascending, in (0, 1] */
  double lambda[8];           /* default {0.1, 0.25, 0.4, 0.6} (Sec. 4.1) */
  int32_t index_min_changed;  /* use the index only when more than this many
                                 centroids changed (Sec. 4.3 suggests ~100);
                                 0 = whenever SKM_INDEX is set */
  int32_t stop_rule;          /* skm_stop_rule */
  int32_t max_iter;           /* cap for skm_iterate */
  double min_moved_frac;      /* SKM_STOP_PAPER: also stop when fewer than this
                                 fraction of rows moved (0 = only when none) */
  double max_shift_sq;        /* SKM_STOP_PAPER shift threshold (Sec. 4.1: 1e-4) */
  const int32_t *init_rows;   /* host, k distinct row ids: c_j = x_r / ||x_r|| */
  const double *init_centroids; /* host, k x n_cols row-major; used when
                                   init_rows is NULL (rows must be unit length,
                                   non-negative) */
  size_t hbm_budget_bytes;    /* 0 = no limit; counts every device allocation
                                 the context makes.  Without a budget skm_init
                                 also allocates the update's largest workspace
                                 (at most 16 GiB) so that no iteration
                                 allocates it; under one it grows on demand */
  void *stream;               /* hipStream_t to enqueue on; NULL = own stream */
  int32_t validate;           /* 1 = check the CSR conventions above at init */
  int32_t head_max_terms;     /* BF16 / FP8 scoring: at most this many of the most
                                 frequent terms are scored as a dense BF16 block on
                                 the matrix cores (rounded to a multiple of 64);
                                 below 64 = off.  Default 4096. */
  double head_min_df;         /* a term joins that head when at least this fraction
                                 of the rows contain it.  Default 1/128. */
  int32_t ncc_adaptive;       /* SKM_NCC: 0 (default) = use Sec. 3.1 whenever its
                                 estimated scoring work is at most 0.9 of a full
                                 pass; 1 = also only when its predicted assignment
                                 time (its share of the last full pass's scoring
                                 plus its own fixed cost, measured at its last use)
                                 is below the last full assignment's.  Results are
                                 the same either way. */
  int32_t index_always;       /* SKM_INDEX: 1 = query and rebuild the index after
                                 every update even when it decides few rows (no
                                 back-off); 0 (default) = back off (Sec. 4.3) */
} skm_config;

typedef struct {
  int32_t iter;               /* index of this iteration (0-based) */
  int32_t changed_centroids;  /* centroids that changed before this assignment
                                 (all of them at iteration 0) */
  int64_t moved;              /* rows whose assignment changed (n_rows at 0) */
  int64_t flagged;            /* rows sent to the exact FP64 tier */
  int64_t band_overflow;      /* flagged rows whose band of possible winners exceeded
                                 the exact tier's buffer (scored in several passes) */
  int64_t ncc_rows;           /* rows that only compared changed centroids */
  int64_t index_rows;         /* rows whose candidates came from the index */
  int64_t index_no_level;     /* index-eligible rows whose baseline reached no
                                 threshold (scored densely) */
  int64_t index_guarded;      /* rows whose index query would read more entries
                                 than a quarter of a dense scan (scored densely) */
  int64_t index_over_cap;     /* rows with more candidates than the per-row list
                                 holds (scored densely) */
  double mean_candidates;     /* centroids scored per row (low precision) */
  double scored_products;     /* sum over rows of nnz_i * (centroids scored):
                                 the multiply-adds of the scoring kernel */
  double objective_assign;    /* J_A = sum_i x_i . c_{a_i} (after update) */
  double objective_update;    /* J_U = sum_j ||S_j||       (after update) */
  double max_shift_sq;        /* max_j ||c_j(new) - c_j(old)||^2 (after update) */
  float ms_assign;            /* device time of the phases, milliseconds:
                                 whole assignment step (all of the below) */
  float ms_score;             /* the low-precision scoring kernel alone */
  float ms_exact;
  float ms_update;
  float ms_index;             /* index query + exact candidate scoring (assign),
                                 index build (update) */
  int32_t head_terms;         /* terms this assignment scored on the matrix cores
                                 (0 = none; NCC rows scored against at most 64
                                 changed centroids do not use it) */
  float ms_head;              /* device time of the head products (part of ms_score) */
  int32_t score_launches;     /* launches of the sparse scoring kernel */
  double sparse_products;     /* scored_products restricted to the terms scored on
                                 the sparse path (all of them when head_terms = 0) */
  float ms_sparse;            /* device time of the sparse scoring kernel's launches
                                 (part of ms_score) */
  int32_t head_launches;      /* launches of the head GEMM */
  double head_pairs;          /* (row, centroid) pairs the head GEMMs multiplied,
                                 each over head_terms terms */
  float ms_index_build;       /* device time of the index build (part of ms_index) */
  int32_t index_build;        /* index build of this update: 0 none, 1 full,
                                 2 only the changed centroids (Sec. 3.2 entries of
                                 the others kept) */
} skm_iter_stats;

/* One measured shape of the scoring work (skm_autotune). */
typedef struct {
  int32_t head_chunks;        /* 512-centroid chunks per head batch (0 = no head) */
  int32_t workgroups_per_cu;  /* workgroups per compute unit of the persistent sparse
                                 scoring grid */
  int64_t head_rows;          /* rows per head batch (0 = no head) */
  double ms;                  /* device time of one full scoring pass at this shape */
} skm_tune_trial;

typedef struct {
  int32_t n_trials;
  int32_t best;               /* index of the shape the context now uses */
  skm_tune_trial trials[16];
} skm_tune_report;

/* Fills *cfg with defaults: k = 0 (must be set), FP32, no flags, the four
 * thresholds of Sec. 4.1, paper stop rule, max_iter 100, shift 1e-4, head of
 * at most 4096 terms with document frequency >= 1/128. */
void skm_config_default(skm_config *cfg);

/* k-means++ seed rows (the initialisation Sec. 2 names; D^2 sampling, where
 * the squared distance of unit rows to the nearest seed is 2 (1 - s) with s
 * the highest cosine), for cfg->init_rows.  docs as for skm_init (host or
 * device, checked the same way; not kept).  draws: host, k uniform 64-bit
 * values supplied by the caller.  Seed 0 is row draws[0] mod n_rows; seed m
 * weighs row i by floor(2^32 max(0, 1 - s_i)), 0 if already a seed, and takes
 * the row whose cumulative weight interval holds draws[m] mod (total weight),
 * or the lowest row not yet a seed when the total is 0.  s_i is the row's FP64
 * dot product with the seed's values (ascending terms, fused multiply-adds)
 * divided by the seed's length, so the result depends only on the inputs and
 * the draws.  out_rows: host, k distinct row ids.  stream: hipStream_t or NULL
 * for a stream of the call's own; the call returns when the seeds are ready.
 * Work: k passes over the rows.  SKM_E_INVALID for bad arguments (k outside
 * [1, n_rows]) or rows that break the CSR conventions, SKM_E_NOMEM when the
 * device cannot hold its temporaries (about 25 bytes per row plus 8 per
 * column). */
skm_status skm_kmeanspp(const skm_csr *docs, int32_t k, const uint64_t *draws, int32_t *out_rows,
                        void *stream);

/* Creates a context for the problem of Sec. 2: unit-length sparse rows and k
 * centroids of unit length.  Copies the rows into HBM (or, with
 * SKM_BORROW_DEVICE, reads the caller's device rows in place), seeds the FP64
 * centroids from init_rows (c_j = x_r / ||x_r||) or init_centroids, and builds
 * their scoring copies (and, with SKM_INDEX, the Sec. 3.2 index).  *out is
 * owned by the caller and released with skm_destroy.  SKM_E_INVALID for a
 * malformed CSR or config, SKM_E_NOMEM when the budget is exceeded. */
skm_status skm_init(const skm_csr *docs, const skm_config *cfg, skm_ctx **out);

/* One assignment step against the current centroids: every row goes to the
 * centroid of highest dot product, lowest index on ties (Sec. 2); with SKM_NCC
 * a row whose previous centroid did not change compares only the changed ones
 * (Sec. 3.1); with SKM_INDEX rows take their candidates from the index at the
 * highest threshold not above their baseline (Sec. 3.2, Lemma 3.1).  The
 * result equals the plain step's.  st (host, may be NULL) receives the step's
 * counters and device times.  SKM_E_BUSY while a server is attached. */
skm_status skm_assign(skm_ctx *c, skm_iter_stats *st);

/* One update step from the last assignment (Sec. 2: a centroid is the sum of
 * its members divided by that sum's length; a cluster without members keeps
 * its centroid): FP64 member sums in ascending row order for every cluster
 * whose membership changed, renormalisation, the changed-centroid set that
 * Sec. 3.1 needs for the next assignment, new scoring copies and, when
 * enabled, the Sec. 3.2 index.  st (host, may be NULL) receives the objective
 * and the largest squared centroid shift.  SKM_E_STATE if no assignment
 * preceded it. */
skm_status skm_update(skm_ctx *c, skm_iter_stats *st);

/* The loop of Sec. 2 with the stopping rule of Sec. 4.1: repeats {assign;
 * stop test; update; stop test} up to max_iter times (the config's cap when
 * max_iter <= 0).  Under SKM_STOP_PAPER it stops after an assignment that moved
 * no row (or fewer than min_moved_frac of them) or after an update whose
 * largest squared centroid shift is below max_shift_sq.  per_iter: host array
 * of max_iter records or NULL.  *n_done = iterations started, *converged = 1
 * if a stop test (not the cap) ended the loop. */
skm_status skm_iterate(skm_ctx *c, int32_t max_iter, skm_iter_stats *per_iter,
                       int32_t *n_done, int32_t *converged);

/* Not part of the paper's method: assigns new rows to the current centroids
 * with the assignment rule of Sec. 2, without changing the context (exact, no
 * NCC since the rows have no previous assignment).  The rows must follow the
 * CSR conventions above (checked: SKM_E_INVALID otherwise).  out_assign
 * [n_rows] and out_score [n_rows] (the FP64 dot product with the chosen
 * centroid) are device pointers when docs->on_device, else host pointers.
 * stream: hipStream_t for this call (NULL = the context's stream).  Calls with
 * different streams may run concurrently with each other; they must not
 * overlap skm_assign/skm_update/skm_iterate on the same context. */
skm_status skm_assign_new(skm_ctx *c, const skm_csr *docs, int32_t *out_assign,
                          double *out_score, void *stream);

/* Rows of the last skm_assign_new to finish that the Sec. 3.2 index assigned (contexts
 * with SKM_INDEX once the index is built; the others score every centroid).
 * A new row's baseline is the certified FP64 score of a probe centroid: the
 * best of the centroids that are largest at the row's three largest values'
 * terms.  Not in the paper, which has no new rows.  -1 for an invalid
 * context. */
int64_t skm_assign_new_index_rows(const skm_ctx *c);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): skm_assign_new for
 * device rows without any device allocation.  docs must be device pointers
 * (on_device = 1) and is read in place; out_assign [n_rows] (int32) and
 * out_score [n_rows] (FP64 dot product with the chosen centroid) are device
 * pointers written directly.  The call's temporaries live in one static
 * device array of the library, skm_static_scratch_bytes() bytes (64 MiB) on
 * each GPU the library runs on, held until the process ends; at most
 * skm_static_max_rows(c) rows fit (about 64 MiB / (32 B x ceil(k / 512) + 45 B)),
 * more gives SKM_E_INVALID with nothing written.  The array is shared by every
 * call on that GPU and keeps the last call's contents: calls that overlap on
 * one GPU (different streams or threads) race and must be serialised by the
 * caller.  Same checks, results and errors as skm_assign_new otherwise; the
 * call synchronises `stream` (NULL = the context's stream) before returning. */
skm_status skm_assign_new_static(skm_ctx *c, const skm_csr *docs, int32_t *out_assign,
                                 double *out_score, void *stream);

/* Size of skm_assign_new_static's static workspace per GPU, in bytes. */
size_t skm_static_scratch_bytes(void);

/* Rows one skm_assign_new_static call on context c can take. */
int64_t skm_static_max_rows(const skm_ctx *c);

/* Current assignment (after skm_assign) into out[n_rows]. */
skm_status skm_get_assignments(const skm_ctx *c, int32_t *out, int32_t on_device);

/* Current FP64 centroids, k x n_cols row-major, into out. */
skm_status skm_get_centroids(const skm_ctx *c, double *out, int32_t on_device);

/* FP64 centroid values at the listed terms: out[j * n_terms + q] = c_j[terms[q]]
 * for every centroid j (host arrays; out holds k * n_terms doubles).  For checks
 * at sizes where the dense k x n_cols copy is too large to fetch. */
skm_status skm_get_centroid_columns(const skm_ctx *c, const int32_t *terms, int32_t n_terms,
                                    double *out);

/* FP64 centroids of the listed ids: out[q * n_cols + t] = c_{ids[q]}[t] (host). */
skm_status skm_get_centroid_rows(const skm_ctx *c, const int32_t *ids, int32_t n, double *out);

/* Replaces the centroids (host, k x n_cols, unit rows, non-negative), rebuilds
 * the scoring copies and marks every centroid changed.  For checks that feed
 * known centroids into one assignment step. */
skm_status skm_set_centroids(skm_ctx *c, const double *centroids);

/* Scoring copy of the centroids, term-major: codes[t * ld + j] for term t and
 * centroid j (4, 2 or 1 bytes per code for FP32 / BF16 / FP8), and the FP8 scale
 * per centroid (1.0 otherwise).  Host buffers: codes of n_cols * ld * bytes,
 * scales of k floats.  *ld receives the row stride (>= k). */
skm_status skm_get_tile(const skm_ctx *c, void *codes, size_t codes_bytes, float *scales,
                        int64_t *ld);

/* Changed-centroid flags (1 = changed since the previous assignment) into a
 * host array of k bytes. */
skm_status skm_get_changed(const skm_ctx *c, uint8_t *out);

/* Checkpoint (resume after a stop or a lost process).  Taken any time after
 * the first skm_update (SKM_E_STATE before); when an skm_assign is pending its
 * skm_update (as after skm_iterate stops on an assignment that moved nothing),
 * the file holds the state before that assignment, which a resumed run
 * repeats with the same result.  Writes to the host file path the assignment
 * that made the current centroids, the
 * certified score intervals of the rows' centroids, the changed-centroid flags,
 * the run's counters, and the centroids of the clusters without members
 * (sparse).  Every other centroid is the normalised sum of its members in
 * ascending row order, a function of the assignment, so it is not stored.
 * Size: 20 bytes per row, 1 per centroid, 12 per stored non-zero.  The file
 * is written as path + ".tmp" and renamed to path when complete, so an earlier
 * checkpoint at path survives a crash while writing.  SKM_E_INVALID when the
 * file cannot be written. */
skm_status skm_save(const skm_ctx *c, const char *path);

/* Resumes a run from skm_save's file: a new context (*out, released with
 * skm_destroy) over docs, which must be the rows the run used (same shape is
 * checked), with cfg's k, precision and SKM_NCC / SKM_INDEX / SKM_NO_EXACT /
 * SKM_DENSE_ONLY flags equal to the saved run's; cfg's other fields (stream,
 * budget, stop rule, limits) apply from here on, and cfg's init fields are
 * ignored.  The centroids are recomputed from the saved assignment, so the
 * resumed run continues bit for bit as the saved one would have.
 * SKM_E_INVALID for a missing, truncated or mismatched file (checked before
 * any device work); otherwise as skm_init. */
skm_status skm_load(skm_ctx **out, const skm_csr *docs, const char *path, const skm_config *cfg);

/* Low-precision scores of the rows in docs against every centroid, before any
 * exact tier: out[i * k + j], host, n_rows * k floats.  Diagnostic for checking
 * the error bound; small inputs only. */
skm_status skm_score_dense(skm_ctx *c, const skm_csr *docs, float *out);

/* The certified error bound the context applies to a low-precision score s of
 * a row with nnz terms and L1 norm l1: |s - exact| <= bound. */
double skm_error_bound(const skm_ctx *c, double s, int64_t nnz, double l1);

/* Number of head terms (the most frequent terms, scored as a dense BF16 block
 * on the matrix cores; see head_max_terms), 0 when the head is off. */
int32_t skm_head_terms(const skm_ctx *c);

/* Autotuner: times one full scoring pass (low precision, all centroids, no
 * exact tier) of the context's own rows for candidate shapes of the work —
 * the workgroups per CU of the persistent sparse scoring grid, from one above
 * its occupancy limit down to four below it, then the head batch shape (rows
 * x 512-centroid chunks filling the head-score buffer) — and keeps the
 * fastest trial for the following assignment steps.  Results are unaffected (the shape only changes the
 * schedule).  Call it with no assignment pending (before skm_assign or after
 * skm_update); SKM_E_STATE otherwise.  report (may be NULL) receives every
 * trial. */
skm_status skm_autotune(skm_ctx *c, skm_tune_report *report);

/* Measured thresholds of the Sec. 3.2 index (skm_tune_lambda). */
typedef struct {
  int32_t n_sample;           /* rows measured */
  int32_t n_grid;             /* thresholds measured */
  double grid[20];            /* ascending */
  double qualify[20];         /* share of the rows whose baseline reaches grid[g] ||x|| */
  double mean_candidates[20]; /* centroids those rows would score at grid[g] */
  int32_t n_before, n_after;
  double before[8], after[8]; /* the set in use before and after the call */
  double cost_before;         /* centroids scored per sampled row with `before` */
  double cost_after;          /* the same with `after` */
  int32_t applied;            /* 1 if the context now uses `after` */
} skm_lambda_report;

/* Tunes the index's threshold set (Sec. 3.2 builds several thresholds and uses
 * the highest one a row's baseline reaches; Sec. 4.1 fixes {0.1, 0.25, 0.4,
 * 0.6}) for this workload: on n_sample rows spread over the corpus, against
 * the current centroids and with each row's previous centroid as baseline, it
 * measures for every threshold of a fixed grid (0.05 .. 0.8, plus the set in
 * use) which rows qualify and how many candidates the index returns, and
 * takes the set of at most four grid values that minimises the centroids
 * scored per row (a qualifying row scores its candidates plus its baseline
 * centroid; another row scores every centroid, or with SKM_NCC the changed
 * ones when its previous centroid did not change), when it is at least 5 %
 * cheaper than the set in use.  Results are unaffected (every set gives the
 * exact assignment).  Needs SKM_INDEX, a completed skm_update and no pending
 * assignment (SKM_E_STATE).  report (host, may be NULL) receives the
 * measurements. */
skm_status skm_tune_lambda(skm_ctx *c, int32_t n_sample, skm_lambda_report *report);

/* Applies a shape found by skm_autotune (for instance on another context of
 * the same workload): workgroups_per_cu, and head_chunks x head_rows when the
 * context scores a head (they must fit its head-score buffer, else
 * SKM_E_INVALID; ignored when the head is off).  ms is not read. */
skm_status skm_set_schedule(skm_ctx *c, const skm_tune_trial *shape);

/* Diagnostic: the low-precision scores of the context's own rows
 * [row0, row0 + n_rows) as an assignment step with the head computes them
 * (head product and the rows' other terms summed apart, then added), before
 * any exact tier: out[i * k + j], host, n_rows * k floats; out_head (host,
 * same layout, may be NULL) receives the head parts alone.  SKM_E_STATE when
 * the head is off; SKM_E_INVALID for a range outside the rows or above one
 * head batch. */
skm_status skm_score_head(skm_ctx *c, int64_t row0, int64_t n_rows, float *out,
                          float *out_head);

/* Not in the paper (it states no precision): the certified bound for such
 * head scores as a function of the score alone, for scores computed with the
 * row values of head terms rounded to BF16 and matrix-core accumulation; -1
 * when the head is off. */
double skm_error_bound_head(const skm_ctx *c, double s, int64_t nnz, double l1);

/* FP8 contexts with a head: the bound the assignment step uses, from the head
 * part hs (BF16 head codes rounded from the FP64 centroids) and the part rs
 * of the n_rest other terms (FP8 codes), both >= 0 and in score units:
 * |s^ - s| <= kh hs + ks rs + 2^-24 (hs + rs) + A.  -1 for other contexts. */
double skm_error_bound_split(const skm_ctx *c, double hs, double rs, int64_t n_rest, double l1);

/* Index of threshold level `level` (Sec. 3.2), after an update with SKM_INDEX:
 * term-major lists.  offsets [n_cols + 1] (host int64), entries (host) of
 * (centroid << 16 | m) uint32 with m the minimum overlap count; each term's
 * list ascending by centroid.  Pass entries = NULL to get *n_entries only. */
skm_status skm_get_index(const skm_ctx *c, int32_t level, int64_t *offsets, uint32_t *entries,
                         int64_t *n_entries);

/* The value the index compares a centroid's prefix-sum differences of
 * squared sorted values against for threshold lambda (Sec. 3.2, Lemma 3.1:
 * "reaches" read as >=): lambda^2 less a bound on the FP64 rounding of those
 * differences for a centroid of n_entries non-zeros whose computed sum of
 * squares is q_total, so that every exact difference >= lambda^2 passes.
 * Host function, no context needed. */
double skm_index_threshold(double lambda, int64_t n_entries, double q_total);

/* Candidate sets of the Sec. 3.2 index at threshold level `level` for the rows
 * of docs (host CSR), without baselines: offsets [n_rows + 1] and cand
 * [cap] (host), each row's candidates ascending.  SKM_E_INVALID if cap is too
 * small (offsets[n_rows] then holds the size needed). */
skm_status skm_index_query(skm_ctx *c, const skm_csr *docs, int32_t level, int64_t *offsets,
                           int32_t *cand, int64_t cap);

/* ---------------------------------------------------------------- serving
 * Not part of the paper's method.  A request server keeps one context's
 * centroids resident and answers assign-new-rows requests (the exact
 * assignment of skm_assign_new) from many client threads, and runs small
 * clustering jobs beside them.
 *
 * Requests: a worker thread batches queued requests continuously: as soon as
 * one of its n_slots batch slots (each with its own stream and preallocated
 * device buffers) is free, it packs the requests at the head of the queue that
 * fit the slot's free rows and non-zeros and launches them; requests that
 * arrive while batches run join the next free slot, so transfers and kernels
 * of different batches overlap.  The slots are sized up front and their total
 * is held within hbm_budget_bytes.
 *
 * Jobs: a clustering job (its own rows and configuration) is admitted by
 * memory: it waits until the budget left by the slots and the running jobs
 * holds skm_context_bytes for it (and fewer than max_jobs run); a job thread
 * then runs the admitted jobs round robin, one iteration (assign, stop test,
 * update, stop test, as skm_iterate) per turn, on their own streams, beside the
 * request batches.  Each job's result is that of skm_init + skm_iterate on the
 * same rows and configuration.
 *
 * Answers are written into the caller's buffers by skm_server_wait when it
 * returns SKM_OK, never later.  While a server is attached, calls that change
 * the context (assign, update, iterate, set_centroids) return SKM_E_BUSY. */
typedef struct skm_server skm_server;

typedef struct {
  int32_t n_slots;          /* batches in flight, default 4 */
  int32_t slot_rows;        /* rows per batch, default 16384 */
  int64_t slot_nnz;         /* non-zeros per batch, default 4 Mi */
  size_t hbm_budget_bytes;  /* device memory cap for the slots and the jobs; n_slots
                               shrinks to fit (0 = none) */
  int32_t max_wait_us;      /* a partly filled batch waits at most this long for more rows
                               when no batch is running, default 100 */
  int32_t use_graphs;       /* 1 = each slot replays its compute pipeline as one captured
                               HIP graph (default); 0 = launch the kernels one by one */
  int32_t max_jobs;         /* clustering jobs run at once, default 2 (0 = none admitted) */
} skm_server_config;

typedef struct {
  int64_t requests_done;
  int64_t rows_done;
  int64_t batches;
  double p50_ms, p99_ms, mean_ms, max_ms;  /* request latency, submit to answers ready */
  double rows_per_s;        /* rows_done over first submit .. last completion */
  int32_t slots;            /* slots actually allocated */
  int32_t max_queue_depth;
  size_t hbm_bytes;         /* device memory held by the slots and the admitted jobs */
  int64_t jobs_done;        /* jobs finished (any status) */
  int64_t job_iterations;   /* iterations run by all jobs */
  int32_t jobs_running;
  int32_t jobs_queued;
} skm_server_stats;

/* Result counters of a clustering job. */
typedef struct {
  int32_t iterations;       /* iterations started, as skm_iterate's n_done */
  int32_t converged;        /* 1 if a stop test ended the job, 0 if max_iter did */
  double objective;         /* J_U = sum_j ||S_j|| after the last update */
  size_t hbm_bytes;         /* device memory the job was admitted with */
} skm_job_info;

void skm_server_config_default(skm_server_config *cfg);

/* Device memory skm_init and the following iterations may need for these rows
 * and this configuration, in bytes (an upper bound, used to admit jobs); 0 for
 * invalid arguments. */
size_t skm_context_bytes(const skm_csr *docs, const skm_config *cfg);

/* Starts a server on context c (which must outlive it). */
skm_status skm_server_start(skm_ctx *c, const skm_server_config *cfg, skm_server **out);

/* Queues the rows of docs (host CSR, copied and checked against the CSR
 * conventions above before return) for assignment; out_assign [n_rows] and
 * out_score [n_rows] are host buffers that skm_server_wait(ticket) fills when
 * it returns SKM_OK.  Thread-safe.  SKM_E_INVALID for a malformed CSR or one
 * larger than a slot. */
skm_status skm_server_submit(skm_server *s, const skm_csr *docs, int32_t *out_assign,
                             double *out_score, int64_t *ticket);

/* Queues a clustering job: docs (host CSR, copied before return; checked when
 * the job starts, as by skm_init) clustered with cfg (k, precision, flags,
 * stop rule, max_iter >= 1, init_rows required and copied; stream and budget
 * are ignored).  When skm_server_wait(ticket) returns SKM_OK it has written
 * the final assignment to out_assign [n_rows] (host), the FP64 centroids to
 * out_centroids [k * n_cols] (host, may be NULL) and the counters to *out_info
 * (may be NULL).  SKM_E_NOMEM when the job alone needs more memory than the
 * budget leaves beside the slots; errors of the job itself (SKM_E_INVALID for
 * its rows, SKM_E_NOMEM, SKM_E_DEVICE) are returned by the wait. */
skm_status skm_server_submit_job(skm_server *s, const skm_csr *docs, const skm_config *cfg,
                                 int32_t *out_assign, double *out_centroids,
                                 skm_job_info *out_info, int64_t *ticket);

/* Blocks until the request or job is answered (SKM_OK, or its error), or
 * timeout_s seconds pass (SKM_E_TIMEOUT; it stays queued and nothing is
 * written; timeout_s < 0 waits forever).  Each ticket is collected at most
 * once; SKM_E_CANCELLED for a cancelled one. */
skm_status skm_server_wait(skm_server *s, int64_t ticket, double timeout_s);

/* Cancels a request or job: a queued one is dropped, a batch in flight
 * finishes but its answers are discarded, a running job ends at its next
 * turn; nothing is written to the caller's buffers, and the request's rows
 * and answers are released.  A waiter (present or later) gets
 * SKM_E_CANCELLED, which collects the ticket.  SKM_E_INVALID for an unknown
 * ticket. */
skm_status skm_server_cancel(skm_server *s, int64_t ticket);

/* Latency and throughput counters since start. */
skm_status skm_server_get_stats(skm_server *s, skm_server_stats *out);

/* Answers every queued request, ends queued and running jobs as cancelled,
 * stops the worker threads, waits until every thread inside skm_server_wait
 * has returned and frees the server. */
skm_status skm_server_stop(skm_server *s);

/* Test aid for the error path (not part of the method): after n_calls more
 * checked HIP calls of this context (0 = the next one) one reports a launch
 * failure instead of being made, so the call that reaches it returns
 * SKM_E_DEVICE with the context poisoned, as after a real device error; no
 * fault happens on the device.  n_calls < 0 disarms it.  SKM_E_DEVICE on a
 * context that is already poisoned. */
skm_status skm_debug_fail_after(skm_ctx *c, int32_t n_calls);

/* Device memory the context currently holds, in bytes. */
size_t skm_hbm_bytes(const skm_ctx *c);

const char *skm_last_error(void);

void skm_destroy(skm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* SKM_H */
