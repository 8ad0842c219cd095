// Internal declarations of libskm: the context, kernel argument blocks and the
// launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace skm {

// Terms summed in LDS by the member-sum kernel (the most frequent ones).
constexpr int kSumHot = 2048;

// ------------------------------------------------------------ argument blocks

// Lists of non-zero codes of the tail terms of one scoring copy (see
// kernels_tail.hip).  tail == nullptr: every term takes the dense path.
// Bit 31 of a list offset word: the term is a list (rare) term of the chunk.
constexpr uint32_t kListFlag = 0x80000000u;
struct TailView {
  const uint8_t *tail;    // [nch][D] 1 = list term of chunk cc
  const uint32_t *off;    // [nch][D + 1] entry offsets within chunk cc's entries,
                          // kListFlag set on list terms (not on off[cc][D])
  const uint64_t *base;   // [nch + 1] first entry of chunk cc
  const uint32_t *ent;    // entries (BF16 / FP8: (col << 16) | code; FP32: (col, bits))
};

struct ScoreArgs {
  // rows
  const int64_t *indptr;
  const int32_t *indices;
  const float *values;
  const double *xl1;          // per-row L1 norm (FP8 absolute error term)
  int64_t n_rows;             // rows (and the row stride of the chunk partials)
  const int64_t *n_dev;       // rows actually present, read on the device (a captured
                              // graph replayed for batches of different sizes), or
                              // nullptr; launches are then sized for n_rows
  // rows the scoring kernel reads: the full rows, or only their terms outside
  // the dense head when head scores are given
  const int64_t *sc_indptr;
  const int32_t *sc_indices;
  const float *sc_values;
  // head scores (kernels_head.hip) of rows [row0, row0 + nb) and chunks
  // [c_first, c_first + c_count): hs[(row - row0) * hs_ld + column - 512 c_first],
  // or nullptr
  const float *hs;
  int64_t hs_ld;
  int64_t row0, nb;           // rows of this scoring launch: row0 .. row0 + nb, or
                              // row_list[row0 .. row0 + nb) when row_list is given
  const int32_t *row_list;
  int32_t c_first, c_count;   // 512-centroid chunks of this launch (items = c_count x nb)
  int32_t ncc_only;           // 1: rows whose previous centroid changed are left out
                              // (a second launch over their list scores them)
  int32_t head_H;             // head terms in the partial scores' bound (0: none)
  int32_t top;                // partial format: 2 = scores, kTop = certified bounds (FP8)
  // scoring copy, chunk-blocked term-major (see tile_index)
  const uint8_t *tile;
  int64_t D;
  int32_t k;
  const float *scale;         // per-centroid scale (FP8) or nullptr
  // Sec. 3.1: rows whose previous centroid is unchanged score the compacted
  // copy of the changed centroids and keep the previous one as a candidate
  const int32_t *a_prev;      // nullptr: no NCC
  const uint8_t *changed;
  const uint8_t *tile_ch;
  int32_t n_ch;
  const int32_t *ch_ids;
  TailView tv;                // tail lists of the full copy
  TailView tv_ch;             // tail lists of the compacted copy
  const double *prev_lo;
  const double *prev_hi;
  // Sec. 3.2: per-row candidate lists (nullptr: no index)
  const int64_t *cand_off;    // [n_rows + 1]; a row with cand_off[i] < 0 marker uses the dense path
  const int32_t *cand;
  const uint8_t *mode;        // 2 = row finished by the index path (skip), or nullptr
  // bound
  double uq;
  double abs_coef;
  int32_t no_exact;
  // outputs
  int32_t *a_out;
  double *lo_out;
  double *hi_out;
  int32_t *flag_rows;
  double *flag_L;
  uint8_t *flag_mode;         // 0 dense all, 1 NCC, 2 candidate list
  int32_t *counters;          // [0] flagged rows, [1] band overflows
  unsigned long long *stat;   // [0] centroids scored, [1] NCC rows, [2] index rows,
                              // [3] products, [8] products of the sparse pass (head on)
};

// Summary of one row against one 512-centroid chunk; -inf where the chunk has
// fewer columns.  top = 2 (FP32 / BF16): e[0] = best score (higher score,
// then lower centroid index) and the score of the second best in e[1].s; the
// merge derives both bounds from the scores.  top = kTop (FP8, whose head and
// sparse parts carry different bounds): certified bounds per column, e[0] =
// the best lower bound and its column, e[1].s = that column's upper bound,
// e[2], e[3] = the two largest upper bounds and their columns.
constexpr int kTop = 4;
struct __align__(16) Partial {
  struct {
    float s;
    int32_t j;
  } e[kTop];
};

struct ExactArgs {
  ScoreArgs s;
  const Partial *part;        // [chunk][row] partials of the scoring pass
  const double *master;       // k x D FP64 centroids
  int64_t D;
  int32_t max_waves;
};

// Device buffers of one batch of new rows (assignment without clustering).
struct NewRows {
  const int64_t *indptr;
  const int32_t *indices;
  const float *values;
  const double *xl1;
  Partial *part;
  int32_t *a;
  double *lo, *hi;
  int32_t *flag_rows;
  double *flag_L;
  uint8_t *flag_mode;
  int32_t *counters;
  unsigned long long *stat;
  double *score;
  const uint8_t *mode = nullptr;   // [n] 2 = row already assigned (index path), or nullptr
};

// Support bitmaps of the update (bit t of a cluster's row: entry t is
// non-zero), so that clusters summed straight into their sum row are
// renormalised and requantised over their non-zeros only
// (kernels_update.hip).
struct SumSupport {
  int64_t W = 0;                     // 32-bit words per cluster row
  uint32_t *nb = nullptr;            // [k][W] support of S_j built by this update's sums
};

struct RenormSupport {
  int64_t W = 0;
  const uint32_t *nb = nullptr;      // [k][W] support of S_j (this update)
  uint32_t *mb = nullptr;            // [k][W] support of the master row c_j
  uint8_t *mvalid = nullptr;         // [k] mb_j is exact
  uint8_t *qmask = nullptr;          // [k] out: changed, left to k_quantize
  uint8_t *tile = nullptr;           // scoring copy (written for the sparse path)
  float *scale = nullptr;            // FP8 scales (written for the sparse path)
};

// Device pieces of the Sec. 3.2 index.
struct IndexBuild {
  const double *master;
  int32_t k;
  int64_t D;
  const int64_t *sstart; // [k] first entry of each centroid's segment
  const int32_t *cnt;    // [k] entries (non-zeros) per centroid
  const int64_t *qstart; // [k] first prefix sum of each centroid (cnt + 1 of them)
  uint64_t *key0, *key1; // sort keys (~bits of the value), ping-pong
  int32_t *term0, *term1;
  double *Q;             // prefix sums of squares
  uint64_t *mask;        // [D][ceil(k/64)] non-zero masks (build scratch)
  int32_t *blkpre;       // [D][ceil(k/64)] per-term prefix of mask popcounts (scratch)
  int32_t *tcnt;         // [D] centroids per term (scratch)
  int64_t *toff;         // [D + 1] G offsets
  uint2 *G;              // (centroid, position) per (term, centroid)
};

struct IndexArgs {
  const int64_t *indptr;
  const int32_t *indices;
  const float *values;
  const double *xl2;
  const double *master;
  int64_t D;
  int32_t k;
  const int32_t *rows;      // rows handled, one workgroup each (nullptr: slot = row)
  const int32_t *a_prev;    // previous assignment (baseline), or nullptr
  const uint8_t *changed;   // Sec. 3.1 changed flags: rows keeping an unchanged
                            // previous centroid only take changed candidates
                            // (nullptr: no filter)
  int32_t n_ch;             // changed centroids (cost guard of those rows)
  const int64_t *toff;
  const uint2 *G;
  const int32_t *cnt;       // entries per centroid
  const int64_t *qstart;    // first prefix sum per centroid
  const double *Q;
  int32_t n_dirty;          // centroids rebuilt since the last full build (0: no G2)
  const uint32_t *dbits;    // [ceil(k / 32)] their bitmap
  const int64_t *toff2;     // [D + 1] G2 offsets
  const uint2 *G2;          // (centroid, position) of the dirty centroids, term-major
  double lambda[8];
  int32_t n_lambda;
  int32_t forced_level;     // >= 0: use this level, no baseline, no cost guard
  double guard;             // max query reads as a fraction of nnz * k
  int32_t cap;              // candidate slots per row
  int32_t *cand;            // [slots][cap]
  int32_t *ncand;           // [slots], -1 = dense path
  int32_t *level;           // [slots]
  uint8_t *mode;            // [n_rows] 2 = finished by the index path, or nullptr
  unsigned long long *stat; // [0] scored, [2] index rows, [3] products, [5] no level,
                            // [6] guard, [7] over cap
  double *base_out;         // [slots] certified lower bound of the baseline, or nullptr
};

// Index threshold.
// The index (Sec. 3.2) compares differences of FP64 prefix sums of a
// centroid's sorted squared values, Q[h] - Q[p], against lam^2 ("reaches the
// threshold" read as >=).  The prefix sums of a centroid with n entries are
// computed by 256 threads (kernels_index.hip, k_prefix_sq): each thread sums
// a chunk of per = ceil(n / 256) squares, a 256-wide scan of 8 rounds adds the
// chunks, one subtraction turns the inclusive scan into the chunk's offset,
// and the chunk's squares are added to it one by one.  Every square therefore
// reaches any prefix through at most m = 2 per + 20 roundings (per + 1 in its
// chunk, 8 in the scan, 1 subtraction, per in the running sum, plus the
// subtraction's carried scan error, counted as 9 more), all on sums of
// non-negative terms, so |Q^[i] - Q[i]| <= g_m S with g_m = m u / (1 - m u),
// u = 2^-53 and S the exact total; the difference adds its own rounding,
// |fl(Q^[h] - Q^[p]) - (Q[h] - Q[p])| <= (2 g_m + 2 u) S.  The threshold is
// lam^2 less that bound (with S <= Q^[n] / (1 - g_m)) and less 4u for the
// rounding of lam^2 and of the subtraction itself, inflated by 2^-20: an
// exact difference >= lam^2 always passes, so the candidate set can only
// grow.  q_total is the computed Q^[n].
__host__ __device__ inline double index_threshold(double lam, int64_t n, double q_total) {
  const double u = 0x1p-53;
  const double m = 2.0 * (double)((n + 255) / 256) + 20.0;
  const double g = m * u / (1.0 - m * u);
  const double S = q_total / (1.0 - g);
  const double E = ((2.0 * g + 2.0 * u) * S + 4.0 * u) * (1.0 + 0x1p-20);
  return lam * lam - E;
}

// LDS of the index query: k positions (4 B) and k 16-bit counts.
__host__ __device__ inline size_t index_lds_bytes(int32_t k) {
  return sizeof(uint32_t) * ((size_t)k + ((size_t)k + 1) / 2 + ((size_t)k + 31) / 32);
}

}  // namespace skm

struct skm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool poisoned = false;
  int32_t fail_after = -1;     // test aid: checked HIP calls left before an injected failure
  skm_config cfg{};

  int64_t N = 0, D = 0, Z = 0;
  int32_t k = 0;
  int64_t ld = 0;      // tile row stride (centroid columns, padded)
  int prec = SKM_FP32;
  int esize = 4;       // bytes per scoring code
  double uq = 0, abs_coef = 0;

  size_t hbm_bytes = 0;
  std::vector<void *> allocations;

  // rows (CSR) and per-row constants
  int64_t *indptr = nullptr;
  int32_t *indices = nullptr;
  float *values = nullptr;
  double *xl1 = nullptr;
  double *xl2 = nullptr;

  // centroids
  double *master = nullptr;    // k x D FP64, unit rows
  double *S = nullptr;         // k x D FP64 member sums (rows of changed clusters)
  uint8_t *tile = nullptr;     // ld / 512 chunks of D x 512 codes (tile_index)
  float *scale = nullptr;      // [ld]
  double *snorm = nullptr;     // ||S_j|| of the current membership
  double *shift = nullptr;     // per-cluster ||dc||^2 of the last update
  double *dot_old = nullptr;   // S_j . c_j(old) of the last update
  uint8_t *changed = nullptr;  // k flags
  int32_t *ch_ids = nullptr;   // compacted changed ids (ascending)
  int32_t n_ch = 0;
  uint8_t *tile_ch = nullptr;  // compacted copy of the changed centroids, same layout

  // assignment state
  int32_t *a = nullptr;        // current assignment
  int32_t *a_prev = nullptr;   // assignment that produced the current centroids
  double *lo = nullptr, *hi = nullptr;   // certified interval of x_i . c_{a_i}
  double *lo_prev = nullptr, *hi_prev = nullptr;  // the same for a_prev

  // scratch
  int32_t *flag_rows = nullptr;
  double *flag_L = nullptr;
  uint8_t *flag_mode = nullptr;
  int32_t *counters = nullptr;
  unsigned long long *stat = nullptr;
  int32_t *hist = nullptr;     // [nblk][k]
  int32_t *counts = nullptr;   // [k]
  int64_t *offsets = nullptr;  // [k + 1]
  int32_t *members = nullptr;  // [N]
  double *red = nullptr;       // reduction outputs
  int32_t *ids_count = nullptr;
  skm::Partial *part = nullptr;  // [ceil(k / 512)][N] scoring partials
  // tail lists: [0] of the full copy, [1] of the compacted (NCC) copy
  struct Tail {
    uint8_t *tail = nullptr;     // [nch][D] 1 = list term in chunk cc
    uint32_t *cnt = nullptr, *off = nullptr, *ent = nullptr;
    uint32_t *totals = nullptr;  // [nch] entries per listed chunk (last build)
    uint32_t *bsum = nullptr;    // [nch][tail_scan_blocks(D)] scan scratch
    int32_t *chunks = nullptr;   // [nch] chunk list of the last build
    uint64_t *base = nullptr;    // [nch + 1] = cc * stride
    int64_t stride = 0;          // entries reserved per chunk
    std::vector<int64_t> h_total;  // entries per chunk, host copy
    bool ready = false;
  } tails[2];
  bool use_tail = true;
  uint8_t *mode = nullptr;       // [N] 2 = row finished by the index path
  // Sec. 3.2 index (built when SKM_INDEX is set)
  bool index_ready = false;
  int64_t idx_cap_entries = 0;   // capacity of the entry-sized buffers
  int64_t idx_g_entries = 0;     // entries of G (last full build)
  int64_t idx_used_e = 0, idx_used_q = 0;  // entry / prefix-sum slots in use
  int32_t *idx_cnt = nullptr;    // [k] entries per centroid
  int64_t *idx_sstart = nullptr, *idx_qstart = nullptr;  // [k] segment, prefix-sum starts
  int64_t *idx_tot = nullptr;    // [2] totals of the last placement
  uint64_t *idx_key0 = nullptr, *idx_key1 = nullptr;
  int32_t *idx_term0 = nullptr, *idx_term1 = nullptr;
  double *idx_Q = nullptr;
  uint2 *idx_G = nullptr;
  uint64_t *idx_mask = nullptr;
  int32_t *idx_blkpre = nullptr, *idx_tcnt = nullptr;
  int64_t *idx_toff = nullptr;
  // centroids rebuilt since the last full build ("dirty") and their G2
  uint8_t *idx_dirty = nullptr;  // [k]
  int32_t *idx_dids = nullptr;   // [k] dirty ids
  uint32_t *idx_dbits = nullptr; // [ceil(k / 32)]
  int64_t *idx_toff2 = nullptr;  // [D + 1]
  uint2 *idx_G2 = nullptr;       // [idx_cap_entries / 4 + 1024]
  int2 *idx_runs = nullptr, *idx_tiles = nullptr;  // sort work lists [cap / run + k]
  std::vector<int2> idx_h_runs, idx_h_tiles;
  std::vector<int32_t> idx_h_cnt;     // host copy of idx_cnt
  std::vector<uint8_t> idx_h_dirty;   // host copy of idx_dirty
  std::vector<int32_t> idx_h_dids;    // host copy of idx_dids
  int32_t idx_last_build = 0;    // 0 none, 1 full, 2 changed centroids only
  int32_t *idx_best = nullptr;   // [D] centroid largest at each term (new rows' probes)
  bool idx_best_ready = false;   // idx_best is that of the current index (under best_mu)
  std::mutex best_mu;            // concurrent skm_assign_new calls build idx_best once
  std::atomic<int64_t> new_index_rows{0};  // rows the index assigned in the last
                                           // skm_assign_new to finish
  int32_t *idx_rows = nullptr, *idx_cand = nullptr, *idx_ncand = nullptr, *idx_level = nullptr;
  int32_t idx_cap = 128;
  double idx_guard = 0.25;
  // dynamic enabling: a probe that decides fewer than 5 % of the eligible rows
  // turns the index off for idx_backoff iterations (doubling up to 64)
  int32_t idx_skip = 0;
  int32_t idx_backoff = 8;
  int32_t idx_skip_pre = 0, idx_backoff_pre = 8;  // the two above when the last assign began
  float ms_index_build = 0.f;
  int64_t idx_eligible = 0;
  int server_attached = 0;     // a request server reads this context
  // dense head on the matrix cores (kernels_head.hip); head_H = 0: off
  int32_t head_H = 0;
  int32_t k_pad = 0;             // head-code rows (k rounded up to 512)
  int64_t head_rows = 0;         // rows per head batch
  int32_t head_chunks = 0;       // 512-centroid chunks per head batch
  int64_t hs_cap = 0;            // floats in hs (head_rows x head_chunks x 512 at most)
  int32_t score_wpc = 0;         // scoring grid workgroups per CU (0 = as many as fit)
  // event pairs around the launches of one step (device time per kernel):
  // the head GEMMs and the sparse scoring kernel
  struct EventPairs {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
  } head_t, sparse_t;
  double head_pairs = 0;         // (row, centroid) pairs the head GEMMs of one step computed
  int32_t *head_terms = nullptr; // [H] term ids, ascending
  int32_t *head_slot = nullptr;  // [D] slot of a head term, -1 otherwise
  int32_t *sum_hot_slot = nullptr;   // [D] LDS slot of a term in the member sums, -1 otherwise
  int32_t *sum_hot_terms = nullptr;  // [n_sum_hot] the kSumHot most frequent terms, ascending
  int32_t n_sum_hot = 0;
  uint16_t *xh = nullptr;        // [N][H] BF16 head values of the rows
  uint16_t *ch_head = nullptr;   // [k_pad][H] BF16 head codes of the centroids
  uint16_t *ch_head_ch = nullptr; // the same for the changed centroids, compacted (NCC)
  int32_t *full_rows = nullptr;  // [N] rows whose previous centroid changed (NCC)
  int32_t *ncc_list = nullptr;   // [N] rows whose previous centroid is unchanged (NCC)
  int32_t *list_work = nullptr;  // row-list compaction workspace
  double full_frac = 1.0;        // share of rows whose centroid changed in the last update
  float *hs = nullptr;           // [head_rows][k_pad] head scores of one batch
  int64_t *r_indptr = nullptr;   // remainder CSR: the rows' non-head terms
  int32_t *r_indices = nullptr;
  float *r_values = nullptr;
  // segmented member sums of large clusters
  int4 *tasks = nullptr;         // [task cap]
  int64_t *task_r0 = nullptr;    // [task cap]
  int4 *groups = nullptr;        // [k]
  int64_t task_cap = 0;
  double *work = nullptr;        // [work_slots][D] partial sums
  int64_t work_slots = 0;
  int n_cu = 256;                // compute units (the persistent scoring grid is sized from it)
  int64_t nblk = 0;             // blocks of the update's counting sort
  // support bitmaps of the update (RenormSupport)
  int64_t sup_W = 0;             // 32-bit words per cluster row
  uint32_t *sup_nb = nullptr, *sup_mb = nullptr;          // [k][sup_W]
  uint8_t *sup_mvalid = nullptr, *sup_qmask = nullptr;  // [k]
  int64_t bucket_rows = 8192;   // rows per block (bucket_rows())

  // state
  int32_t iter = 0;            // completed updates
  bool assigned = false;       // an assignment is pending an update
  bool have_prev = false;      // a_prev / changed are meaningful for NCC
  bool force_all = true;       // next update recomputes every cluster
  int32_t last_changed = 0;    // changed centroids before the last assignment
  int64_t last_moved = 0;

  hipEvent_t ev[10] = {};
  float ms_full_score = -1.f;  // device time of the last scoring pass over every centroid
  float ms_full_assign = -1.f; // device time of the last assignment without Sec. 3.1
  float ms_ncc_fixed = -1.f;   // last Sec. 3.1 assignment's time beyond its scaled scoring
};

namespace skm {

// kernels_score.hip
// n_cu: compute units of the device; the grid holds as many workgroups as fit
// on them at once.
// wpc: workgroups per CU of the persistent scoring grid (0 = as many as fit).
hipError_t launch_score(const ScoreArgs &a, Partial *part, int n_cu, int prec, hipStream_t s,
                        int wpc = 0);
// The two halves of launch_score: partials of rows [a.row0, a.row0 + a.nb),
// then the merge and certificate of all a.n_rows rows.
hipError_t launch_score_part(const ScoreArgs &a, Partial *part, int n_cu, int prec, hipStream_t s,
                             int wpc = 0);
// Sec. 3.1 rows keeping their centroid against at most kNarrowMax compacted
// changed centroids (a.tile_ch, a.n_ch, a.ch_ids), all terms, no head scores:
// partials of compacted chunk 0; the other rows are left untouched.
constexpr int kNarrowMax = 64;
// Sec. 3.1 is used when its estimated share of a full scoring pass is at most
// this (the compacted copy and the two passes cost the rest).
constexpr double kNccMaxCost = 0.9;
hipError_t launch_score_narrow(const ScoreArgs &a, Partial *part, int prec, hipStream_t s);
// Workgroups of the scoring kernel that fit on one CU at once.
int score_occupancy(int prec);
hipError_t launch_finalize(const ScoreArgs &a, const Partial *part, hipStream_t s);
hipError_t launch_exact(const ExactArgs &a, int prec, hipStream_t s);
hipError_t launch_score_dense(const int64_t *indptr, const int32_t *indices, const float *values,
                              int64_t n_rows, const uint8_t *tile, int64_t D, int32_t k,
                              const float *scale, const TailView &tv, int prec, const float *hs,
                              int64_t hs_ld, float *out, hipStream_t s,
                              float *out_head = nullptr);
hipError_t launch_exact_scores(const int64_t *indptr, const int32_t *indices, const float *values,
                               int64_t n_rows, const int32_t *a, const double *master, int64_t D,
                               double *out, hipStream_t s, const int64_t *n_dev = nullptr);

// api.hip
// n rows of new rows; with n_dev the launches are sized for n rows of
// capacity and the kernels read the actual count from *n_dev.
hipError_t launch_new_rows(skm_ctx *c, const NewRows &b, int64_t n, hipStream_t s,
                           const int64_t *n_dev = nullptr);
skm_status set_error(skm_status st, const std::string &msg);  // thread-local last error

// noalloc.hip: looks up the static workspace's device address on `device`
// (the current device), once per device.
skm_status noalloc_setup(int device);

// kernels_tail.hip
// Chunks chunks[0 .. n_list) of a copy with ncols columns: classification,
// counts and per-chunk offsets (totals[q] = entries of chunks[q]); then the
// entries, chunk cc's from entry cc * stride.
hipError_t tail_count(const uint8_t *tile, int64_t D, int32_t ncols, int prec,
                      const int32_t *chunks, int32_t n_list, uint32_t *cnt, uint8_t *tail,
                      uint32_t *off, uint32_t *totals, uint32_t *bsum, hipStream_t s);
int64_t tail_scan_blocks(int64_t D);   // bsum entries per listed chunk
hipError_t tail_fill(const uint8_t *tile, int64_t D, int32_t ncols, int prec,
                     const int32_t *chunks, int32_t n_list, const uint8_t *tail,
                     const uint32_t *off, int64_t stride, uint32_t *ent, hipStream_t s);
hipError_t tail_bases(uint64_t *base, int32_t nch, int64_t stride, hipStream_t s);

// k-means++ seeding (kernels_seed.hip), one seed per place/weights/select.
hipError_t pp_place(const int64_t *indptr, const int32_t *indices, const float *values, int64_t n,
                    const int32_t *rows, int32_t m, double *dense, double *nrm2, hipStream_t s);
hipError_t pp_weights(const int64_t *indptr, const int32_t *indices, const float *values,
                      int64_t n, const double *dense, double nrm, double *best,
                      const uint8_t *chosen, uint64_t *w, uint64_t *bsum, hipStream_t s);
hipError_t pp_select(const uint64_t *bsum, const uint64_t *w, int64_t n, uint64_t draw,
                     uint8_t *chosen, int32_t *rows, int32_t m, hipStream_t s);

// kernels_index.hip
hipError_t index_counts(const double *master, int32_t k, int64_t D, const int32_t *ids,
                        int32_t n, int32_t *cnt, hipStream_t s);
hipError_t index_place(const int32_t *ids, int32_t n, const int32_t *cnt, int64_t base_e,
                       int64_t base_q, int64_t *sstart, int64_t *qstart, int64_t *tot,
                       hipStream_t s);
// Segments of the n listed centroids (all when ids is nullptr): extraction,
// sort and prefix sums.  runs: (centroid, first entry) of every run of
// index_run_len() entries of the listed segments with more than one entry;
// tiles: the same for the segments longer than one run; max_len: their
// longest segment.
int32_t index_run_len();
hipError_t index_segments(const IndexBuild &ib, const int32_t *ids, int32_t n, const int2 *runs,
                          int64_t n_runs, const int2 *tiles, int64_t n_tiles, int64_t max_len,
                          hipStream_t s);
hipError_t index_terms(const IndexBuild &ib, hipStream_t s);
hipError_t index_delta(const IndexBuild &ib, const int32_t *dirty_ids, int32_t n_dirty,
                       const uint8_t *dirty, int64_t *toff2, uint2 *G2, uint32_t *dbits,
                       hipStream_t s);
// Ascending list of the rows whose previous centroid is flagged in `changed`
// (keep = 0) or not flagged (keep = 1), all rows when changed is nullptr,
// leaving out rows the index finished (mode[i] == 2) when mode is given, and
// its length; `work` holds index_rows_work(n) int32 values.
int64_t index_rows_work(int64_t n);
hipError_t index_rows(const int32_t *a_prev, const uint8_t *changed, int64_t n, int32_t *rows,
                      int32_t *count, int32_t *work, hipStream_t s, int32_t keep = 0,
                      const uint8_t *mode = nullptr);
hipError_t index_query(const IndexArgs &x, int64_t n_slots, hipStream_t s);
// best[t]: the centroid largest at term t (-1: none), from the built index.
hipError_t index_best_centroid(const IndexArgs &x, const uint8_t *dirty, const int64_t *sstart,
                               const uint64_t *key, int32_t *best, hipStream_t s);
// probe[i]: a new row's probe centroid (baseline of its index query).
hipError_t index_probe(const int64_t *indptr, const int32_t *indices, const float *values,
                       int64_t n, const int32_t *best, const double *master, int64_t D,
                       int32_t *probe, hipStream_t s);
hipError_t index_score(const IndexArgs &x, int64_t n_slots, int32_t *a_out, double *lo_out,
                       double *hi_out, hipStream_t s);

// kernels_update.hip
hipError_t launch_row_stats_only(const int64_t *indptr, const int32_t *indices, const float *values,
                                 int64_t n_rows, double *xl1, hipStream_t s,
                                 const int64_t *n_dev = nullptr);
hipError_t launch_row_stats(const int64_t *indptr, const int32_t *indices, const float *values,
                            int64_t n_rows, int64_t D, double *xl1, double *xl2, int32_t *bad,
                            hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_seed(const int64_t *indptr, const int32_t *indices, const float *values,
                       const int32_t *rows, int32_t k, int64_t D, double *master, hipStream_t s);
hipError_t launch_fp8_scales(const double *master, int32_t k, int64_t D, const uint8_t *changed,
                             float *scale, hipStream_t s);
hipError_t launch_quantize(const double *master, int32_t k, int64_t D, const uint8_t *changed,
                           const float *scale, int prec, uint8_t *tile, hipStream_t s);
hipError_t launch_count_moved(const int32_t *a, const int32_t *a_prev, int64_t n,
                              unsigned long long *out, hipStream_t s);
hipError_t launch_mark_changed(const int32_t *a, const int32_t *a_prev, int64_t n, uint8_t *changed,
                               hipStream_t s);
hipError_t launch_compact_changed(const uint8_t *changed, int32_t k, int32_t *ids, int32_t *count,
                                  hipStream_t s);
hipError_t launch_gather_tile(const uint8_t *tile, int64_t D, int esize, const int32_t *ids,
                              int32_t n, uint8_t *out, hipStream_t s);
hipError_t launch_centroid_columns(const double *master, int32_t k, int64_t D, const int32_t *terms,
                                   int32_t n, double *out, hipStream_t s);
hipError_t launch_bucket(const int32_t *a, int64_t n, int32_t k, int64_t blk, int32_t *hist,
                         int32_t *counts, int64_t *offsets, int32_t *members, hipStream_t s);
// Rows per block of the update's counting sort: blocks are walked by one
// wavefront each, so more of them help, but the per-(block, cluster) counts
// cost blocks x k: about 5e6 counts, 1,024 to 8,192 rows a block.
inline int64_t bucket_rows(int64_t N, int64_t k) {
  const int64_t target = std::min<int64_t>(2048, std::max<int64_t>(128, 5000000 / std::max<int64_t>(k, 1)));
  const int64_t blk = ((N + target - 1) / target + 255) / 256 * 256;
  return std::min<int64_t>(8192, std::max<int64_t>(1024, blk));
}
// Member sums of the tasks; terms with hot_slot[t] >= 0 (n_hot <= kSumHot of
// them, hot_terms[slot] = t) are summed in LDS.  short_rows: the corpus has
// short rows, summed several rows per step (when D < 2^24).
hipError_t launch_sum_tasks(const int64_t *indptr, const int32_t *indices, const float *values,
                            const int32_t *members, const int4 *tasks, const int64_t *task_r0,
                            int32_t n_tasks, int64_t D, double *S, double *work,
                            const int32_t *hot_slot, const int32_t *hot_terms, int32_t n_hot,
                            hipStream_t s, bool short_rows, SumSupport sp);
hipError_t launch_combine(const int4 *groups, int32_t n_groups, int64_t D, const double *work,
                          double *S, uint32_t *nb, int64_t W, hipStream_t s);
// Renormalisation of the n_ids listed clusters (see k_renorm).
hipError_t launch_renorm(double *S, const int32_t *counts, const int32_t *ids, int32_t n_ids,
                         int64_t D, double *master, double *snorm, double *shift, double *dot_old,
                         const RenormSupport &rs, int prec, hipStream_t s);
hipError_t launch_reduce_stats(const uint8_t *changed, const double *snorm, const double *shift,
                               const double *dot_old, int32_t k, double *out, hipStream_t s);

// kernels_head.hip
hipError_t launch_df(const int32_t *indices, int64_t nnz, uint32_t *df, int64_t D, hipStream_t s);
int64_t head_split_scan_blocks(int64_t n_rows);
hipError_t launch_head_split(const int64_t *indptr, const int32_t *indices, const float *values,
                             int64_t n_rows, const int32_t *slot, int32_t H, int64_t *cnt,
                             int64_t *scan_work, int64_t *r_indptr, int32_t *r_indices,
                             float *r_values, uint16_t *xh, hipStream_t s);
hipError_t launch_head_codes(const uint8_t *tile, const double *master, const float *scale,
                             int64_t D, int32_t k, int prec, const int32_t *terms, int32_t H,
                             int32_t k_pad, uint16_t *ch, hipStream_t s);
// hs[r][j] = sum_h xh[x_r][h] * ch[col0 + j][h], r < nb, j < ncols, where
// x_r = row0 + r, or rows[row0 + r] when rows is given (ncols a multiple of
// 256, col0 + ncols <= rows of ch).
hipError_t launch_head_gemm(const uint16_t *xh, int32_t H, int64_t row0, int64_t nb,
                            const int32_t *rows, const uint16_t *ch, int64_t col0, int64_t ncols,
                            float *hs, int64_t ldh, hipStream_t s);
// out[o][:] = ch[ids[o]][:] for o < n (rows of H BF16 codes).
hipError_t launch_gather_head(const uint16_t *ch, int32_t H, const int32_t *ids, int32_t n,
                              uint16_t *out, hipStream_t s);

}  // namespace skm
