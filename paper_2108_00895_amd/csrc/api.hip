// The C ABI of libskm (declared in include/skm.h): context lifetime, HBM
// accounting, the assignment / update / iterate state machine, and the
// getters used by tests.  Every step of the method runs in the kernels of
// kernels_score.hip and kernels_update.hip; this file only sequences them.
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "host_checks.h"
#include "internal.h"

using namespace skm;

namespace {

thread_local std::string g_err;

skm_status fail(skm_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

skm_status device_fail(skm_ctx *c, const char *what, hipError_t e) {
  if (c) c->poisoned = true;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return SKM_E_DEVICE;
}

// Test aid (skm_debug_fail_after): the armed call reports a launch failure
// instead of being made.
bool injected(skm_ctx *c) {
  if (!c || c->fail_after < 0) return false;
  return c->fail_after-- == 0;
}

#define HIP_TRY(c, expr)                                                        \
  do {                                                                          \
    hipError_t _e = injected(c) ? hipErrorLaunchFailure : (expr);               \
    if (_e != hipSuccess) return device_fail(c, #expr, _e);                     \
  } while (0)

#define ST_TRY(expr)                \
  do {                              \
    skm_status _s = (expr);         \
    if (_s != SKM_OK) return _s;    \
  } while (0)

template <typename T>
skm_status dalloc(skm_ctx *c, T **p, size_t count) {
  size_t bytes = round_up((int64_t)std::max<size_t>(count * sizeof(T), 1), 256);
  if (c->cfg.hbm_budget_bytes && c->hbm_bytes + bytes > c->cfg.hbm_budget_bytes)
    return fail(SKM_E_NOMEM, "HBM budget exceeded: need " + std::to_string(c->hbm_bytes + bytes) +
                                 " bytes, budget " + std::to_string(c->cfg.hbm_budget_bytes));
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return fail(SKM_E_NOMEM, "device out of memory allocating " + std::to_string(bytes) + " bytes");
  }
  if (e != hipSuccess) return device_fail(c, "hipMalloc", e);
  c->allocations.push_back(q);
  c->hbm_bytes += bytes;
  *p = static_cast<T *>(q);
  return SKM_OK;
}

// Frees one allocation made by dalloc.
void dfree(skm_ctx *c, void *p, size_t count_bytes) {
  if (!p) return;
  auto it = std::find(c->allocations.begin(), c->allocations.end(), p);
  if (it != c->allocations.end()) c->allocations.erase(it);
  (void)hipFree(p);
  c->hbm_bytes -= round_up((int64_t)std::max<size_t>(count_bytes, 1), 256);
}

double unit_roundoff(int prec) {
  switch (prec) {
    case SKM_FP32: return 0x1p-24;
    case SKM_BF16: return 0x1p-8;
    default: return 0x1p-4;
  }
}

int code_bytes(int prec) { return prec == SKM_FP32 ? 4 : (prec == SKM_BF16 ? 2 : 1); }

// Absolute error term of the encoding per unit of a row's L1 norm.  FP8 codes
// below 2^-6 are subnormal with spacing 2^-9, so a value can be off by half of
// that times the centroid's scale; scales are at most 2^-8 because centroid
// entries are at most 1 (unit rows) and the scale is the least power of two
// with max <= 448 * scale.  FP32 / BF16 only lose values below 2^-126.
double abs_coefficient(int prec) {
  const double uq = unit_roundoff(prec);
  if (prec == SKM_FP8_E4M3) return 0x1p-8 * 0x1p-10 / (1.0 - uq) * (1.0 + 0x1p-20);
  return 0x1p-120;
}

// The shape and pointers of a CSR description (host_checks.cpp).
skm_status check_csr_header(const skm_csr *d, int64_t max_cols) {
  std::string why;
  bool unsupported = false;
  if (!host::csr_header_ok(d, max_cols, &unsupported, &why))
    return fail(unsupported ? SKM_E_UNSUPPORTED : SKM_E_INVALID, why);
  return SKM_OK;
}

// indptr must be checked before any kernel walks rows.
skm_status check_indptr(const int64_t *ip, int64_t n, int64_t nnz) {
  std::string why;
  if (!host::indptr_ok(ip, n, nnz, &why)) return fail(SKM_E_INVALID, why);
  return SKM_OK;
}

struct DevRows {
  int64_t *indptr = nullptr;
  int32_t *indices = nullptr;
  float *values = nullptr;
  double *xl1 = nullptr, *xl2 = nullptr;
};

// Copies (host or device) rows into context-owned or temporary device memory
// and computes per-row norms; checks the CSR conventions on the device.
template <typename Alloc>
skm_status upload_rows(skm_ctx *c, const skm_csr *d, int64_t D, bool validate, hipStream_t s,
                       Alloc alloc, DevRows *out, bool borrow = false) {
  const int64_t n = d->n_rows, z = d->nnz;
  std::vector<int64_t> ip_host;
  const int64_t *ip = d->indptr;
  if (d->on_device) {
    ip_host.resize(n + 1);
    HIP_TRY(c, hipMemcpyAsync(ip_host.data(), d->indptr, sizeof(int64_t) * (n + 1),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    ip = ip_host.data();
  }
  ST_TRY(check_indptr(ip, n, z));
  if (borrow && d->on_device) {
    // the caller's device arrays are used in place (read only)
    out->indptr = const_cast<int64_t *>(d->indptr);
    out->indices = const_cast<int32_t *>(d->indices);
    out->values = const_cast<float *>(d->values);
  } else {
    ST_TRY(alloc(&out->indptr, (size_t)(n + 1) * sizeof(int64_t)));
    ST_TRY(alloc(&out->indices, (size_t)std::max<int64_t>(z, 1) * sizeof(int32_t)));
    ST_TRY(alloc(&out->values, (size_t)std::max<int64_t>(z, 1) * sizeof(float)));
    const hipMemcpyKind kind = d->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(c, hipMemcpyAsync(out->indptr, d->indptr, sizeof(int64_t) * (n + 1), kind, s));
    if (z > 0) {
      HIP_TRY(c, hipMemcpyAsync(out->indices, d->indices, sizeof(int32_t) * z, kind, s));
      HIP_TRY(c, hipMemcpyAsync(out->values, d->values, sizeof(float) * z, kind, s));
    }
  }
  ST_TRY(alloc(&out->xl1, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
  ST_TRY(alloc(&out->xl2, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
  int32_t *bad = nullptr;
  ST_TRY(alloc(&bad, sizeof(int32_t)));
  HIP_TRY(c, launch_fill_i32(bad, 0, 1, s));
  HIP_TRY(c, launch_row_stats(out->indptr, out->indices, out->values, n, D, out->xl1, out->xl2, bad,
                              s));
  int32_t hbad = 0;
  HIP_TRY(c, hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (hbad & 4) return fail(SKM_E_INVALID, "term index out of range [0, n_cols)");
  if (validate) {
    if (hbad & 2) return fail(SKM_E_INVALID, "values must be finite and > 0");
    if (hbad & 8) return fail(SKM_E_INVALID, "indices must be strictly ascending within a row");
    if (hbad & 32) return fail(SKM_E_INVALID, "empty row");
    if (hbad & 16) return fail(SKM_E_INVALID, "row L2 norm differs from 1 by more than 1e-5");
  }
  return SKM_OK;
}

skm_status check_ctx(const skm_ctx *c) {
  if (!c) return fail(SKM_E_INVALID, "context is NULL");
  if (c->poisoned) return fail(SKM_E_DEVICE, "context is poisoned by an earlier device error");
  return SKM_OK;
}

// Calls that change the clustering state are refused while a server reads it.
skm_status check_ctx_writable(const skm_ctx *c) {
  ST_TRY(check_ctx(c));
  if (c->server_attached) return fail(SKM_E_BUSY, "a request server is attached to this context");
  return SKM_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

int ent_words(int prec) { return prec == SKM_FP32 ? 2 : 1; }

// Tail lists (kernels_tail.hip) of copy `which` (0 full, 1 compacted) with
// ncols columns.  `chunks` (ascending) lists the chunks whose codes changed
// since the last build, nullptr = all; the other chunks keep their lists.
// Each chunk owns `stride` entries of the entry buffer; when a chunk outgrows
// it the buffer is reallocated with 25 % headroom and every chunk refilled.
skm_status build_tail(skm_ctx *c, int which, const uint8_t *tile, int32_t ncols,
                      const std::vector<int32_t> *chunks) {
  skm_ctx::Tail &T = c->tails[which];
  const bool was_ready = T.ready;
  T.ready = false;
  if (!c->use_tail || ncols <= 0) return SKM_OK;
  hipStream_t s = c->stream;
  const int32_t nch = (ncols + kChunk - 1) / kChunk;
  const int32_t nch_max = (c->k + kChunk - 1) / kChunk;
  std::vector<int32_t> all(nch);
  for (int32_t q = 0; q < nch; ++q) all[q] = q;
  const bool partial = chunks && was_ready && (int32_t)T.h_total.size() == nch;
  const std::vector<int32_t> &list = partial ? *chunks : all;
  T.h_total.resize(nch, 0);
  const int32_t n = (int32_t)list.size();
  if (n > 0) {
    std::vector<uint32_t> tot(n);
    HIP_TRY(c, hipMemcpyAsync(T.chunks, list.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(c, tail_count(tile, c->D, ncols, c->prec, T.chunks, n, T.cnt, T.tail, T.off, T.totals,
                          T.bsum, s));
    HIP_TRY(c, hipMemcpyAsync(tot.data(), T.totals, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    for (int32_t q = 0; q < n; ++q) T.h_total[list[q]] = tot[q];
  }
  int64_t need = 0;
  for (int64_t v : T.h_total) need = std::max(need, v);
  need *= ent_words(c->prec);
  const std::vector<int32_t> *fill = &list;
  if (need > T.stride) {
    if (T.ent) dfree(c, T.ent, sizeof(uint32_t) * T.stride * nch_max);
    T.ent = nullptr;
    T.stride = 0;
    const int64_t stride = std::max<int64_t>(need + need / 4, 1024);
    ST_TRY(dalloc(c, &T.ent, (size_t)(stride * nch_max)));
    T.stride = stride;
    HIP_TRY(c, tail_bases(T.base, nch_max, stride / ent_words(c->prec), s));
    if (partial && n != nch) {
      HIP_TRY(c, hipMemcpyAsync(T.chunks, all.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice,
                                s));
      fill = &all;
    }
  }
  HIP_TRY(c, tail_fill(tile, c->D, ncols, c->prec, T.chunks, (int32_t)fill->size(), T.tail, T.off,
                       T.stride / ent_words(c->prec), T.ent, s));
  if (fill == &all && partial) HIP_TRY(c, hipStreamSynchronize(s));   // `all` leaves scope
  T.ready = true;
  return SKM_OK;
}

TailView tail_view(const skm_ctx *c, int which) {
  const skm_ctx::Tail &T = c->tails[which];
  if (!T.ready) return TailView{nullptr, nullptr, nullptr, nullptr};
  return TailView{T.tail, T.off, T.base, T.ent};
}

// Scoring copies of the centroids flagged in `changed` (all when nullptr),
// and the full copy's tail lists (of the chunks in `chunks` when given).
skm_status rebuild_tiles(skm_ctx *c, const uint8_t *changed,
                         const std::vector<int32_t> *chunks, const uint8_t *qmask = nullptr) {
  // qmask: the changed centroids whose codes k_renorm has not written
  const uint8_t *q = qmask ? qmask : changed;
  if (c->prec == SKM_FP8_E4M3)
    HIP_TRY(c, launch_fp8_scales(c->master, c->k, c->D, q, c->scale, c->stream));
  HIP_TRY(c, launch_quantize(c->master, c->k, c->D, q, c->scale, c->prec, c->tile, c->stream));
  ST_TRY(build_tail(c, 0, c->tile, c->k, changed ? chunks : nullptr));
  if (c->head_H > 0)
    HIP_TRY(c, launch_head_codes(c->tile, c->master, c->scale, c->D, c->k, c->prec, c->head_terms,
                                 c->head_H, c->k_pad, c->ch_head, c->stream));
  return SKM_OK;
}

// The dense head (kernels_head.hip): the terms contained in at least
// head_min_df of the rows, most frequent first, at most head_max_terms, padded
// to a multiple of 64 with the next most frequent terms.  Builds the rows'
// BF16 head block and the remainder CSR once (the rows never change).  The
// head stays off for FP32 scoring, when fewer than 64 terms qualify, or when
// its buffers would not fit the HBM budget.
// Document frequency of every term (rows containing it), on the host.
skm_status term_df(skm_ctx *c, std::vector<uint32_t> &df) {
  df.assign(c->D, 0u);
  if (c->Z == 0) return SKM_OK;
  hipStream_t s = c->stream;
  uint32_t *d_df = nullptr;
  ST_TRY(dalloc(c, &d_df, (size_t)c->D));
  hipError_t e = launch_df(c->indices, c->Z, d_df, c->D, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(df.data(), d_df, sizeof(uint32_t) * c->D, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(c, d_df, sizeof(uint32_t) * c->D);
  if (e != hipSuccess) return device_fail(c, "term df", e);
  return SKM_OK;
}

// The kSumHot most frequent terms (ties: lower id), whose member sums the
// update accumulates in LDS.
skm_status setup_sum_hot(skm_ctx *c, const std::vector<uint32_t> &df) {
  std::vector<int32_t> order;
  for (int64_t t = 0; t < c->D; ++t)
    if (df[t] > 0) order.push_back((int32_t)t);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return df[x] > df[y]; });
  if ((int64_t)order.size() > kSumHot) order.resize(kSumHot);
  std::sort(order.begin(), order.end());
  c->n_sum_hot = 0;
  if (order.empty()) return SKM_OK;
  std::vector<int32_t> slot(c->D, -1);
  for (size_t h = 0; h < order.size(); ++h) slot[order[h]] = (int32_t)h;
  ST_TRY(dalloc(c, &c->sum_hot_slot, (size_t)c->D));
  ST_TRY(dalloc(c, &c->sum_hot_terms, order.size()));
  hipStream_t s = c->stream;
  HIP_TRY(c, hipMemcpyAsync(c->sum_hot_slot, slot.data(), sizeof(int32_t) * c->D,
                            hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->sum_hot_terms, order.data(), sizeof(int32_t) * order.size(),
                            hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->n_sum_hot = (int32_t)order.size();
  return SKM_OK;
}

skm_status setup_head(skm_ctx *c, const std::vector<uint32_t> &df) {
  c->head_H = 0;
  if (c->prec == SKM_FP32 || c->cfg.head_max_terms < 64 || c->Z == 0) return SKM_OK;
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;

  const double thr = std::max(1.0, std::ceil(c->cfg.head_min_df * (double)c->N));
  std::vector<int32_t> order;
  int64_t n_pos = 0, n_qual = 0;
  for (int64_t t = 0; t < c->D; ++t) {
    if (df[t] == 0) continue;
    ++n_pos;
    if ((double)df[t] >= thr) ++n_qual;
  }
  int64_t H = round_up(n_qual, 64);
  H = std::min<int64_t>(H, (c->cfg.head_max_terms / 64) * 64);
  H = std::min<int64_t>(H, (n_pos / 64) * 64);
  if (H < 64) return SKM_OK;
  order.reserve(n_pos);
  for (int64_t t = 0; t < c->D; ++t)
    if (df[t] > 0) order.push_back((int32_t)t);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return df[x] > df[y]; });
  order.resize(H);
  std::sort(order.begin(), order.end());
  std::vector<int32_t> slot(c->D, -1);
  int64_t head_nnz = 0;
  for (int64_t h = 0; h < H; ++h) {
    slot[order[h]] = (int32_t)h;
    head_nnz += df[order[h]];
  }
  const int64_t rest_nnz = c->Z - head_nnz;
  const int32_t k_pad = (int32_t)round_up(c->k, kChunk);
  // head scores of one batch: up to 4 chunks (2048 centroids) of up to 2^20
  // rows, 8 GiB at most
  const int32_t chunks = (int32_t)std::min<int64_t>(4, k_pad / kChunk);
  const int64_t rows = std::min<int64_t>(1ll << 20, round_up(c->N, 256));
  const int64_t nscan = head_split_scan_blocks(c->N);
  const size_t need = 4 * (size_t)H + 4 * (size_t)c->D + 2 * (size_t)c->N * H +
                      2 * (size_t)k_pad * H * ((c->cfg.flags & SKM_NCC) ? 2 : 1) +
                      4 * (size_t)rows * chunks * kChunk +
                      4 * (size_t)c->N * (((c->cfg.flags & SKM_NCC) ? 1 : 0) +
                                          ((c->cfg.flags & (SKM_NCC | SKM_INDEX)) ? 1 : 0)) +
                      8 * (size_t)(c->N + 1) +
                      8 * (size_t)rest_nnz + 8 * (size_t)c->N + 8 * (size_t)nscan + 16 * 256;
  if (c->cfg.hbm_budget_bytes && c->hbm_bytes + need > c->cfg.hbm_budget_bytes) return SKM_OK;

  ST_TRY(dalloc(c, &c->head_terms, (size_t)H));
  ST_TRY(dalloc(c, &c->head_slot, (size_t)c->D));
  ST_TRY(dalloc(c, &c->xh, (size_t)c->N * H));
  ST_TRY(dalloc(c, &c->ch_head, (size_t)k_pad * H));
  if (c->cfg.flags & SKM_NCC) {
    ST_TRY(dalloc(c, &c->ch_head_ch, (size_t)k_pad * H));
    ST_TRY(dalloc(c, &c->ncc_list, (size_t)c->N));
  }
  if (c->cfg.flags & (SKM_NCC | SKM_INDEX)) ST_TRY(dalloc(c, &c->full_rows, (size_t)c->N));
  ST_TRY(dalloc(c, &c->hs, (size_t)rows * chunks * kChunk));
  ST_TRY(dalloc(c, &c->r_indptr, (size_t)c->N + 1));
  ST_TRY(dalloc(c, &c->r_indices, (size_t)std::max<int64_t>(rest_nnz, 1)));
  ST_TRY(dalloc(c, &c->r_values, (size_t)std::max<int64_t>(rest_nnz, 1)));
  int64_t *cnt = nullptr, *work = nullptr;
  ST_TRY(dalloc(c, &cnt, (size_t)c->N));
  ST_TRY(dalloc(c, &work, (size_t)nscan));
  e = hipMemcpyAsync(c->head_terms, order.data(), sizeof(int32_t) * H, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->head_slot, slot.data(), sizeof(int32_t) * c->D, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_head_split(c->indptr, c->indices, c->values, c->N, c->head_slot, (int32_t)H, cnt,
                          work, c->r_indptr, c->r_indices, c->r_values, c->xh, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(c, cnt, sizeof(int64_t) * c->N);
  dfree(c, work, sizeof(int64_t) * nscan);
  if (e != hipSuccess) return device_fail(c, "head split", e);
  c->head_H = (int32_t)H;
  c->k_pad = k_pad;
  c->head_rows = rows;
  c->head_chunks = chunks;
  c->hs_cap = rows * chunks * kChunk;
  return SKM_OK;
}

ScoreArgs base_args(skm_ctx *c) {
  ScoreArgs a{};
  a.indptr = c->indptr;
  a.indices = c->indices;
  a.values = c->values;
  a.xl1 = c->xl1;
  a.n_rows = c->N;
  a.n_dev = nullptr;
  a.sc_indptr = c->indptr;
  a.sc_indices = c->indices;
  a.sc_values = c->values;
  a.hs = nullptr;
  a.hs_ld = 0;
  a.row0 = 0;
  a.nb = c->N;
  a.c_first = 0;
  a.c_count = (int32_t)((c->k + kChunk - 1) / kChunk);
  a.row_list = nullptr;
  a.ncc_only = 0;
  a.head_H = 0;
  a.top = c->prec == SKM_FP8_E4M3 ? kTop : 2;
  a.tile = c->tile;
  a.D = c->D;
  a.k = c->k;
  a.scale = c->prec == SKM_FP8_E4M3 ? c->scale : nullptr;
  a.uq = c->uq;
  a.abs_coef = c->abs_coef;
  a.no_exact = (c->cfg.flags & SKM_NO_EXACT) ? 1 : 0;
  a.tv = tail_view(c, 0);
  a.tv_ch = TailView{nullptr, nullptr, nullptr, nullptr};
  a.a_out = c->a;
  a.lo_out = c->lo;
  a.hi_out = c->hi;
  a.flag_rows = c->flag_rows;
  a.flag_L = c->flag_L;
  a.flag_mode = c->flag_mode;
  a.counters = c->counters;
  a.stat = c->stat;
  return a;
}

int exact_waves() { return 4096; }

constexpr int64_t kSegRows = 256;       // least members per summation segment
constexpr int64_t kWorkBytes = 16ll << 30;  // partial-row workspace cap

// Rows shorter than this on average are summed several rows per step.
constexpr int64_t kShortRow = 32;

bool short_rows(int64_t N, int64_t Z) { return Z <= kShortRow * N; }

// Members per summation segment: kSegRows, or for corpora of short rows
// (summed several rows per step) as many rows as make about 256 steps of 256
// entries, so that a segment's own adds stay comparable to the D-entry
// workspace row it clears and the combine reads back (with a large
// vocabulary and short rows that row would otherwise cost hundreds of times
// the adds).  A function of the corpus shape alone, so a cluster's segments
// (and its FP64 sum) depend only on its member set.
int64_t seg_rows_for(int64_t N, int64_t D, int64_t Z) {
  (void)D;
  if (!short_rows(N, Z) || Z <= 0) return kSegRows;
  return std::max<int64_t>(kSegRows, (int64_t(1) << 16) * N / Z);
}

// Workspace rows any update can need: the segments of the clusters with more
// than seg members number at most N / (seg / 2) + 1 (each such cluster has at
// most count / seg + 1 of them), within kWorkBytes.
int64_t work_slots_bound(const skm_ctx *c) {
  const int64_t max_slots = std::max<int64_t>(1, kWorkBytes / (8 * c->D));
  const int64_t seg = seg_rows_for(c->N, c->D, c->Z);
  return std::min<int64_t>(max_slots, c->N / (seg / 2) + 2);
}

// FP64 member sums of the n_ids changed clusters (ids in c->ch_ids): clusters
// with at most seg_rows_for members are summed by one workgroup each; larger
// ones are split into segments summed in parallel into workspace rows and
// combined in segment order.  Rounds keep the workspace within kWorkBytes.
skm_status sum_changed(skm_ctx *c, int32_t n_ids, std::vector<int32_t> &ids) {
  ids.clear();
  c->full_frac = 0.0;
  if (n_ids <= 0) return SKM_OK;
  hipStream_t s = c->stream;
  ids.resize(n_ids);
  std::vector<int32_t> counts(c->k);
  std::vector<int64_t> offs(c->k + 1);
  HIP_TRY(c, hipMemcpyAsync(ids.data(), c->ch_ids, 4 * n_ids, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(counts.data(), c->counts, 4 * c->k, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(offs.data(), c->offsets, 8 * (c->k + 1), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  int64_t n_full = 0;   // rows of the changed clusters: they score every centroid next time
  for (int32_t j : ids) n_full += counts[j];
  c->full_frac = c->N > 0 ? (double)n_full / (double)c->N : 0.0;
  // workspace rows: at most kWorkBytes, and within the HBM budget when one is
  // set (one slot means every cluster is summed by a single workgroup)
  int64_t work_cap = kWorkBytes;
  if (c->cfg.hbm_budget_bytes) {
    const int64_t held = c->work ? (int64_t)round_up(c->work_slots * 8 * c->D, 256) : 0;
    work_cap = std::min<int64_t>(work_cap, std::max<int64_t>(
                   0, (int64_t)c->cfg.hbm_budget_bytes - c->hbm_bytes + held));
  }
  const int64_t max_slots = std::max<int64_t>(1, work_cap / (8 * c->D));
  const int64_t seg_rows = seg_rows_for(c->N, c->D, c->Z);
  size_t pos = 0;
  std::vector<int4> tasks, groups;
  std::vector<int64_t> r0s;
  while (pos < ids.size()) {
    tasks.clear();
    groups.clear();
    r0s.clear();
    int64_t slots = 0;
    for (; pos < ids.size(); ++pos) {
      const int32_t j = ids[pos];
      const int64_t cnt = counts[j];
      const int64_t nseg =
          std::min<int64_t>(max_slots, std::max<int64_t>(1, (cnt + seg_rows - 1) / seg_rows));
      const int64_t seg = nseg > 0 ? (cnt + nseg - 1) / nseg : cnt;
      if (nseg == 1) {
        tasks.push_back(make_int4(j, (int)cnt, -1, 0));
        r0s.push_back(offs[j]);
        continue;
      }
      if (slots + nseg > max_slots && slots > 0) break;   // next round
      groups.push_back(make_int4(j, (int)slots, (int)nseg, 0));
      for (int64_t g = 0; g < nseg; ++g) {
        const int64_t r0 = offs[j] + g * seg;
        const int64_t len = std::max<int64_t>(0, std::min<int64_t>(seg, offs[j] + cnt - r0));
        tasks.push_back(make_int4(j, (int)len, (int)(slots + g), 0));
        r0s.push_back(r0);
      }
      slots += nseg;
    }
    if ((int64_t)tasks.size() > c->task_cap) {
      const int64_t cap = std::max<int64_t>((int64_t)tasks.size() * 2, 1024);
      if (c->tasks) dfree(c, c->tasks, c->task_cap * sizeof(int4));
      if (c->task_r0) dfree(c, c->task_r0, c->task_cap * sizeof(int64_t));
      c->tasks = nullptr;
      c->task_r0 = nullptr;
      c->task_cap = 0;
      ST_TRY(dalloc(c, &c->tasks, (size_t)cap));
      ST_TRY(dalloc(c, &c->task_r0, (size_t)cap));
      c->task_cap = cap;
    }
    if (slots > c->work_slots) {
      // Only under an HBM budget (without one, skm_init allocates the bound).
      // A multi-GB hipMalloc can take seconds: grow to the bound at once
      // unless the budget leaves less.
      const int64_t want = std::max<int64_t>(slots, std::min<int64_t>(max_slots,
                                                                    work_slots_bound(c)));
      if (c->work) dfree(c, c->work, c->work_slots * 8 * c->D);
      c->work = nullptr;
      c->work_slots = 0;
      ST_TRY(dalloc(c, &c->work, (size_t)(want * c->D)));
      c->work_slots = want;
    }
    if (!c->groups) ST_TRY(dalloc(c, &c->groups, (size_t)c->k));
    HIP_TRY(c, hipMemcpyAsync(c->tasks, tasks.data(), sizeof(int4) * tasks.size(),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->task_r0, r0s.data(), 8 * r0s.size(), hipMemcpyHostToDevice, s));
    if (!groups.empty())
      HIP_TRY(c, hipMemcpyAsync(c->groups, groups.data(), sizeof(int4) * groups.size(),
                                hipMemcpyHostToDevice, s));
    SumSupport sp;
    sp.W = c->sup_W;
    sp.nb = c->sup_nb;
    HIP_TRY(c, launch_sum_tasks(c->indptr, c->indices, c->values, c->members, c->tasks, c->task_r0,
                                (int32_t)tasks.size(), c->D, c->S, c->work, c->sum_hot_slot,
                                c->sum_hot_terms, c->n_sum_hot, s, short_rows(c->N, c->Z), sp));
    HIP_TRY(c, launch_combine(c->groups, (int32_t)groups.size(), c->D, c->work, c->S, c->sup_nb,
                              c->sup_W, s));
    // the host vectors are reused next round: wait for the copies to finish
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return SKM_OK;
}

// Entry-sized buffers of the index (keys and terms twice for the sort, prefix
// sums, G, and G2 for a quarter of them): 42 bytes per entry (plus 16 per
// centroid).
skm_status alloc_index_entries(skm_ctx *c, int64_t cap) {
  const int64_t old = c->idx_cap_entries;
  dfree(c, c->idx_key0, old * 8);
  dfree(c, c->idx_key1, old * 8);
  dfree(c, c->idx_term0, old * 4);
  dfree(c, c->idx_term1, old * 4);
  dfree(c, c->idx_Q, (old + 2 * (int64_t)c->k) * 8);
  dfree(c, c->idx_G, old * 8);
  dfree(c, c->idx_G2, (old / 4 + 1024) * 8);
  dfree(c, c->idx_runs, (old / index_run_len() + c->k + 1) * 8);
  dfree(c, c->idx_tiles, (old / index_run_len() + c->k + 1) * 8);
  c->idx_runs = c->idx_tiles = nullptr;
  c->idx_key0 = c->idx_key1 = nullptr;
  c->idx_term0 = c->idx_term1 = nullptr;
  c->idx_Q = nullptr;
  c->idx_G = c->idx_G2 = nullptr;
  c->idx_cap_entries = 0;
  c->index_ready = false;
  ST_TRY(dalloc(c, &c->idx_key0, (size_t)cap));
  ST_TRY(dalloc(c, &c->idx_key1, (size_t)cap));
  ST_TRY(dalloc(c, &c->idx_term0, (size_t)cap));
  ST_TRY(dalloc(c, &c->idx_term1, (size_t)cap));
  ST_TRY(dalloc(c, &c->idx_Q, (size_t)(cap + 2 * (int64_t)c->k)));
  ST_TRY(dalloc(c, &c->idx_G, (size_t)cap));
  ST_TRY(dalloc(c, &c->idx_G2, (size_t)(cap / 4 + 1024)));
  ST_TRY(dalloc(c, &c->idx_runs, (size_t)(cap / index_run_len() + c->k + 1)));
  ST_TRY(dalloc(c, &c->idx_tiles, (size_t)(cap / index_run_len() + c->k + 1)));
  c->idx_cap_entries = cap;
  return SKM_OK;
}

IndexBuild index_build_args(skm_ctx *c) {
  return IndexBuild{c->master,     c->k,         c->D,         c->idx_sstart, c->idx_cnt,
                    c->idx_qstart, c->idx_key0,  c->idx_key1,  c->idx_term0,  c->idx_term1,
                    c->idx_Q,      c->idx_mask,  c->idx_blkpre, c->idx_tcnt,  c->idx_toff,
                    c->idx_G};
}

// Extracts, sorts and sums the segments of the listed centroids (all when ids
// is nullptr), whose counts are in idx_h_cnt: the sort's work lists (runs of
// every segment, merge tiles of the long ones) are built here.
skm_status index_segments_of(skm_ctx *c, const int32_t *ids_dev, const std::vector<int32_t> *ids) {
  const int32_t R = index_run_len();
  std::vector<int2> &runs = c->idx_h_runs, &tiles = c->idx_h_tiles;
  runs.clear();
  tiles.clear();
  int64_t max_len = 0;
  auto add = [&](int32_t j) {
    const int32_t n = c->idx_h_cnt[j];
    if (n > 1)
      for (int32_t y = 0; y < n; y += R) runs.push_back(make_int2(j, y));
    if (n > R) {
      for (int32_t y = 0; y < n; y += R) tiles.push_back(make_int2(j, y));
      max_len = std::max<int64_t>(max_len, n);
    }
  };
  if (ids) {
    for (int32_t j : *ids) add(j);
  } else {
    for (int32_t j = 0; j < c->k; ++j) add(j);
  }
  hipStream_t s = c->stream;
  if (!runs.empty())
    HIP_TRY(c, hipMemcpyAsync(c->idx_runs, runs.data(), sizeof(int2) * runs.size(),
                              hipMemcpyHostToDevice, s));
  if (!tiles.empty())
    HIP_TRY(c, hipMemcpyAsync(c->idx_tiles, tiles.data(), sizeof(int2) * tiles.size(),
                              hipMemcpyHostToDevice, s));
  const int32_t n = ids ? (int32_t)ids->size() : c->k;
  HIP_TRY(c, index_segments(index_build_args(c), ids_dev, n, c->idx_runs, (int64_t)runs.size(),
                            c->idx_tiles, (int64_t)tiles.size(), max_len, s));
  return SKM_OK;
}

// Sec. 3.2 index from the current master.  With the changed centroids of the
// last update (ids, ascending, device and host copies) and an index that was
// valid before it, only those centroids are rebuilt (segments appended, G2
// over every centroid rebuilt since the last full build); otherwise, or when
// the rebuilt centroids hold more than a quarter of all entries or the
// buffers are full, everything is rebuilt and compacted.  Entry-sized buffers
// grow on demand (by half again, so that a growing run reallocates only a
// few times); without an HBM budget skm_init reserves min(nnz, k D) entries
// up to 16 GiB at once.
skm_status build_index(skm_ctx *c, const int32_t *ids_dev = nullptr,
                       const std::vector<int32_t> *ids = nullptr) {
  hipStream_t s = c->stream;
  const int32_t k = c->k;
  HIP_TRY(c, hipEventRecord(c->ev[6], s));
  {
    std::lock_guard<std::mutex> lock(c->best_mu);
    c->idx_best_ready = false;
  }
  c->idx_h_cnt.resize(k, 0);
  c->idx_h_dirty.resize(k, 0);
  const bool can_delta = ids && ids_dev && c->index_ready && c->idx_cap_entries > 0 &&
                         4 * (int64_t)ids->size() <= (int64_t)k;
  c->index_ready = false;
  bool full = !can_delta;
  if (!full) {
    const int32_t n = (int32_t)ids->size();
    if (n > 0) {
      HIP_TRY(c, index_counts(c->master, k, c->D, ids_dev, n, c->idx_cnt, s));
      HIP_TRY(c, index_place(ids_dev, n, c->idx_cnt, c->idx_used_e, c->idx_used_q, c->idx_sstart,
                             c->idx_qstart, c->idx_tot, s));
      int64_t tot[2] = {0, 0};
      HIP_TRY(c, hipMemcpyAsync(tot, c->idx_tot, sizeof(tot), hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipMemcpyAsync(c->idx_h_cnt.data(), c->idx_cnt, sizeof(int32_t) * k,
                                hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipStreamSynchronize(s));
      for (int32_t j : *ids)
        if (!c->idx_h_dirty[j]) {
          c->idx_h_dirty[j] = 1;
          c->idx_h_dids.push_back(j);
        }
      int64_t live = 0, dirty = 0;
      for (int32_t j = 0; j < k; ++j) live += c->idx_h_cnt[j];
      for (int32_t j : c->idx_h_dids) dirty += c->idx_h_cnt[j];
      if (c->idx_used_e + tot[0] > c->idx_cap_entries ||
          c->idx_used_q + tot[1] > c->idx_cap_entries + 2 * (int64_t)k || 4 * dirty > live) {
        full = true;
      } else {
        const IndexBuild ib = index_build_args(c);
        ST_TRY(index_segments_of(c, ids_dev, ids));
        c->idx_used_e += tot[0];
        c->idx_used_q += tot[1];
        std::sort(c->idx_h_dids.begin(), c->idx_h_dids.end());
        const int32_t nd = (int32_t)c->idx_h_dids.size();
        HIP_TRY(c, hipMemcpyAsync(c->idx_dids, c->idx_h_dids.data(), sizeof(int32_t) * nd,
                                  hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(c->idx_dirty, c->idx_h_dirty.data(), k, hipMemcpyHostToDevice, s));
        HIP_TRY(c, index_delta(ib, c->idx_dids, nd, c->idx_dirty, c->idx_toff2, c->idx_G2,
                               c->idx_dbits, s));
        c->idx_last_build = 2;
      }
    } else {
      c->idx_last_build = 2;
    }
  }
  if (full) {
    HIP_TRY(c, index_counts(c->master, k, c->D, nullptr, k, c->idx_cnt, s));
    HIP_TRY(c, index_place(nullptr, k, c->idx_cnt, 0, 0, c->idx_sstart, c->idx_qstart, c->idx_tot,
                           s));
    int64_t tot[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(tot, c->idx_tot, sizeof(tot), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(c->idx_h_cnt.data(), c->idx_cnt, sizeof(int32_t) * k,
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const int64_t total = tot[0];
    if (total > c->idx_cap_entries) {
      const int64_t bound = std::min<int64_t>(c->Z, (int64_t)k * c->D);
      const int64_t cap = std::max<int64_t>(std::min<int64_t>(total + total / 2, bound), total);
      ST_TRY(alloc_index_entries(c, std::max<int64_t>(cap, 1024)));
    }
    const IndexBuild ib = index_build_args(c);
    ST_TRY(index_segments_of(c, nullptr, nullptr));
    HIP_TRY(c, index_terms(ib, s));
    std::fill(c->idx_h_dirty.begin(), c->idx_h_dirty.end(), 0);
    c->idx_h_dids.clear();
    c->idx_used_e = total;
    c->idx_used_q = tot[1];
    c->idx_g_entries = total;
    c->idx_last_build = 1;
  }
  HIP_TRY(c, hipEventRecord(c->ev[7], s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->index_ready = true;
  c->ms_index_build = elapsed(c->ev[6], c->ev[7]);
  return SKM_OK;
}

IndexArgs index_args(skm_ctx *c) {
  IndexArgs x{};
  x.indptr = c->indptr;
  x.indices = c->indices;
  x.values = c->values;
  x.xl2 = c->xl2;
  x.master = c->master;
  x.D = c->D;
  x.k = c->k;
  x.rows = c->idx_rows;
  x.a_prev = c->a_prev;
  x.toff = c->idx_toff;
  x.G = c->idx_G;
  x.cnt = c->idx_cnt;
  x.qstart = c->idx_qstart;
  x.Q = c->idx_Q;
  x.n_dirty = (int32_t)c->idx_h_dids.size();
  x.dbits = c->idx_dbits;
  x.toff2 = c->idx_toff2;
  x.G2 = c->idx_G2;
  for (int i = 0; i < 8; ++i) x.lambda[i] = c->cfg.lambda[i];
  x.n_lambda = c->cfg.n_lambda;
  x.forced_level = -1;
  x.guard = c->idx_guard;
  x.cap = c->idx_cap;
  x.cand = c->idx_cand;
  x.ncand = c->idx_ncand;
  x.level = c->idx_level;
  x.mode = c->mode;
  x.stat = c->stat;
  return x;
}

}  // namespace

namespace skm {

skm_status set_error(skm_status st, const std::string &msg) { return fail(st, msg); }

// Exact assignment of rows that are not part of the clustering (no NCC, no
// index): low-precision scoring with certification, the FP64 exact tier for
// uncertain rows, and the FP64 score of the chosen centroid.  Enqueues only.
hipError_t launch_new_rows(skm_ctx *c, const NewRows &b, int64_t n, hipStream_t s,
                           const int64_t *n_dev) {
  ScoreArgs sa = base_args(c);
  sa.n_dev = n_dev;
  sa.indptr = b.indptr;
  sa.indices = b.indices;
  sa.values = b.values;
  sa.xl1 = b.xl1;
  sa.n_rows = n;
  sa.sc_indptr = b.indptr;
  sa.sc_indices = b.indices;
  sa.sc_values = b.values;
  sa.nb = n;
  sa.c_first = 0;
  sa.c_count = (int32_t)((c->k + kChunk - 1) / kChunk);
  sa.a_out = b.a;
  sa.lo_out = b.lo;
  sa.hi_out = b.hi;
  sa.flag_rows = b.flag_rows;
  sa.flag_L = b.flag_L;
  sa.flag_mode = b.flag_mode;
  sa.counters = b.counters;
  sa.stat = b.stat;
  sa.no_exact = 0;
  sa.mode = b.mode;
  hipError_t e = launch_fill_i32(b.counters, 0, 8, s);
  if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t *>(b.stat), 0, 16, s);
  if (e == hipSuccess) e = launch_score(sa, b.part, c->n_cu, c->prec, s, c->score_wpc);
  if (e == hipSuccess) {
    ExactArgs x{sa, b.part, c->master, c->D, exact_waves()};
    e = launch_exact(x, c->prec, s);
  }
  if (e == hipSuccess)
    e = launch_exact_scores(b.indptr, b.indices, b.values, n, b.a, c->master, c->D, b.score, s,
                            n_dev);
  return e;
}

}  // namespace skm

extern "C" {

void skm_config_default(skm_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->precision = SKM_FP32;
  cfg->head_max_terms = 4096;
  cfg->head_min_df = 1.0 / 128.0;
  cfg->n_lambda = 4;
  cfg->lambda[0] = 0.1;
  cfg->lambda[1] = 0.25;
  cfg->lambda[2] = 0.4;
  cfg->lambda[3] = 0.6;
  cfg->index_min_changed = 0;
  cfg->stop_rule = SKM_STOP_PAPER;
  cfg->max_iter = 100;
  cfg->min_moved_frac = 0.0;
  cfg->max_shift_sq = 1e-4;
  cfg->validate = 1;
}

const char *skm_last_error(void) { return g_err.c_str(); }

skm_status skm_debug_fail_after(skm_ctx *c, int32_t n_calls) {
  ST_TRY(check_ctx(c));
  c->fail_after = n_calls < 0 ? -1 : n_calls;
  return SKM_OK;
}

double skm_index_threshold(double lambda, int64_t n_entries, double q_total) {
  return index_threshold(lambda, n_entries, q_total);
}

size_t skm_hbm_bytes(const skm_ctx *c) { return c ? c->hbm_bytes : 0; }

void skm_destroy(skm_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void *p : c->allocations) (void)hipFree(p);
  for (hipEvent_t &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto *t : {&c->head_t, &c->sparse_t})
    for (hipEvent_t &e : t->ev)
      if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  (void)hipGetLastError();
  delete c;
}

size_t skm_context_bytes(const skm_csr *docs, const skm_config *cfg) {
  if (!docs || !cfg || docs->n_rows < 1 || docs->n_cols < 1 || docs->nnz < 0 || cfg->k < 1 ||
      cfg->precision < SKM_FP32 || cfg->precision > SKM_FP8_E4M3)
    return 0;
  // An upper bound of what skm_init allocates and what the iterations may
  // grow to, for the allocations of this file (each rounded up to 256 bytes).
  const double N = (double)docs->n_rows, D = (double)docs->n_cols, Z = (double)docs->nnz;
  const double k = (double)cfg->k;
  const double ld = (double)round_up(cfg->k, kChunk), nch = ld / kChunk;
  const double esize = (double)code_bytes(cfg->precision);
  const bool ncc = cfg->flags & SKM_NCC, index = cfg->flags & SKM_INDEX;
  const bool borrow = (cfg->flags & SKM_BORROW_DEVICE) && docs->on_device;
  double b = 0;
  if (!borrow) b += 8 * (N + 1) + 8 * Z;                      // rows
  b += 16 * N;                                                 // norms
  b += 16 * k * D + D * ld * esize * (ncc ? 2 : 1);            // master, sums, codes
  b += 8 * k * std::ceil(D / 32) + 2 * k;                      // support bitmaps
  b += 4 * ld + 48 * k + 8 * (k + 1);                          // scales, per-centroid state
  b += N * (4 + 4 + 8 * 4 + 4 + 8 + 1 + 4);                    // per-row state, members
  b += 4 * std::ceil(N / (double)bucket_rows(docs->n_rows, cfg->k)) * k +
       sizeof(Partial) * nch * N;                              // histogram, partials
  if (!(cfg->flags & SKM_DENSE_ONLY))                          // list offsets, flags, counts
    b += (ncc ? 2 : 1) * nch * (9 * D + D / 1024 + 32);
  if (index) {
    const double nb = std::ceil(k / 64);
    b += N * (1 + 4 + 4 * 128 + 4 + 4) + 72 * (k + 1) + D * (12 * nb + 20);
  }
  // non-zeros of all centroids are at most min(Z, k D): index entries (42 B
  // each, 25 % headroom) and code lists (8 B each, per-chunk stride headroom)
  const double cnz = std::min(Z, k * D);
  if (index) b += 1.25 * 42 * cnz;
  if (!(cfg->flags & SKM_DENSE_ONLY)) b += (ncc ? 2 : 1) * 1.25 * 8 * std::min(cnz, nch * 512 * D);
  // the dense head (BF16 / FP8): at most head_max_terms terms
  if (cfg->precision != SKM_FP32 && cfg->head_max_terms >= 64) {
    const double H = std::min<double>((double)(cfg->head_max_terms / 64) * 64, D);
    const double rows = std::min<double>((double)(1 << 20), (double)round_up(docs->n_rows, 256));
    b += 4 * H + 8 * D + 2 * N * H + 2 * ld * H * (ncc ? 2 : 1) + 4 * rows * 4 * kChunk +
         4 * N * 2 + 8 * (N + 1) + 8 * Z + 16 * N;
  }
  // the update's workspace: the bound skm_init allocates without a budget
  b += 8 * D * (double)std::min<int64_t>(
                   std::max<int64_t>(1, kWorkBytes / (8 * docs->n_cols)),
                   docs->n_rows / (seg_rows_for(docs->n_rows, docs->n_cols, docs->nnz) / 2) + 2);
  b += 8 * 1024 * 1024 + 64 * 256.0;   // task lists, small buffers, rounding
  return (size_t)b;
}

skm_status skm_init(const skm_csr *docs, const skm_config *cfg, skm_ctx **out) {
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(SKM_E_INVALID, "cfg is NULL");
  ST_TRY(check_csr_header(docs, 0));
  if (docs->n_rows < 1) return fail(SKM_E_INVALID, "need at least one row");
  if (cfg->k < 1 || cfg->k > 65535) return fail(SKM_E_INVALID, "k must be in [1, 65535]");
  if (cfg->precision < SKM_FP32 || cfg->precision > SKM_FP8_E4M3)
    return fail(SKM_E_INVALID, "unknown precision");
  if (!cfg->init_rows && !cfg->init_centroids)
    return fail(SKM_E_INVALID, "init_rows or init_centroids is required");
  if (cfg->init_rows) {
    if (cfg->k > docs->n_rows) return fail(SKM_E_INVALID, "k exceeds n_rows");
    for (int32_t j = 0; j < cfg->k; ++j)
      if (cfg->init_rows[j] < 0 || cfg->init_rows[j] >= docs->n_rows)
        return fail(SKM_E_INVALID, "init_rows entry out of range");
  }
  if (cfg->flags & SKM_INDEX) {
    if (cfg->n_lambda < 1 || cfg->n_lambda > 8) return fail(SKM_E_INVALID, "n_lambda must be 1..8");
    for (int i = 0; i < cfg->n_lambda; ++i)
      if (!(cfg->lambda[i] > 0.0 && cfg->lambda[i] <= 1.0) ||
          (i > 0 && !(cfg->lambda[i] > cfg->lambda[i - 1])))
        return fail(SKM_E_INVALID, "lambda must be ascending in (0, 1]");
  }
  if (docs->n_cols * kChunk * code_bytes(cfg->precision) > INT32_MAX)
    return fail(SKM_E_UNSUPPORTED, "n_cols too large: one 512-centroid slab of codes must stay "
                                   "below 2 GiB");
  if (cfg->stop_rule != SKM_STOP_PAPER && cfg->stop_rule != SKM_STOP_FIXED)
    return fail(SKM_E_INVALID, "unknown stop rule");

  skm_ctx *c = new (std::nothrow) skm_ctx();
  if (!c) return fail(SKM_E_NOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->cfg.init_rows = nullptr;
  c->cfg.init_centroids = nullptr;
  c->N = docs->n_rows;
  c->D = docs->n_cols;
  c->Z = docs->nnz;
  c->k = cfg->k;
  c->prec = cfg->precision;
  c->esize = code_bytes(c->prec);
  c->uq = unit_roundoff(c->prec);
  c->abs_coef = abs_coefficient(c->prec);
  c->ld = round_up(c->k, kChunk);
  c->bucket_rows = bucket_rows(c->N, c->k);
  c->nblk = (c->N + c->bucket_rows - 1) / c->bucket_rows;

  auto cleanup = [&](skm_status st) {
    skm_destroy(c);
    return st;
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return cleanup(device_fail(nullptr, "hipGetDevice", e));
  {
    const skm_status sn = noalloc_setup(c->device);
    if (sn != SKM_OK) return cleanup(sn);
  }
  if (cfg->stream) {
    c->stream = static_cast<hipStream_t>(cfg->stream);
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(device_fail(nullptr, "hipStreamCreate", e));
    c->own_stream = true;
  }
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        cus > 0)
      c->n_cu = cus;
    (void)hipGetLastError();
  }
  for (hipEvent_t &ev : c->ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) return cleanup(device_fail(nullptr, "hipEventCreate", e));
  }
  auto alloc = [c](auto **p, size_t bytes) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
    return dalloc(c, reinterpret_cast<T **>(p), (bytes + sizeof(T) - 1) / sizeof(T));
  };
  DevRows rows;
  skm_status st = upload_rows(c, docs, c->D, cfg->validate != 0, c->stream, alloc, &rows,
                              (cfg->flags & SKM_BORROW_DEVICE) != 0);
  if (st != SKM_OK) return cleanup(st);
  c->indptr = rows.indptr;
  c->indices = rows.indices;
  c->values = rows.values;
  c->xl1 = rows.xl1;
  c->xl2 = rows.xl2;

  const int64_t kD = (int64_t)c->k * c->D;
  const int64_t N = c->N, k = c->k;
#define A_(p, n)                                  \
  do {                                            \
    skm_status _s = dalloc(c, &(p), (size_t)(n)); \
    if (_s != SKM_OK) return cleanup(_s);         \
  } while (0)
  A_(c->master, kD);
  c->sup_W = (c->D + 31) / 32;
  A_(c->sup_nb, k * c->sup_W);
  A_(c->sup_mb, k * c->sup_W);
  A_(c->sup_mvalid, k);
  A_(c->sup_qmask, k);
  A_(c->S, kD);
  A_(c->tile, c->D * c->ld * c->esize);
  A_(c->scale, c->ld);
  A_(c->snorm, k);
  A_(c->shift, k);
  A_(c->dot_old, k);
  A_(c->changed, k);
  A_(c->ch_ids, k);
  A_(c->a, N);
  A_(c->a_prev, N);
  A_(c->lo, N);
  A_(c->hi, N);
  A_(c->lo_prev, N);
  A_(c->hi_prev, N);
  A_(c->flag_rows, N);
  A_(c->flag_L, N);
  A_(c->flag_mode, N);
  A_(c->counters, 8);
  A_(c->stat, 16);
  A_(c->hist, c->nblk * k);
  A_(c->counts, k);
  A_(c->offsets, k + 1);
  A_(c->members, N);
  A_(c->list_work, index_rows_work(N));
  A_(c->red, 8);
  A_(c->ids_count, 2);
  A_(c->part, ((int64_t)c->k + kChunk - 1) / kChunk * N);
  c->use_tail = !(c->cfg.flags & SKM_DENSE_ONLY);
  for (int w = 0; w < ((c->cfg.flags & SKM_NCC) ? 2 : 1) && c->use_tail; ++w) {
    const int64_t nch = ((int64_t)c->k + kChunk - 1) / kChunk;
    A_(c->tails[w].tail, nch * c->D);
    A_(c->tails[w].cnt, nch * c->D);
    A_(c->tails[w].off, nch * (c->D + 1));
    A_(c->tails[w].base, nch + 1);
    A_(c->tails[w].totals, nch);
    A_(c->tails[w].chunks, nch);
    A_(c->tails[w].bsum, nch * tail_scan_blocks(c->D));
  }
  if (c->cfg.flags & SKM_NCC) A_(c->tile_ch, c->D * c->ld * c->esize);
  if (c->cfg.flags & SKM_INDEX) {
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) !=
        hipSuccess)
      max_lds = 65536;
    (void)hipGetLastError();
    if (index_lds_bytes(c->k) + 4096 > (size_t)max_lds)
      return cleanup(fail(SKM_E_UNSUPPORTED, "k too large for the index query's LDS (" +
                                                 std::to_string(max_lds) + " bytes per workgroup)"));
    const int64_t nb = (k + 63) / 64;
    A_(c->mode, N);
    A_(c->idx_cnt, k);
    A_(c->idx_sstart, k);
    A_(c->idx_qstart, k);
    A_(c->idx_tot, 2);
    A_(c->idx_mask, c->D * nb);
    A_(c->idx_blkpre, c->D * nb);
    A_(c->idx_tcnt, c->D);
    A_(c->idx_toff, c->D + 1);
    A_(c->idx_dirty, k);
    A_(c->idx_dids, k);
    A_(c->idx_dbits, (k + 31) / 32);
    A_(c->idx_toff2, c->D + 1);
    A_(c->idx_best, c->D);
    A_(c->idx_rows, N);
    A_(c->idx_cand, N * (int64_t)c->idx_cap);
    A_(c->idx_ncand, N);
    A_(c->idx_level, N);
  }
  if (!cfg->hbm_budget_bytes) {
    // the update's partial-sum rows, once for the context's lifetime: a
    // multi-GB hipMalloc inside an iteration can take seconds
    c->work_slots = work_slots_bound(c);
    A_(c->work, c->work_slots * c->D);
    if (c->cfg.flags & SKM_INDEX) {
      // the index's entries: every centroid's non-zeros, at most min(nnz, k D)
      // (the members' terms), reserved up to 16 GiB
      const int64_t bound = std::min<int64_t>(c->Z, (int64_t)c->k * c->D);
      const int64_t cap = std::max<int64_t>(1024, std::min<int64_t>(bound, (16ll << 30) / 40));
      if ((st = alloc_index_entries(c, cap)) != SKM_OK) return cleanup(st);
    }
  }
#undef A_

  hipStream_t s = c->stream;
  if (launch_fill_u8(c->tile, 0, c->D * c->ld * c->esize, s) != hipSuccess ||
      launch_fill_u8(c->sup_mvalid, 0, k, s) != hipSuccess ||
      launch_fill_f64(c->S, 0.0, kD, s) != hipSuccess ||
      launch_fill_f64(c->snorm, 0.0, k, s) != hipSuccess ||
      launch_fill_u8(c->changed, 1, k, s) != hipSuccess)
    return cleanup(device_fail(c, "fill", hipGetLastError()));
  {
    std::vector<float> ones(c->ld, 1.0f);
    e = hipMemcpyAsync(c->scale, ones.data(), sizeof(float) * c->ld, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return cleanup(device_fail(c, "hipMemcpy scale", e));
    if (cfg->init_rows) {
      int32_t *drows = nullptr;
      if ((st = dalloc(c, &drows, (size_t)k)) != SKM_OK) return cleanup(st);
      e = hipMemcpyAsync(drows, cfg->init_rows, sizeof(int32_t) * k, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = launch_seed(c->indptr, c->indices, c->values, drows, c->k, c->D,
                                           c->master, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return cleanup(device_fail(c, "seed", e));
    } else {
      e = hipMemcpyAsync(c->master, cfg->init_centroids, sizeof(double) * kD, hipMemcpyHostToDevice,
                         s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return cleanup(device_fail(c, "init centroids", e));
    }
  }
  {
    std::vector<uint32_t> df;
    if ((st = term_df(c, df)) != SKM_OK) return cleanup(st);
    if ((st = setup_sum_hot(c, df)) != SKM_OK) return cleanup(st);
    if ((st = setup_head(c, df)) != SKM_OK) return cleanup(st);
  }
  if ((st = rebuild_tiles(c, nullptr, nullptr)) != SKM_OK) return cleanup(st);
  if ((c->cfg.flags & SKM_INDEX) && (st = build_index(c)) != SKM_OK) return cleanup(st);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(device_fail(c, "init sync", e));
  c->force_all = true;
  c->have_prev = false;
  c->last_changed = c->k;
  *out = c;
  return SKM_OK;
}

// Records the next event of a pair list on stream s (events created on demand).
skm_status mark(skm_ctx *c, skm_ctx::EventPairs &p, hipStream_t s) {
  if (p.used == p.ev.size()) {
    hipEvent_t x = nullptr;
    hipError_t e = hipEventCreate(&x);
    if (e != hipSuccess) return device_fail(c, "hipEventCreate", e);
    p.ev.push_back(x);
  }
  HIP_TRY(c, hipEventRecord(p.ev[p.used++], s));
  return SKM_OK;
}

// Device time of the pairs recorded since the last reset (after a sync).
float pairs_ms(const skm_ctx::EventPairs &p) {
  float ms = 0.f;
  for (size_t i = 0; i + 1 < p.used; i += 2) ms += elapsed(p.ev[i], p.ev[i + 1]);
  return ms;
}

void reset_timers(skm_ctx *c) {
  c->head_t.used = 0;
  c->sparse_t.used = 0;
  c->head_pairs = 0;
}

// One launch of the sparse scoring kernel, bracketed by a timing pair.
skm_status score_part_timed(skm_ctx *c, const ScoreArgs &a, hipStream_t s) {
  ST_TRY(mark(c, c->sparse_t, s));
  HIP_TRY(c, launch_score_part(a, c->part, c->n_cu, c->prec, s, c->score_wpc));
  ST_TRY(mark(c, c->sparse_t, s));
  return SKM_OK;
}

// Low-precision scoring with the head product of the rows [0, n_rows), or of
// the listed rows, against the first ncols columns of a code copy whose head
// codes are chead: in batches of head_rows rows x head_chunks chunks, head
// GEMM into hs, then the sparse kernel adds the rows' other terms.  Batches
// are large so that the sparse kernel still sweeps each chunk of codes over
// many rows while its term rows are cached.  Both launches are bracketed by
// timing pairs (head_t, sparse_t).
skm_status head_pass(skm_ctx *c, ScoreArgs &a, hipStream_t s, const uint16_t *chead,
                     int64_t ncols, const int32_t *rows, int64_t n_rows) {
  a.sc_indptr = c->r_indptr;
  a.sc_indices = c->r_indices;
  a.sc_values = c->r_values;
  a.hs = c->hs;
  a.head_H = c->head_H;
  a.row_list = rows;
  const int32_t nch = (int32_t)((ncols + kChunk - 1) / kChunk);
  // fewer rows than a batch (the rows of changed clusters late in a run): as
  // many chunks per batch as the head-score buffer holds, so that each sparse
  // launch still has many items to spread over the GPU
  const int64_t rb = std::max<int64_t>(1, std::min<int64_t>(c->head_rows, n_rows));
  const int32_t g = (int32_t)std::max<int64_t>(
      c->head_chunks, std::min<int64_t>(nch, c->hs_cap / (rb * kChunk)));
  a.hs_ld = (int64_t)g * kChunk;
  for (int64_t r0 = 0; r0 < n_rows; r0 += rb) {
    const int64_t nb = std::min<int64_t>(rb, n_rows - r0);
    for (int32_t g0 = 0; g0 < nch; g0 += g) {
      const int32_t gc = std::min<int32_t>(g, nch - g0);
      // the product stops at the first 256-column tile boundary past the last
      // live column (a compacted copy of few changed centroids)
      const int64_t gcols =
          std::min<int64_t>((int64_t)gc * kChunk, round_up(ncols - (int64_t)g0 * kChunk, 256));
      ST_TRY(mark(c, c->head_t, s));
      HIP_TRY(c, launch_head_gemm(c->xh, c->head_H, r0, nb, rows, chead, (int64_t)g0 * kChunk,
                                  gcols, c->hs, a.hs_ld, s));
      ST_TRY(mark(c, c->head_t, s));
      c->head_pairs += (double)nb * (double)gcols;
      a.row0 = r0;
      a.nb = nb;
      a.c_first = g0;
      a.c_count = gc;
      ST_TRY(score_part_timed(c, a, s));
    }
  }
  a.row_list = nullptr;
  a.row0 = 0;
  a.nb = c->N;
  a.c_first = 0;
  a.c_count = (int32_t)((c->k + kChunk - 1) / kChunk);
  return SKM_OK;
}

skm_status skm_assign(skm_ctx *c, skm_iter_stats *st_out) {
  ST_TRY(check_ctx_writable(c));
  hipStream_t s = c->stream;
  c->idx_skip_pre = c->idx_skip;       // a checkpoint taken before the update restores these
  c->idx_backoff_pre = c->idx_backoff;
  ScoreArgs a = base_args(c);
  // Sec. 3.1 pays when the work it leaves, (1 - r) n_ch / k of the scores of
  // the rows keeping their centroid plus the share r of rows whose centroid
  // changed (all of theirs), is clearly below a full pass; otherwise every
  // row scores the full copy.
  const double ncc_cost = (1.0 - c->full_frac) * (double)c->last_changed / (double)c->k + c->full_frac;
  bool ncc = (c->cfg.flags & SKM_NCC) && c->have_prev && ncc_cost <= kNccMaxCost;
  if (ncc && c->cfg.ncc_adaptive && c->ms_full_assign >= 0.f) {
    // predicted Sec. 3.1 assignment: the share ncc_cost of the last full
    // pass's scoring plus its own fixed cost (the compacted copy and lists,
    // the row lists, the extra launches and waits), measured at its last use
    // as its assignment time beyond the scaled scoring, else estimated from
    // the bytes the compacted copy moves; against the last full assignment
    const double fixed = c->ms_ncc_fixed >= 0.f
                             ? (double)c->ms_ncc_fixed
                             : 3.0 * (double)c->D * c->last_changed * c->esize / 2e9;
    if (fixed + ncc_cost * (double)c->ms_full_score >= (double)c->ms_full_assign) ncc = false;
  }
  int32_t n_ch = c->k;
  HIP_TRY(c, hipEventRecord(c->ev[0], s));
  if (ncc) {
    // the flags are those of the last update, which counted them
    n_ch = c->last_changed;
    HIP_TRY(c, launch_compact_changed(c->changed, c->k, c->ch_ids, c->ids_count, s));
    HIP_TRY(c, launch_gather_tile(c->tile, c->D, c->esize, c->ch_ids, n_ch, c->tile_ch, s));
    ST_TRY(build_tail(c, 1, c->tile_ch, n_ch, nullptr));
    a.a_prev = c->a_prev;
    a.changed = c->changed;
    a.tile_ch = c->tile_ch;
    a.n_ch = n_ch;
    a.ch_ids = c->ch_ids;
    a.tv_ch = tail_view(c, 1);
    a.prev_lo = c->lo_prev;
    a.prev_hi = c->hi_prev;
  }
  HIP_TRY(c, launch_fill_i32(c->counters, 0, 8, s));
  HIP_TRY(c, launch_fill_i32(reinterpret_cast<int32_t *>(c->stat), 0, 32, s));
  const bool use_index = (c->cfg.flags & SKM_INDEX) && c->have_prev && c->index_ready &&
                         (c->cfg.index_min_changed <= 0 || c->last_changed > c->cfg.index_min_changed);
  if (use_index) {
    // every row queries the index; with NCC on, a row keeping an unchanged
    // previous centroid only takes changed candidates (end of Sec. 3.2)
    HIP_TRY(c, hipEventRecord(c->ev[6], s));
    HIP_TRY(c, launch_fill_u8(c->mode, 0, c->N, s));
    const int64_t n_rows_idx = c->N;
    IndexArgs x = index_args(c);
    x.rows = nullptr;   // every row, slot = row
    x.changed = ncc ? c->changed : nullptr;
    x.n_ch = n_ch;
    HIP_TRY(c, index_query(x, n_rows_idx, s));
    HIP_TRY(c, index_score(x, n_rows_idx, c->a, c->lo, c->hi, s));
    HIP_TRY(c, hipEventRecord(c->ev[7], s));
    a.mode = c->mode;
    c->idx_eligible = n_rows_idx;
  }
  HIP_TRY(c, hipEventRecord(c->ev[5], s));
  const bool head = c->head_H > 0;
  reset_timers(c);
  // rows the index finished take no part in the head products
  const uint8_t *undecided = use_index ? c->mode : nullptr;
  if (head && !ncc) {
    if (use_index) {
      int32_t n_list = 0;
      HIP_TRY(c, index_rows(c->a_prev, nullptr, c->N, c->full_rows, c->ids_count, c->list_work, s,
                            0, undecided));
      HIP_TRY(c, hipMemcpyAsync(&n_list, c->ids_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipStreamSynchronize(s));
      ST_TRY(head_pass(c, a, s, c->ch_head, c->k, c->full_rows, n_list));
    } else {
      ST_TRY(head_pass(c, a, s, c->ch_head, c->k, nullptr, c->N));
    }
    HIP_TRY(c, launch_finalize(a, c->part, s));
  } else if (head) {
    // Sec. 3.1 with the head: every row keeping its previous centroid scores
    // the changed centroids only (their head codes compacted alongside the
    // compacted code copy); the rows whose previous centroid changed score
    // all centroids, from their list.  One merge over all rows at the end.
    int32_t n_full = 0, n_keep = 0;
    HIP_TRY(c, index_rows(c->a_prev, c->changed, c->N, c->full_rows, c->ids_count, c->list_work, s,
                          0, undecided));
    HIP_TRY(c, hipMemcpyAsync(&n_full, c->ids_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (n_ch > kNarrowMax) {
      HIP_TRY(c, launch_gather_head(c->ch_head, c->head_H, c->ch_ids, n_ch, c->ch_head_ch, s));
      HIP_TRY(c, index_rows(c->a_prev, c->changed, c->N, c->ncc_list, c->ids_count + 1,
                            c->list_work, s, 1, undecided));
      HIP_TRY(c, hipMemcpyAsync(&n_keep, c->ids_count + 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                                s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    a.ncc_only = 1;
    if (n_ch <= kNarrowMax) {
      // few changed centroids: all terms of those rows straight from the
      // compacted codes, no head product
      HIP_TRY(c, launch_score_narrow(a, c->part, c->prec, s));
    } else {
      // head products of the rows keeping their centroid only
      ST_TRY(head_pass(c, a, s, c->ch_head_ch, n_ch, c->ncc_list, n_keep));
    }
    a.ncc_only = 0;
    ST_TRY(head_pass(c, a, s, c->ch_head, c->k, c->full_rows, n_full));
    HIP_TRY(c, launch_finalize(a, c->part, s));
  } else {
    ST_TRY(score_part_timed(c, a, s));
    HIP_TRY(c, launch_finalize(a, c->part, s));
  }
  HIP_TRY(c, hipEventRecord(c->ev[1], s));
  if (!a.no_exact) {
    ExactArgs x{a, c->part, c->master, c->D, exact_waves()};
    HIP_TRY(c, launch_exact(x, c->prec, s));
  }
  HIP_TRY(c, hipEventRecord(c->ev[2], s));
  if (c->have_prev) HIP_TRY(c, launch_count_moved(c->a, c->a_prev, c->N, c->stat + 4, s));
  int32_t cnt[8];
  unsigned long long stv[16];
  HIP_TRY(c, hipMemcpyAsync(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(stv, c->stat, sizeof(stv), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  {
    const float ms_assign = elapsed(c->ev[0], c->ev[2]);
    if (!ncc) {
      c->ms_full_score = elapsed(c->ev[5], c->ev[1]);
      c->ms_full_assign = ms_assign;
    } else if (c->ms_full_score >= 0.f) {
      c->ms_ncc_fixed = std::max(0.f, ms_assign - (float)(ncc_cost * c->ms_full_score));
    }
  }
  c->assigned = true;
  c->last_moved = c->have_prev ? (int64_t)stv[4] : c->N;
  if (use_index && !c->cfg.index_always) {
    // Sec. 4.3: the index only pays when it decides rows; back off otherwise
    if ((double)stv[2] < 0.05 * (double)std::max<int64_t>(c->idx_eligible, 1)) {
      c->idx_skip = c->idx_backoff;
      c->idx_backoff = std::min(2 * c->idx_backoff, 64);
    } else {
      c->idx_backoff = 8;
    }
  }
  if (st_out) {
    std::memset(st_out, 0, sizeof(*st_out));
    st_out->iter = c->iter;
    st_out->changed_centroids = c->have_prev ? c->last_changed : c->k;
    st_out->moved = c->last_moved;
    st_out->flagged = cnt[0];
    st_out->band_overflow = cnt[1];
    st_out->ncc_rows = (int64_t)stv[1];
    st_out->index_rows = (int64_t)stv[2];
    st_out->index_no_level = (int64_t)stv[5];
    st_out->index_guarded = (int64_t)stv[6];
    st_out->index_over_cap = (int64_t)stv[7];
    st_out->mean_candidates = (double)stv[0] / (double)c->N;
    st_out->scored_products = (double)stv[3];
    st_out->ms_assign = elapsed(c->ev[0], c->ev[2]);
    st_out->ms_score = elapsed(c->ev[5], c->ev[1]);
    st_out->ms_exact = elapsed(c->ev[1], c->ev[2]);
    st_out->ms_index = use_index ? elapsed(c->ev[6], c->ev[7]) : 0.f;
    st_out->head_terms = head ? c->head_H : 0;
    st_out->score_launches = (int32_t)(c->sparse_t.used / 2);
    st_out->ms_sparse = pairs_ms(c->sparse_t);
    st_out->sparse_products = (double)stv[3];
    if (head) {
      st_out->ms_head = pairs_ms(c->head_t);
      st_out->head_launches = (int32_t)(c->head_t.used / 2);
      st_out->head_pairs = c->head_pairs;
      st_out->sparse_products = (double)stv[8];
    }
    st_out->objective_assign = st_out->objective_update = st_out->max_shift_sq = -1.0;
  }
  return SKM_OK;
}

skm_status skm_tune_lambda(skm_ctx *c, int32_t n_sample, skm_lambda_report *report) {
  ST_TRY(check_ctx_writable(c));
  if (!(c->cfg.flags & SKM_INDEX)) return fail(SKM_E_STATE, "skm_tune_lambda needs SKM_INDEX");
  if (!c->have_prev || c->assigned)
    return fail(SKM_E_STATE, "skm_tune_lambda needs a completed update and no pending assignment");
  if (n_sample < 1) return fail(SKM_E_INVALID, "n_sample must be >= 1");
  hipStream_t s = c->stream;
  if (!c->index_ready) ST_TRY(build_index(c));
  const int64_t n = std::min<int64_t>(n_sample, c->N);
  // rows spread evenly over the corpus (deterministic)
  std::vector<int32_t> rows(n);
  for (int64_t q = 0; q < n; ++q) rows[q] = (int32_t)((q * c->N) / n);
  HIP_TRY(c, hipMemcpyAsync(c->idx_rows, rows.data(), 4 * n, hipMemcpyHostToDevice, s));
  // the thresholds measured: a fixed grid and the set in use
  std::vector<double> grid = {0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.5, 0.6, 0.7, 0.8};
  for (int l = 0; l < c->cfg.n_lambda; ++l)
    if (std::find(grid.begin(), grid.end(), c->cfg.lambda[l]) == grid.end())
      grid.push_back(c->cfg.lambda[l]);
  std::sort(grid.begin(), grid.end());
  if (grid.size() > 20) grid.resize(20);
  const int32_t G = (int32_t)grid.size();
  // rows keeping an unchanged previous centroid only take changed candidates
  // (and would otherwise score the n_ch changed centroids)
  const bool ncc = (c->cfg.flags & SKM_NCC) != 0;
  std::vector<uint8_t> ch(c->k);
  std::vector<int32_t> ap(c->N);
  std::vector<double> xn(c->N), blo(n);
  HIP_TRY(c, hipMemcpyAsync(ch.data(), c->changed, c->k, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(ap.data(), c->a_prev, 4 * c->N, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(xn.data(), c->xl2, 8 * c->N, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  int32_t n_ch = 0;
  for (uint8_t f : ch) n_ch += f != 0;
  std::vector<double> dense(n), ratio(n);
  std::vector<int32_t> cand((size_t)G * n);
  for (int32_t g = 0; g < G; ++g) {
    IndexArgs x = index_args(c);
    x.lambda[0] = grid[g];
    x.n_lambda = 1;
    x.forced_level = 0;
    x.guard = 1e300;
    x.mode = nullptr;
    x.changed = ncc ? c->changed : nullptr;
    x.n_ch = n_ch;
    x.base_out = g == 0 ? c->flag_L : nullptr;
    HIP_TRY(c, launch_fill_i32(reinterpret_cast<int32_t *>(c->stat), 0, 32, s));
    HIP_TRY(c, index_query(x, n, s));
    HIP_TRY(c, hipMemcpyAsync(cand.data() + (size_t)g * n, c->idx_ncand, 4 * n,
                              hipMemcpyDeviceToHost, s));
    if (g == 0) HIP_TRY(c, hipMemcpyAsync(blo.data(), c->flag_L, 8 * n, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(c, hipStreamSynchronize(s));
  for (int64_t q = 0; q < n; ++q) {
    const int32_t r = rows[q];
    const bool keep = ncc && !ch[ap[r]];
    dense[q] = keep ? (double)n_ch + 1.0 : (double)c->k;
    ratio[q] = blo[q] / (xn[r] * (1.0 + 0x1p-40));   // qualifies for lam <= ratio
  }
  // cost of a row at grid level g: candidates + 1 when its baseline reaches
  // the threshold (and the list fits), else the dense scan
  auto row_cost = [&](int64_t q, int32_t g) {
    if (!(grid[g] <= ratio[q])) return dense[q];
    const int32_t nc = cand[(size_t)g * n + q];
    return nc >= 0 ? (double)nc + 1.0 : dense[q];
  };
  auto set_cost = [&](const std::vector<int32_t> &set) {   // set ascending
    double sum = 0.0;
    for (int64_t q = 0; q < n; ++q) {
      double cst = dense[q];
      for (int32_t i = (int32_t)set.size() - 1; i >= 0; --i)
        if (grid[set[i]] <= ratio[q]) {
          cst = row_cost(q, set[i]);
          break;
        }
      sum += cst;
    }
    return sum / (double)n;
  };
  std::vector<int32_t> cur;
  for (int l = 0; l < c->cfg.n_lambda; ++l)
    cur.push_back((int32_t)(std::find(grid.begin(), grid.end(), c->cfg.lambda[l]) - grid.begin()));
  std::sort(cur.begin(), cur.end());
  const double cost_before = set_cost(cur);
  // every set of at most four grid thresholds (the paper uses four levels)
  std::vector<int32_t> best = cur, set;
  double best_cost = cost_before;
  std::function<void(int32_t)> walk = [&](int32_t from) {
    if (!set.empty()) {
      const double cst = set_cost(set);
      if (cst < best_cost - 1e-12 || (cst <= best_cost + 1e-12 && set.size() < best.size())) {
        best_cost = cst;
        best = set;
      }
    }
    if (set.size() == 4) return;
    for (int32_t g = from; g < G; ++g) {
      set.push_back(g);
      walk(g + 1);
      set.pop_back();
    }
  };
  walk(0);
  // a new set is taken only when it is clearly cheaper (5 %)
  const bool apply = best != cur && best_cost < 0.95 * cost_before;
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->n_sample = (int32_t)n;
    report->n_grid = G;
    for (int32_t g = 0; g < G; ++g) {
      int64_t nq = 0;
      double sc = 0.0;
      for (int64_t q = 0; q < n; ++q)
        if (grid[g] <= ratio[q]) {
          ++nq;
          sc += row_cost(q, g);
        }
      report->grid[g] = grid[g];
      report->qualify[g] = (double)nq / (double)n;
      report->mean_candidates[g] = nq ? sc / (double)nq : 0.0;
    }
    report->n_before = (int32_t)cur.size();
    for (size_t i = 0; i < cur.size(); ++i) report->before[i] = grid[cur[i]];
    report->cost_before = cost_before;
    const std::vector<int32_t> &fin = apply ? best : cur;
    report->n_after = (int32_t)fin.size();
    for (size_t i = 0; i < fin.size(); ++i) report->after[i] = grid[fin[i]];
    report->cost_after = apply ? best_cost : cost_before;
    report->applied = apply ? 1 : 0;
  }
  if (apply) {
    c->cfg.n_lambda = (int32_t)best.size();
    for (size_t i = 0; i < best.size(); ++i) c->cfg.lambda[i] = grid[best[i]];
  }
  return SKM_OK;
}

skm_status skm_autotune(skm_ctx *c, skm_tune_report *report) {
  ST_TRY(check_ctx_writable(c));
  if (c->assigned)
    return fail(SKM_E_STATE, "skm_autotune needs no pending assignment (call it before "
                             "skm_assign or after skm_update)");
  hipStream_t s = c->stream;
  skm_tune_report rep;
  std::memset(&rep, 0, sizeof(rep));
  // one full scoring pass (no exact tier, no NCC) at a given shape
  auto pass = [&](int32_t chunks, int64_t rows, int32_t wpc, double *ms) -> skm_status {
    c->head_chunks = chunks;
    c->head_rows = rows;
    c->score_wpc = wpc;
    ScoreArgs a = base_args(c);
    HIP_TRY(c, launch_fill_i32(c->counters, 0, 8, s));
    HIP_TRY(c, launch_fill_i32(reinterpret_cast<int32_t *>(c->stat), 0, 32, s));
    HIP_TRY(c, hipEventRecord(c->ev[5], s));
    reset_timers(c);
    if (c->head_H > 0) {
      ST_TRY(head_pass(c, a, s, c->ch_head, c->k, nullptr, c->N));
      HIP_TRY(c, launch_finalize(a, c->part, s));
    } else {
      HIP_TRY(c, launch_score(a, c->part, c->n_cu, c->prec, s, wpc));
    }
    HIP_TRY(c, hipEventRecord(c->ev[1], s));
    HIP_TRY(c, hipStreamSynchronize(s));
    *ms = (double)elapsed(c->ev[5], c->ev[1]);
    return SKM_OK;
  };
  auto trial = [&](int32_t chunks, int64_t rows, int32_t wpc) -> skm_status {
    double ms = 0;
    ST_TRY(pass(chunks, rows, wpc, &ms));
    if (rep.n_trials < (int32_t)(sizeof(rep.trials) / sizeof(rep.trials[0]))) {
      skm_tune_trial &t = rep.trials[rep.n_trials++];
      t.head_chunks = c->head_H > 0 ? chunks : 0;
      t.head_rows = c->head_H > 0 ? rows : 0;
      t.workgroups_per_cu = wpc;
      t.ms = ms;
    }
    return SKM_OK;
  };
  const int32_t chunks0 = c->head_chunks;
  const int64_t rows0 = c->head_rows;
  double warm = 0;
  ST_TRY(pass(chunks0, rows0, c->score_wpc, &warm));   // first-use costs, not recorded
  // stage 1: workgroups per CU of the sparse kernel, from one above the
  // occupancy limit down to four below it (fewer rows in flight can keep more
  // of a chunk's code rows in L2)
  const int occ = score_occupancy(c->prec);
  for (int32_t w = std::min(occ + 1, 8); w >= std::max(occ - 4, 2); --w)
    ST_TRY(trial(chunks0, rows0, w));
  // the fastest trial (equal times: the earlier one)
  auto best_of = [&]() {
    int32_t b = 0;
    for (int32_t i = 1; i < rep.n_trials; ++i)
      if (rep.trials[i].ms < rep.trials[b].ms) b = i;
    return b;
  };
  const int32_t wbest = rep.trials[best_of()].workgroups_per_cu;
  // stage 2: the head batch shape (chunks x rows filling the head-score buffer)
  if (c->head_H > 0) {
    const int32_t nch = (int32_t)((c->k + kChunk - 1) / kChunk);
    for (int32_t g : {1, 2, 4, 8}) {
      if (g > nch || g == chunks0) continue;
      int64_t rows = c->hs_cap / ((int64_t)g * kChunk) / 256 * 256;
      rows = std::min<int64_t>(rows, round_up(c->N, 256));
      if (rows < 256) continue;
      ST_TRY(trial(g, rows, wbest));
    }
  }
  rep.best = best_of();
  const skm_tune_trial &b = rep.trials[rep.best];
  c->score_wpc = b.workgroups_per_cu;
  if (c->head_H > 0) {
    c->head_chunks = b.head_chunks;
    c->head_rows = b.head_rows;
  } else {
    c->head_chunks = chunks0;
    c->head_rows = rows0;
  }
  if (report) *report = rep;
  return SKM_OK;
}

skm_status skm_set_schedule(skm_ctx *c, const skm_tune_trial *shape) {
  ST_TRY(check_ctx_writable(c));
  if (!shape) return fail(SKM_E_INVALID, "shape is NULL");
  if (shape->workgroups_per_cu < 0 || shape->workgroups_per_cu > 16)
    return fail(SKM_E_INVALID, "workgroups_per_cu must be in [0, 16]");
  if (c->head_H > 0) {
    const int64_t nch = (c->k + kChunk - 1) / kChunk;
    if (shape->head_chunks < 1 || shape->head_chunks > nch || shape->head_rows < 1 ||
        shape->head_rows * shape->head_chunks * kChunk > c->hs_cap)
      return fail(SKM_E_INVALID, "head batch shape does not fit the head-score buffer");
    c->head_chunks = shape->head_chunks;
    c->head_rows = shape->head_rows;
  }
  c->score_wpc = shape->workgroups_per_cu;
  return SKM_OK;
}

skm_status skm_update(skm_ctx *c, skm_iter_stats *st_out) {
  ST_TRY(check_ctx_writable(c));
  if (!c->assigned) return fail(SKM_E_STATE, "skm_update needs a preceding skm_assign");
  hipStream_t s = c->stream;
  HIP_TRY(c, hipEventRecord(c->ev[3], s));
  if (c->force_all || !c->have_prev) {
    HIP_TRY(c, launch_fill_u8(c->changed, 1, c->k, s));
  } else {
    HIP_TRY(c, launch_fill_u8(c->changed, 0, c->k, s));
    HIP_TRY(c, launch_mark_changed(c->a, c->a_prev, c->N, c->changed, s));
  }
  int32_t n_ids = 0;
  HIP_TRY(c, launch_compact_changed(c->changed, c->k, c->ch_ids, c->ids_count, s));
  HIP_TRY(c, hipMemcpyAsync(&n_ids, c->ids_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, launch_bucket(c->a, c->N, c->k, c->bucket_rows, c->hist, c->counts, c->offsets,
                           c->members, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  std::vector<int32_t> ids, chunks;
  ST_TRY(sum_changed(c, n_ids, ids));
  for (int32_t j : ids)   // ascending ids: ascending chunks
    if (chunks.empty() || chunks.back() != j / kChunk) chunks.push_back(j / kChunk);
  RenormSupport rs;
  rs.W = c->sup_W;
  rs.nb = c->sup_nb;
  rs.mb = c->sup_mb;
  rs.mvalid = c->sup_mvalid;
  rs.qmask = c->sup_qmask;
  rs.tile = c->tile;
  rs.scale = c->scale;
  HIP_TRY(c, launch_fill_u8(c->sup_qmask, 0, c->k, s));
  HIP_TRY(c, launch_renorm(c->S, c->counts, c->ch_ids, n_ids, c->D, c->master, c->snorm, c->shift,
                           c->dot_old, rs, c->prec, s));
  HIP_TRY(c, launch_reduce_stats(c->changed, c->snorm, c->shift, c->dot_old, c->k, c->red, s));
  ST_TRY(rebuild_tiles(c, c->changed, &chunks, c->sup_qmask));
  HIP_TRY(c, hipEventRecord(c->ev[4], s));
  c->ms_index_build = 0.f;
  c->idx_last_build = 0;
  const bool index_was_ready = c->index_ready;
  c->index_ready = false;
  if (c->cfg.flags & SKM_INDEX) {
    if (c->idx_skip > 0) {
      c->idx_skip -= 1;   // index off for this iteration: no rebuild (the next is full)
    } else {
      // valid for the previous centroids: rebuild the changed ones
      c->index_ready = index_was_ready;
      ST_TRY(build_index(c, c->ch_ids, &ids));
    }
  }
  double red[3];
  HIP_TRY(c, hipMemcpyAsync(red, c->red, sizeof(red), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  std::swap(c->a, c->a_prev);
  std::swap(c->lo, c->lo_prev);
  std::swap(c->hi, c->hi_prev);
  c->have_prev = true;
  c->force_all = false;
  c->assigned = false;
  c->last_changed = n_ids;
  c->iter += 1;
  if (st_out) {
    st_out->objective_assign = red[0];
    st_out->objective_update = red[1];
    st_out->max_shift_sq = red[2];
    st_out->ms_update = elapsed(c->ev[3], c->ev[4]);
    if (c->cfg.flags & SKM_INDEX) st_out->ms_index += c->ms_index_build;
    st_out->ms_index_build = c->ms_index_build;
    st_out->index_build = c->idx_last_build;
  }
  return SKM_OK;
}

skm_status skm_iterate(skm_ctx *c, int32_t max_iter, skm_iter_stats *per_iter, int32_t *n_done,
                       int32_t *converged) {
  ST_TRY(check_ctx_writable(c));
  if (max_iter <= 0) max_iter = c->cfg.max_iter;
  int32_t done = 0;
  int32_t conv = 0;
  for (int32_t t = 0; t < max_iter; ++t) {
    skm_iter_stats st{};
    ST_TRY(skm_assign(c, &st));
    done += 1;
    const bool paper = c->cfg.stop_rule == SKM_STOP_PAPER;
    if (paper && c->iter >= 1 &&
        (st.moved == 0 || (double)st.moved < c->cfg.min_moved_frac * (double)c->N)) {
      conv = 1;
      if (per_iter) per_iter[t] = st;
      break;
    }
    ST_TRY(skm_update(c, &st));
    if (per_iter) per_iter[t] = st;
    if (paper && st.max_shift_sq < c->cfg.max_shift_sq) {
      conv = 1;
      break;
    }
  }
  if (n_done) *n_done = done;
  if (converged) *converged = conv;
  return SKM_OK;
}

skm_status skm_assign_new(skm_ctx *c, const skm_csr *docs, int32_t *out_assign, double *out_score,
                          void *stream) {
  ST_TRY(check_ctx(c));
  ST_TRY(check_csr_header(docs, c->D));
  if (!out_assign || !out_score) return fail(SKM_E_INVALID, "output pointer is NULL");
  const int64_t n = docs->n_rows;
  if (n == 0) return SKM_OK;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  std::vector<void *> tmp;
  auto talloc = [&](auto **p, size_t bytes) -> skm_status {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 1));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SKM_E_NOMEM, "temporary device allocation failed");
    }
    tmp.push_back(q);
    *p = static_cast<std::remove_reference_t<decltype(*p)>>(q);
    return SKM_OK;
  };
  auto release = [&]() {
    for (void *q : tmp) (void)hipFree(q);
  };
  DevRows r;
  // the certificate assumes positive values and ascending terms: always check
  skm_status st = upload_rows(c, docs, c->D, true, s, talloc, &r);
  if (st != SKM_OK) {
    release();
    return st;
  }
  skm::Partial *part = nullptr;
  if ((st = talloc(&part, sizeof(skm::Partial) * (((int64_t)c->k + kChunk - 1) / kChunk) * n)) !=
      SKM_OK) {
    release();
    return st;
  }
  int32_t *a = nullptr, *flag_rows = nullptr, *counters = nullptr;
  double *lo = nullptr, *hi = nullptr, *flag_L = nullptr, *score = nullptr;
  uint8_t *flag_mode = nullptr;
  unsigned long long *stat = nullptr;
  if ((st = talloc(&a, n * 4)) != SKM_OK || (st = talloc(&flag_rows, n * 4)) != SKM_OK ||
      (st = talloc(&counters, 32)) != SKM_OK || (st = talloc(&lo, n * 8)) != SKM_OK ||
      (st = talloc(&hi, n * 8)) != SKM_OK || (st = talloc(&flag_L, n * 8)) != SKM_OK ||
      (st = talloc(&score, n * 8)) != SKM_OK || (st = talloc(&flag_mode, n)) != SKM_OK ||
      (st = talloc(&stat, 64)) != SKM_OK) {
    release();
    return st;
  }
  NewRows nr{r.indptr, r.indices, r.values, r.xl1, part, a, lo, hi, flag_rows, flag_L, flag_mode,
             counters, stat, score};
  hipError_t e = hipSuccess;
  unsigned long long *istat = nullptr;
  if ((c->cfg.flags & SKM_INDEX) && c->index_ready) {
    // Sec. 3.2 for rows without a previous assignment: the baseline is the
    // certified score of a probe centroid (the best of the centroids largest
    // at the row's largest values); the true maximum scores at least as
    // much, so by Lemma 3.1 it is among the index's candidates at the level
    // that baseline selects.  Rows the index settles skip the scoring pass.
    int32_t *probe = nullptr, *cand = nullptr, *ncand = nullptr, *level = nullptr;
    uint8_t *mode = nullptr;
    if ((st = talloc(&probe, n * 4)) != SKM_OK || (st = talloc(&ncand, n * 4)) != SKM_OK ||
        (st = talloc(&level, n * 4)) != SKM_OK || (st = talloc(&mode, n)) != SKM_OK ||
        (st = talloc(&cand, n * 4 * (int64_t)c->idx_cap)) != SKM_OK ||
        (st = talloc(&istat, 128)) != SKM_OK) {
      release();
      return st;
    }
    IndexArgs x = index_args(c);
    {
      std::lock_guard<std::mutex> lock(c->best_mu);
      if (!c->idx_best_ready) {
        e = index_best_centroid(x, c->idx_dirty, c->idx_sstart, c->idx_key0, c->idx_best, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // other streams read it next
        c->idx_best_ready = e == hipSuccess;
      }
    }
    if (e == hipSuccess) e = launch_fill_u8(mode, 0, n, s);
    if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t *>(istat), 0, 32, s);
    if (e == hipSuccess)
      e = index_probe(r.indptr, r.indices, r.values, n, c->idx_best, c->master, c->D, probe, s);
    x.indptr = r.indptr;
    x.indices = r.indices;
    x.values = r.values;
    x.xl2 = r.xl2;
    x.rows = nullptr;
    x.a_prev = probe;
    x.changed = nullptr;
    x.n_ch = c->k;
    x.cand = cand;
    x.ncand = ncand;
    x.level = level;
    x.mode = mode;
    x.stat = istat;
    x.base_out = nullptr;
    if (e == hipSuccess) e = index_query(x, n, s);
    if (e == hipSuccess) e = index_score(x, n, a, lo, hi, s);
    nr.mode = mode;
  }
  if (e == hipSuccess) e = launch_new_rows(c, nr, n, s);
  unsigned long long ist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (e == hipSuccess && istat) e = hipMemcpyAsync(ist, istat, sizeof(ist), hipMemcpyDeviceToHost, s);
  const hipMemcpyKind kind = docs->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess) e = hipMemcpyAsync(out_assign, a, n * 4, kind, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out_score, score, n * 8, kind, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) return device_fail(c, "skm_assign_new", e);
  c->new_index_rows = (int64_t)ist[2];
  return SKM_OK;
}

int64_t skm_assign_new_index_rows(const skm_ctx *c) {
  if (check_ctx(c) != SKM_OK) return -1;
  return c->new_index_rows;
}

skm_status skm_get_assignments(const skm_ctx *c, int32_t *out, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  const int32_t *src = c->assigned ? c->a : c->a_prev;
  if (!c->assigned && !c->have_prev) return fail(SKM_E_STATE, "no assignment yet");
  hipError_t e = hipMemcpyAsync(out, src, sizeof(int32_t) * c->N,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return device_fail(const_cast<skm_ctx *>(c), "get_assignments", e);
  return SKM_OK;
}

skm_status skm_get_centroids(const skm_ctx *c, double *out, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  hipError_t e = hipMemcpyAsync(out, c->master, sizeof(double) * c->k * c->D,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return device_fail(const_cast<skm_ctx *>(c), "get_centroids", e);
  return SKM_OK;
}

skm_status skm_get_centroid_columns(const skm_ctx *c, const int32_t *terms, int32_t n_terms,
                                    double *out) {
  ST_TRY(check_ctx(c));
  if (n_terms < 0 || (n_terms > 0 && (!terms || !out)))
    return fail(SKM_E_INVALID, "terms or out is NULL");
  if (n_terms == 0) return SKM_OK;
  for (int32_t q = 0; q < n_terms; ++q)
    if (terms[q] < 0 || terms[q] >= c->D) return fail(SKM_E_INVALID, "term index out of range");
  int32_t *d_terms = nullptr;
  double *d_out = nullptr;
  if (hipMalloc(&d_terms, sizeof(int32_t) * n_terms) != hipSuccess ||
      hipMalloc(&d_out, sizeof(double) * n_terms * (size_t)c->k) != hipSuccess) {
    (void)hipGetLastError();
    if (d_terms) (void)hipFree(d_terms);
    return fail(SKM_E_NOMEM, "temporary device allocation failed");
  }
  hipStream_t s = c->stream;
  hipError_t e = hipMemcpyAsync(d_terms, terms, sizeof(int32_t) * n_terms, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_centroid_columns(c->master, c->k, c->D, d_terms, n_terms, d_out, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, d_out, sizeof(double) * n_terms * (size_t)c->k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_terms);
  (void)hipFree(d_out);
  if (e != hipSuccess) return device_fail(const_cast<skm_ctx *>(c), "get_centroid_columns", e);
  return SKM_OK;
}

skm_status skm_get_centroid_rows(const skm_ctx *c, const int32_t *ids, int32_t n, double *out) {
  ST_TRY(check_ctx(c));
  if (n < 0 || (n > 0 && (!ids || !out))) return fail(SKM_E_INVALID, "ids or out is NULL");
  for (int32_t q = 0; q < n; ++q)
    if (ids[q] < 0 || ids[q] >= c->k) return fail(SKM_E_INVALID, "centroid id out of range");
  hipError_t e = hipSuccess;
  for (int32_t q = 0; q < n && e == hipSuccess; ++q)
    e = hipMemcpyAsync(out + (size_t)q * c->D, c->master + (size_t)ids[q] * c->D,
                       sizeof(double) * c->D, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return device_fail(const_cast<skm_ctx *>(c), "get_centroid_rows", e);
  return SKM_OK;
}

skm_status skm_set_centroids(skm_ctx *c, const double *centroids) {
  ST_TRY(check_ctx_writable(c));
  if (!centroids) return fail(SKM_E_INVALID, "centroids is NULL");
  HIP_TRY(c, hipMemcpyAsync(c->master, centroids, sizeof(double) * c->k * c->D,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_fill_u8(c->sup_mvalid, 0, c->k, c->stream));   // supports unknown
  ST_TRY(rebuild_tiles(c, nullptr, nullptr));
  if (c->cfg.flags & SKM_INDEX) ST_TRY(build_index(c));
  HIP_TRY(c, launch_fill_u8(c->changed, 1, c->k, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->force_all = true;
  c->have_prev = false;
  c->assigned = false;
  c->last_changed = c->k;
  return SKM_OK;
}

// Checkpoint (file format and checks in host_checks.cpp): the assignment that
// made the centroids, the certified intervals, the changed flags, the run's
// counters and the centroids of the clusters with no members.  Every other
// centroid is the normalised sum of its members in ascending row order, so it
// is recomputed on load and comes out bit for bit the same.
constexpr uint32_t kStateFlags = SKM_NCC | SKM_INDEX | SKM_NO_EXACT | SKM_DENSE_ONLY;

skm_status skm_save(const skm_ctx *cc, const char *path) {
  ST_TRY(check_ctx(cc));
  skm_ctx *c = const_cast<skm_ctx *>(cc);
  if (!path) return fail(SKM_E_INVALID, "path is NULL");
  if (!c->have_prev) return fail(SKM_E_STATE, "a checkpoint needs a completed skm_update");
  // With an assignment pending (taken but not yet followed by its update) the
  // checkpoint holds the state before it: the assignment leaves a_prev, the
  // intervals, the flags and the master alone, and the resumed run repeats it.
  hipStream_t s = c->stream;
  const int64_t N = c->N, D = c->D;
  const int32_t k = c->k;
  std::vector<int32_t> a(N);
  std::vector<double> lo(N), hi(N);
  std::vector<uint8_t> ch(k);
  HIP_TRY(c, hipMemcpyAsync(a.data(), c->a_prev, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(lo.data(), c->lo_prev, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(hi.data(), c->hi_prev, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(ch.data(), c->changed, k, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  std::vector<int64_t> count(k, 0);
  for (int32_t j : a) {
    if (j < 0 || j >= k) return fail(SKM_E_STATE, "the assignment holds an invalid centroid id");
    count[j] += 1;
  }
  host::Checkpoint ck;
  std::vector<double> row(D);
  ck.e_off.push_back(0);
  for (int32_t j = 0; j < k; ++j) {
    if (count[j] != 0) continue;
    HIP_TRY(c, hipMemcpyAsync(row.data(), c->master + (size_t)j * D, sizeof(double) * D,
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    ck.e_ids.push_back(j);
    for (int64_t t = 0; t < D; ++t)
      if (row[t] != 0.0) {
        ck.e_terms.push_back((int32_t)t);
        ck.e_vals.push_back(row[t]);
      }
    ck.e_off.push_back((int64_t)ck.e_terms.size());
  }
  ck.k = k;
  ck.n_rows = N;
  ck.n_cols = D;
  ck.nnz = c->Z;
  ck.precision = c->prec;
  ck.flags = c->cfg.flags & kStateFlags;
  ck.iter = c->iter;
  ck.last_changed = c->last_changed;
  ck.last_moved = c->last_moved;
  ck.idx_skip = c->assigned ? c->idx_skip_pre : c->idx_skip;
  ck.idx_backoff = c->assigned ? c->idx_backoff_pre : c->idx_backoff;
  ck.index_ready = c->index_ready ? 1 : 0;
  ck.full_frac = c->full_frac;
  ck.a = std::move(a);
  ck.lo = std::move(lo);
  ck.hi = std::move(hi);
  ck.changed = std::move(ch);
  std::string why;
  if (!host::write_checkpoint(path, ck, &why)) return fail(SKM_E_INVALID, why);
  return SKM_OK;
}

skm_status skm_load(skm_ctx **out, const skm_csr *docs, const char *path, const skm_config *cfg) {
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg || !path) return fail(SKM_E_INVALID, "cfg or path is NULL");
  ST_TRY(check_csr_header(docs, 0));
  // the whole file is read and checked before any device work
  host::Checkpoint h;
  std::string why;
  if (!host::read_checkpoint(path, docs->n_rows, docs->n_cols, docs->nnz, &h, &why))
    return fail(SKM_E_INVALID, why);
  if (h.k != cfg->k || h.precision != cfg->precision || h.flags != (cfg->flags & kStateFlags))
    return fail(SKM_E_INVALID, std::string("checkpoint ") + path +
                                   ": k, precision or flags differ from cfg");
  const int64_t N = h.n_rows, D = h.n_cols;
  const int32_t k = h.k;
  const int64_t n_empty = (int64_t)h.e_ids.size();
  const std::vector<int32_t> &a = h.a, &e_ids = h.e_ids, &e_terms = h.e_terms;
  const std::vector<double> &lo = h.lo, &hi = h.hi, &e_vals = h.e_vals;
  const std::vector<int64_t> &e_off = h.e_off;
  const std::vector<uint8_t> &ch = h.changed;

  // A context seeded from stand-in rows; then the saved state replaces it.
  std::vector<int32_t> rows(k);
  for (int32_t j = 0; j < k; ++j) rows[j] = j;
  skm_config c2 = *cfg;
  c2.init_rows = rows.data();
  c2.init_centroids = nullptr;
  skm_ctx *c = nullptr;
  ST_TRY(skm_init(docs, &c2, &c));
  auto cleanup = [&](skm_status st) {
    skm_destroy(c);
    return st;
  };
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  {
    // clusters without members keep the saved centroid through the update
    std::vector<double> row(D);
    for (int64_t q = 0; q < n_empty && e == hipSuccess; ++q) {
      std::fill(row.begin(), row.end(), 0.0);
      for (int64_t p = e_off[q]; p < e_off[q + 1]; ++p) row[e_terms[p]] = e_vals[p];
      e = hipMemcpyAsync(c->master + (size_t)e_ids[q] * D, row.data(), sizeof(double) * D,
                         hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(c->a, a.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->lo, lo.data(), sizeof(double) * N, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->hi, hi.data(), sizeof(double) * N, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(device_fail(c, "checkpoint upload", e));
  // every centroid from the saved assignment (the update swaps a, lo, hi into
  // their _prev slots), then the counters of the saved run
  c->assigned = true;
  c->force_all = true;
  c->have_prev = false;
  c->idx_skip = 0;
  skm_iter_stats st{};
  skm_status rs = skm_update(c, &st);
  if (rs != SKM_OK) return cleanup(rs);
  e = hipMemcpyAsync(c->changed, ch.data(), (size_t)k, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cleanup(device_fail(c, "checkpoint upload", e));
  c->iter = h.iter;
  c->last_changed = h.last_changed;
  c->last_moved = h.last_moved;
  c->idx_skip = h.idx_skip;
  c->idx_backoff = h.idx_backoff;
  c->index_ready = c->index_ready && h.index_ready;
  c->full_frac = h.full_frac;
  *out = c;
  return SKM_OK;
}

skm_status skm_get_tile(const skm_ctx *c, void *codes, size_t codes_bytes, float *scales,
                        int64_t *ld) {
  ST_TRY(check_ctx(c));
  const size_t need = (size_t)c->D * c->ld * c->esize;
  if (ld) *ld = c->ld;
  skm_ctx *m = const_cast<skm_ctx *>(c);
  if (codes) {
    if (codes_bytes < need) return fail(SKM_E_INVALID, "codes buffer too small");
    std::vector<uint8_t> blocked(need);
    HIP_TRY(m, hipMemcpyAsync(blocked.data(), c->tile, need, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(m, hipStreamSynchronize(c->stream));
    uint8_t *dst = static_cast<uint8_t *>(codes);
    for (int64_t t = 0; t < c->D; ++t)
      for (int64_t j0 = 0; j0 < c->ld; j0 += kChunk)
        std::memcpy(dst + (t * c->ld + j0) * c->esize, blocked.data() + tile_index(t, j0, c->D) * c->esize,
                    (size_t)kChunk * c->esize);
  }
  if (scales)
    HIP_TRY(m, hipMemcpyAsync(scales, c->scale, sizeof(float) * c->k, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(m, hipStreamSynchronize(c->stream));
  return SKM_OK;
}

skm_status skm_get_changed(const skm_ctx *c, uint8_t *out) {
  ST_TRY(check_ctx(c));
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  HIP_TRY(const_cast<skm_ctx *>(c),
          hipMemcpyAsync(out, c->changed, c->k, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(const_cast<skm_ctx *>(c), hipStreamSynchronize(c->stream));
  return SKM_OK;
}

skm_status skm_score_dense(skm_ctx *c, const skm_csr *docs, float *out) {
  ST_TRY(check_ctx(c));
  ST_TRY(check_csr_header(docs, c->D));
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  const int64_t n = docs->n_rows;
  if (n == 0) return SKM_OK;
  std::vector<void *> tmp;
  auto talloc = [&](auto **p, size_t bytes) -> skm_status {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(bytes, 1)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SKM_E_NOMEM, "temporary device allocation failed");
    }
    tmp.push_back(q);
    *p = static_cast<std::remove_reference_t<decltype(*p)>>(q);
    return SKM_OK;
  };
  auto release = [&]() {
    for (void *q : tmp) (void)hipFree(q);
  };
  DevRows r;
  skm_status st = upload_rows(c, docs, c->D, false, c->stream, talloc, &r);
  float *d_out = nullptr;
  if (st == SKM_OK) st = talloc(&d_out, sizeof(float) * n * c->k);
  if (st != SKM_OK) {
    release();
    return st;
  }
  hipError_t e = launch_score_dense(r.indptr, r.indices, r.values, n, c->tile, c->D, c->k, c->scale,
                                    tail_view(c, 0), c->prec, nullptr, 0, d_out, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, d_out, sizeof(float) * n * c->k, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  release();
  if (e != hipSuccess) return device_fail(c, "score_dense", e);
  return SKM_OK;
}

skm_status skm_kmeanspp(const skm_csr *docs, int32_t k, const uint64_t *draws, int32_t *out_rows,
                        void *stream) {
  ST_TRY(check_csr_header(docs, 0));
  if (!draws || !out_rows) return fail(SKM_E_INVALID, "draws or out_rows is NULL");
  const int64_t n = docs->n_rows, D = docs->n_cols;
  if (k < 1 || (int64_t)k > n) return fail(SKM_E_INVALID, "k must be in [1, n_rows]");
  // a scratch context carries this call's device, stream and error state
  skm_ctx *c = new (std::nothrow) skm_ctx();
  if (!c) return fail(SKM_E_NOMEM, "host allocation failed");
  std::vector<void *> tmp;
  auto finish = [&](skm_status st) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *q : tmp) (void)hipFree(q);
    skm_destroy(c);
    return st;
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return finish(device_fail(nullptr, "hipGetDevice", e));
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return finish(device_fail(nullptr, "hipStreamCreate", e));
    c->own_stream = true;
  }
  hipStream_t s = c->stream;
  auto talloc = [&](auto **p, size_t bytes) -> skm_status {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(bytes, 1)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SKM_E_NOMEM, "temporary device allocation failed");
    }
    tmp.push_back(q);
    *p = static_cast<std::remove_reference_t<decltype(*p)>>(q);
    return SKM_OK;
  };
  DevRows r;
  skm_status st = upload_rows(c, docs, D, true, s, talloc, &r);
  const int64_t nb = (n + 255) / 256;
  double *best = nullptr, *dense = nullptr, *nrm2 = nullptr;
  uint64_t *w = nullptr, *bsum = nullptr;
  uint8_t *chosen = nullptr;
  int32_t *rows = nullptr;
  if (st == SKM_OK) st = talloc(&best, sizeof(double) * n);
  if (st == SKM_OK) st = talloc(&dense, sizeof(double) * D);
  if (st == SKM_OK) st = talloc(&nrm2, sizeof(double));
  if (st == SKM_OK) st = talloc(&w, sizeof(uint64_t) * n);
  if (st == SKM_OK) st = talloc(&bsum, sizeof(uint64_t) * nb);
  if (st == SKM_OK) st = talloc(&chosen, (size_t)n);
  if (st == SKM_OK) st = talloc(&rows, sizeof(int32_t) * k);
  if (st != SKM_OK) return finish(st);
  const int32_t r0 = (int32_t)(draws[0] % (uint64_t)n);
  e = launch_fill_f64(best, 0.0, n, s);
  if (e == hipSuccess) e = launch_fill_f64(dense, 0.0, D, s);
  if (e == hipSuccess) e = launch_fill_u8(chosen, 0, n, s);
  if (e == hipSuccess) e = launch_fill_u8(chosen + r0, 1, 1, s);
  if (e == hipSuccess) e = hipMemcpyAsync(rows, &r0, sizeof(int32_t), hipMemcpyHostToDevice, s);
  for (int32_t m = 1; m < k && e == hipSuccess; ++m) {
    double h_nrm2 = 0.0;
    e = pp_place(r.indptr, r.indices, r.values, n, rows, m, dense, nrm2, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_nrm2, nrm2, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    if (!(h_nrm2 > 0.0)) return finish(fail(SKM_E_DEVICE, "k-means++ lost its seed row"));
    // the length on the host: one correctly rounded square root
    e = pp_weights(r.indptr, r.indices, r.values, n, dense, std::sqrt(h_nrm2), best, chosen, w, bsum,
                   s);
    if (e == hipSuccess) e = pp_select(bsum, w, n, draws[m], chosen, rows, m, s);
  }
  std::vector<int32_t> h(k);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), rows, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return finish(device_fail(nullptr, "kmeanspp", e));
  for (int32_t m = 0; m < k; ++m)
    if (h[m] < 0 || h[m] >= n) return finish(fail(SKM_E_DEVICE, "k-means++ drew no row"));
  std::memcpy(out_rows, h.data(), sizeof(int32_t) * k);
  return finish(SKM_OK);
}

int32_t skm_head_terms(const skm_ctx *c) { return c ? c->head_H : 0; }

skm_status skm_score_head(skm_ctx *c, int64_t row0, int64_t n_rows, float *out,
                          float *out_head) {
  ST_TRY(check_ctx(c));
  if (!out) return fail(SKM_E_INVALID, "out is NULL");
  if (c->head_H <= 0) return fail(SKM_E_STATE, "this context scores no head terms");
  if (row0 < 0 || n_rows < 0 || row0 + n_rows > c->N || n_rows * c->k_pad > c->hs_cap)
    return fail(SKM_E_INVALID, "row range outside the context or larger than one head batch");
  if (n_rows == 0) return SKM_OK;
  float *d_out = nullptr, *d_head = nullptr;
  const size_t bytes = sizeof(float) * n_rows * c->k;
  if (hipMalloc(&d_out, bytes) != hipSuccess || (out_head && hipMalloc(&d_head, bytes) != hipSuccess)) {
    (void)hipGetLastError();
    if (d_out) (void)hipFree(d_out);
    return fail(SKM_E_NOMEM, "temporary device allocation failed");
  }
  // all centroid columns of these rows at once (the batch buffer holds them)
  hipError_t e = launch_head_gemm(c->xh, c->head_H, row0, n_rows, nullptr, c->ch_head, 0, c->k_pad,
                                  c->hs, c->k_pad, c->stream);
  if (e == hipSuccess)
    e = launch_score_dense(c->r_indptr + row0, c->r_indices, c->r_values, n_rows, c->tile, c->D,
                           c->k, c->scale, tail_view(c, 0), c->prec, c->hs, c->k_pad, d_out,
                           c->stream, d_head);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, bytes, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && out_head)
    e = hipMemcpyAsync(out_head, d_head, bytes, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d_out);
  if (d_head) (void)hipFree(d_head);
  if (e != hipSuccess) return device_fail(c, "score_head", e);
  return SKM_OK;
}

double skm_error_bound_head(const skm_ctx *c, double s, int64_t nnz, double l1) {
  if (!c || c->head_H <= 0) return -1.0;
  return bound_kappa_head(nnz, c->head_H, c->uq) * s + bound_abs(nnz, l1, c->abs_coef) +
         bound_abs_head(c->head_H, l1, c->abs_coef);
}

double skm_error_bound_split(const skm_ctx *c, double hs, double rs, int64_t n_rest, double l1) {
  if (!c || c->head_H <= 0 || c->prec != SKM_FP8_E4M3) return -1.0;
  const double A = bound_abs(n_rest, l1, c->abs_coef) + (double)c->head_H * 0x1p-120;
  return bound_split(hs, rs, bound_kappa_head_bf16(c->head_H), bound_kappa(n_rest, c->uq), A);
}

double skm_error_bound(const skm_ctx *c, double s, int64_t nnz, double l1) {
  if (!c) return -1.0;
  return bound_kappa(nnz, c->uq) * s + bound_abs(nnz, l1, c->abs_coef);
}

skm_status skm_get_index(const skm_ctx *c, int32_t level, int64_t *offsets, uint32_t *entries,
                         int64_t *n_entries) {
  ST_TRY(check_ctx(c));
  if (!(c->cfg.flags & SKM_INDEX) || !c->index_ready)
    return fail(SKM_E_STATE, "the index is not built (SKM_INDEX not set)");
  if (level < 0 || level >= c->cfg.n_lambda) return fail(SKM_E_INVALID, "level out of range");
  if (!offsets || !n_entries) return fail(SKM_E_INVALID, "offsets / n_entries is NULL");
  skm_ctx *m = const_cast<skm_ctx *>(c);
  const int64_t D = c->D, k = c->k, EG = c->idx_g_entries;
  const int64_t nd = (int64_t)c->idx_h_dids.size();
  std::vector<int64_t> toff(D + 1), toff2(D + 1, 0), qstart(k);
  std::vector<int32_t> cnt(k);
  std::vector<uint2> G(std::max<int64_t>(EG, 1));
  std::vector<double> Q(std::max<int64_t>(c->idx_used_q, 1));
  HIP_TRY(m, hipMemcpyAsync(toff.data(), c->idx_toff, 8 * (D + 1), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(m, hipMemcpyAsync(cnt.data(), c->idx_cnt, 4 * k, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(m, hipMemcpyAsync(qstart.data(), c->idx_qstart, 8 * k, hipMemcpyDeviceToHost, c->stream));
  if (EG > 0) HIP_TRY(m, hipMemcpyAsync(G.data(), c->idx_G, 8 * EG, hipMemcpyDeviceToHost, c->stream));
  if (c->idx_used_q > 0)
    HIP_TRY(m, hipMemcpyAsync(Q.data(), c->idx_Q, 8 * c->idx_used_q, hipMemcpyDeviceToHost,
                              c->stream));
  if (nd > 0)
    HIP_TRY(m, hipMemcpyAsync(toff2.data(), c->idx_toff2, 8 * (D + 1), hipMemcpyDeviceToHost,
                              c->stream));
  HIP_TRY(m, hipStreamSynchronize(c->stream));
  std::vector<uint2> G2(std::max<int64_t>(toff2[D], 1));
  if (toff2[D] > 0) {
    HIP_TRY(m, hipMemcpyAsync(G2.data(), c->idx_G2, 8 * toff2[D], hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(m, hipStreamSynchronize(c->stream));
  }
  const double lam = c->cfg.lambda[level];
  // m_p = least m with Q_j[min(p + m, n_j)] - Q_j[p] >= thr (the query's
  // threshold for centroid j); no P entry when none.  A term's (centroid,
  // position) pairs: those of G of centroids not rebuilt since the last full
  // build, and those of G2, ascending by centroid.
  int64_t n = 0;
  offsets[0] = 0;
  std::vector<uint2> pairs;
  for (int64_t t = 0; t < D; ++t) {
    pairs.clear();
    for (int64_t g = toff[t]; g < toff[t + 1]; ++g)
      if (nd == 0 || !c->idx_h_dirty[G[g].x]) pairs.push_back(G[g]);
    for (int64_t g = toff2[t]; g < toff2[t + 1]; ++g) pairs.push_back(G2[g]);
    std::sort(pairs.begin(), pairs.end(), [](const uint2 &x, const uint2 &y) { return x.x < y.x; });
    for (const uint2 &pr : pairs) {
      const int64_t j = pr.x, p = pr.y, nj = cnt[j];
      const double *q = Q.data() + qstart[j];
      const double thr = index_threshold(lam, nj, q[nj]);
      if (q[nj] - q[p] < thr) continue;
      int64_t lo = 1, hi = nj - p;
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (q[p + mid] - q[p] >= thr) hi = mid;
        else lo = mid + 1;
      }
      if (entries) entries[n] = (uint32_t)(j << 16) | (uint32_t)std::min<int64_t>(lo, 0xFFFF);
      ++n;
    }
    offsets[t + 1] = n;
  }
  *n_entries = n;
  return SKM_OK;
}

skm_status skm_index_query(skm_ctx *c, const skm_csr *docs, int32_t level, int64_t *offsets,
                           int32_t *cand, int64_t cap) {
  ST_TRY(check_ctx(c));
  ST_TRY(check_csr_header(docs, c->D));
  if (!(c->cfg.flags & SKM_INDEX) || !c->index_ready)
    return fail(SKM_E_STATE, "the index is not built (SKM_INDEX not set)");
  if (level < 0 || level >= c->cfg.n_lambda) return fail(SKM_E_INVALID, "level out of range");
  if (!offsets || (!cand && cap > 0)) return fail(SKM_E_INVALID, "output pointer is NULL");
  const int64_t n = docs->n_rows;
  offsets[0] = 0;
  if (n == 0) return SKM_OK;
  std::vector<void *> tmp;
  auto talloc = [&](auto **p, size_t bytes) -> skm_status {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(bytes, 1)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SKM_E_NOMEM, "temporary device allocation failed");
    }
    tmp.push_back(q);
    *p = static_cast<std::remove_reference_t<decltype(*p)>>(q);
    return SKM_OK;
  };
  auto release = [&]() {
    for (void *q : tmp) (void)hipFree(q);
  };
  DevRows r;
  skm_status st = upload_rows(c, docs, c->D, false, c->stream, talloc, &r);
  int32_t *rows = nullptr, *dcand = nullptr, *ncand = nullptr, *lvl = nullptr;
  unsigned long long *stat = nullptr;
  if (st == SKM_OK) st = talloc(&rows, 4 * n);
  if (st == SKM_OK) st = talloc(&dcand, 4 * n * (int64_t)c->k);
  if (st == SKM_OK) st = talloc(&ncand, 4 * n);
  if (st == SKM_OK) st = talloc(&lvl, 4 * n);
  if (st == SKM_OK) st = talloc(&stat, 128);
  if (st != SKM_OK) {
    release();
    return st;
  }
  std::vector<int32_t> hrows(n);
  for (int64_t i = 0; i < n; ++i) hrows[i] = (int32_t)i;
  IndexArgs x = index_args(c);
  x.indptr = r.indptr;
  x.indices = r.indices;
  x.values = r.values;
  x.xl2 = r.xl2;
  x.rows = rows;
  x.a_prev = nullptr;
  x.forced_level = level;
  x.guard = 1e300;
  x.cap = c->k;
  x.cand = dcand;
  x.ncand = ncand;
  x.level = lvl;
  x.mode = nullptr;
  x.stat = stat;
  std::vector<int32_t> hn(n);
  hipError_t e = hipMemcpyAsync(rows, hrows.data(), 4 * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t *>(stat), 0, 32, c->stream);
  if (e == hipSuccess) e = index_query(x, n, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hn.data(), ncand, 4 * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    release();
    return device_fail(c, "skm_index_query", e);
  }
  for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + hn[i];
  if (offsets[n] > cap) {
    release();
    return fail(SKM_E_INVALID, "cand buffer too small");
  }
  for (int64_t i = 0; i < n && e == hipSuccess; ++i)
    if (hn[i] > 0)
      e = hipMemcpyAsync(cand + offsets[i], dcand + i * (int64_t)c->k, 4 * hn[i],
                         hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  release();
  if (e != hipSuccess) return device_fail(c, "skm_index_query copy", e);
  return SKM_OK;
}

}  // extern "C"
