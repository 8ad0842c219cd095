// The dot-product index of paper Sec. 3.2 on the GPU.
//
// Build (from the FP64 master):
//   - every centroid's non-zero entries, sorted by value descending (equal
//     values: ascending term), with the FP64 prefix sums Q_j of their squares
//     (a segment per centroid at sstart[j] with cnt[j] entries, its prefix
//     sums at qstart[j]);
//   - G: for every term t, the centroids with a non-zero at t, ascending, each
//     with the term's position p in that centroid's sorted order.
// After an update only the changed centroids are rebuilt: their new segments
// are appended behind the others, they are marked dirty, their entries in G
// are skipped, and G2 holds the (centroid, position) entries of every dirty
// centroid, term-major.  A full build (when the dirty entries exceed a
// quarter of all, or the buffers run out) compacts everything into G again.
// The paper's minimum overlap count of position p for threshold lam is
//   m_p = least m with Q_j[min(p + m, n_j)] - Q_j[p] >= lam^2,
// and the positions entering P are those where such an m exists.  m_p is
// non-decreasing in p, so "some overlapping term t of x has (j, m_p) in P with
// count_j >= m_p" holds exactly when it holds at the highest-valued overlapping
// position p*: the query computes count_j and p*_j from G and tests
//   Q_j[min(p*_j + count_j, n_j)] - Q_j[p*_j] >= lam^2,
// which returns the same set as the paper's two-map query.  Sums are compared
// against index_threshold (internal.h): lam^2 less a margin derived from the
// prefix kernel's summation order, so FP64 rounding of the prefix
// differences can only enlarge the candidate set.
#include <algorithm>

#include "internal.h"

namespace skm {
namespace {

constexpr int kRun = 2048;   // LDS sort run

__device__ inline bool key_less(uint64_t ka, int32_t ta, uint64_t kb, int32_t tb) {
  return ka < kb || (ka == kb && ta < tb);
}

// Non-zeros per centroid (the listed ones, or all when ids is nullptr).
__global__ __launch_bounds__(256) void k_centroid_nnz(const double *master, int64_t D,
                                                      const int32_t *ids, int32_t *cnt) {
  __shared__ int32_t sh[256];
  const int j = ids ? ids[blockIdx.x] : blockIdx.x;
  int c = 0;
  for (int64_t t = threadIdx.x; t < D; t += 256) c += master[(int64_t)j * D + t] != 0.0;
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[j] = sh[0];
}

// Segments of the listed centroids (all when ids is nullptr), in list order
// from base_e (entries) and base_q (prefix sums, one more each):
// sstart[j] = base_e + entries before j, qstart[j] = base_q + the same + i
// for the i-th listed centroid; tot = {entries, prefix-sum slots}.  One
// workgroup of 1024 threads, each scanning a contiguous piece of the list.
__global__ __launch_bounds__(1024) void k_place(const int32_t *ids, int64_t n, const int32_t *cnt,
                                                int64_t base_e, int64_t base_q, int64_t *sstart,
                                                int64_t *qstart, int64_t *tot) {
  __shared__ int64_t sh[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = min<int64_t>(t * per, n), hi = min(n, lo + per);
  int64_t c = 0;
  for (int64_t i = lo; i < hi; ++i) c += cnt[ids ? ids[i] : i];
  sh[t] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int64_t pos = sh[t] - c;
  for (int64_t i = lo; i < hi; ++i) {
    const int64_t j = ids ? ids[i] : i;
    sstart[j] = base_e + pos;
    qstart[j] = base_q + pos + i;
    pos += cnt[j];
  }
  if (t == 1023) {
    tot[0] = sh[1023];
    tot[1] = sh[1023] + n;
  }
}

// Entries of centroid j: key = ~bits(value) (ascending key = descending
// value, values are positive), term.  Coalesced sweeps of the FP64 row, each
// wavefront appending its non-zeros by ballot at a workgroup counter; the
// order within the segment is arbitrary, since the sort orders the (key,
// term) pairs, which are unique, completely.
__global__ __launch_bounds__(256) void k_extract(const double *master, int64_t D, const int32_t *ids,
                                                 const int64_t *sstart, uint64_t *key,
                                                 int32_t *term) {
  __shared__ int32_t fill;
  const int j = ids ? ids[blockIdx.x] : blockIdx.x;
  const double *row = master + (int64_t)j * D;
  const int64_t base = sstart[j];
  const int lane = lane_id();
  if (threadIdx.x == 0) fill = 0;
  __syncthreads();
  for (int64_t t0 = 0; t0 < D; t0 += 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t t = t0 + u * 256 + threadIdx.x;
      v[u] = t < D ? row[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t t = t0 + u * 256 + threadIdx.x;
      const bool nz = v[u] != 0.0;
      const uint64_t m = __ballot(nz);
      int wb = 0;
      if (lane == 0 && m) wb = atomicAdd(&fill, __popcll(m));
      wb = __shfl(wb, 0, kWave);
      if (nz) {
        const int64_t p = base + wb + __popcll(m & lanemask_lt());
        key[p] = ~(uint64_t)__double_as_longlong(v[u]);
        term[p] = (int32_t)t;
      }
    }
  }
}

// Merge-path co-rank: number of elements of A among the first o outputs of
// merge(A, B) (keys are unique within a centroid).
__device__ inline int64_t corank(int64_t o, const uint64_t *ka, const int32_t *ta, int64_t na,
                                 const uint64_t *kb, const int32_t *tb, int64_t nb) {
  int64_t lo = o > nb ? o - nb : 0, hi = o < na ? o : na;
  while (lo < hi) {
    const int64_t i = (lo + hi) / 2, j = o - i;
    const bool too_small = i < na && j > 0 && !key_less(kb[j - 1], tb[j - 1], ka[i], ta[i]);
    if (too_small) lo = i + 1;
    else hi = i;
  }
  return lo;
}

// Segments are sorted ascending by (key, term) in two stages spread over the
// whole GPU, so that one long centroid does not hold a build up: every run of
// kRun entries is sorted by a workgroup in LDS (bitonic), then merge passes of
// width w = kRun, 2 kRun, ... between the two buffers, each workgroup producing
// one tile of kRun outputs of one merge (a tile never straddles two merges:
// both are aligned to kRun and merges span 2w).  runs / tiles list (centroid,
// first entry within its segment).

__global__ __launch_bounds__(256) void k_sort_runs(const int2 *runs, const int64_t *sstart,
                                                   const int32_t *cnt, uint64_t *key,
                                                   int32_t *term) {
  __shared__ uint64_t sk[kRun];
  __shared__ int32_t st[kRun];
  const int2 rr = runs[blockIdx.x];
  const int64_t s0 = sstart[rr.x] + rr.y;
  const int64_t m = min<int64_t>(kRun, (int64_t)cnt[rr.x] - rr.y);
  for (int i = threadIdx.x; i < kRun; i += 256) {
    sk[i] = i < m ? key[s0 + i] : ~0ull;
    st[i] = i < m ? term[s0 + i] : 0x7FFFFFFF;
  }
  __syncthreads();
  for (int size = 2; size <= kRun; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < kRun / 2; i += 256) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const bool gt = key_less(sk[hi], st[hi], sk[lo], st[lo]);
        if (gt == up) {
          const uint64_t k2 = sk[lo];
          sk[lo] = sk[hi];
          sk[hi] = k2;
          const int32_t t2 = st[lo];
          st[lo] = st[hi];
          st[hi] = t2;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < m; i += 256) {
    key[s0 + i] = sk[i];
    term[s0 + i] = st[i];
  }
}

// One merge pass of width w (src -> dst); a merge with one run copies it.
// Each thread produces kRun / 256 consecutive outputs from its own co-rank.
__global__ __launch_bounds__(256) void k_merge_pass(const int2 *tiles, const int64_t *sstart,
                                                    const int32_t *cnt, int64_t w,
                                                    const uint64_t *ks, const int32_t *ts,
                                                    uint64_t *kd, int32_t *td) {
  constexpr int kPer = kRun / 256;
  const int2 tl = tiles[blockIdx.x];
  const int64_t s0 = sstart[tl.x], n = cnt[tl.x];
  const int64_t a = ((int64_t)tl.y / (2 * w)) * (2 * w);   // first entry of the merge
  const int64_t na = min(w, n - a), nb = max<int64_t>(0, min(w, n - a - w));
  const int64_t len = na + nb;
  const uint64_t *KA = ks + s0 + a, *KB = KA + na;
  const int32_t *TA = ts + s0 + a, *TB = TA + na;
  const int64_t o0 = (int64_t)tl.y - a + (int64_t)threadIdx.x * kPer;
  if (o0 >= len) return;
  const int64_t o1 = min<int64_t>(o0 + kPer, len);
  int64_t i = corank(o0, KA, TA, na, KB, TB, nb);
  int64_t j = o0 - i;
  for (int64_t o = o0; o < o1; ++o) {
    const bool takeB = j < nb && (i >= na || key_less(KB[j], TB[j], KA[i], TA[i]));
    if (takeB) {
      kd[s0 + a + o] = KB[j];
      td[s0 + a + o] = TB[j];
      ++j;
    } else {
      kd[s0 + a + o] = KA[i];
      td[s0 + a + o] = TA[i];
      ++i;
    }
  }
}

// Copies the listed tiles (kRun entries each) from src to dst.
__global__ __launch_bounds__(256) void k_copy_tiles(const int2 *tiles, const int64_t *sstart,
                                                    const int32_t *cnt, const uint64_t *ks,
                                                    const int32_t *ts, uint64_t *kd, int32_t *td) {
  const int2 tl = tiles[blockIdx.x];
  const int64_t s0 = sstart[tl.x] + tl.y;
  const int64_t m = min<int64_t>(kRun, (int64_t)cnt[tl.x] - tl.y);
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    kd[s0 + i] = ks[s0 + i];
    td[s0 + i] = ts[s0 + i];
  }
}

// Q_j[0] = 0, Q_j[p + 1] = Q_j[p] + v_p^2 over the sorted entries (fixed
// per-thread pieces + block scan: deterministic).  Q_j starts at qstart[j].
__global__ __launch_bounds__(256) void k_prefix_sq(const int32_t *ids, const int64_t *sstart,
                                                   const int32_t *cnt, const int64_t *qstart,
                                                   const uint64_t *key, double *Q) {
  __shared__ double sh[256];
  const int j = ids ? ids[blockIdx.x] : blockIdx.x;
  const int64_t s0 = sstart[j], n = cnt[j];
  double *q = Q + qstart[j];
  const int64_t per = (n + 255) / 256;
  const int64_t lo = min<int64_t>((int64_t)threadIdx.x * per, n), hi = min(n, lo + per);
  double c = 0.0;
  for (int64_t p = lo; p < hi; ++p) {
    const double v = __longlong_as_double((long long)~key[s0 + p]);
    c += v * v;
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    double v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  double run = sh[threadIdx.x] - c;
  if (threadIdx.x == 0) q[0] = 0.0;
  for (int64_t p = lo; p < hi; ++p) {
    const double v = __longlong_as_double((long long)~key[s0 + p]);
    run += v * v;
    q[p + 1] = run;
  }
}

// Non-zero masks, term-major, over the listed centroids (all k when ids is
// nullptr): mask[t * nb + b] bit i = (c_{ids[64b+i], t} != 0).
__global__ __launch_bounds__(256) void k_term_masks(const double *master, const int32_t *ids,
                                                    int32_t k, int64_t D, int64_t nb,
                                                    uint64_t *mask) {
  __shared__ uint8_t nz[64][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64, t0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = j0 + jj, t = t0 + tx;
    const int64_t j = i < k ? (ids ? (int64_t)ids[i] : i) : 0;
    nz[jj][tx] = (i < k && t < D) ? (master[j * D + t] != 0.0) : 0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int64_t t = t0 + threadIdx.x;
    if (t < D) {
      uint64_t m = 0;
      for (int jj = 0; jj < 64; ++jj) m |= (uint64_t)nz[jj][threadIdx.x] << jj;
      mask[t * nb + blockIdx.x] = m;
    }
  }
}

// Per term: exclusive prefix of mask popcounts over its blocks, total count.
__global__ void k_term_prefix(const uint64_t *mask, int64_t D, int64_t nb, int32_t *blkpre,
                              int32_t *tcnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= D) return;
  int32_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    blkpre[t * nb + b] = run;
    run += __popcll(mask[t * nb + b]);
  }
  tcnt[t] = run;
}

// G entries: (centroid, position) at term t's slot ordered by centroid.
__global__ __launch_bounds__(256) void k_fill_G(const int32_t *ids, const int64_t *sstart,
                                                const int32_t *cnt, const int32_t *term,
                                                const uint64_t *mask, const int32_t *blkpre,
                                                const int64_t *toff, int64_t nb, uint2 *G) {
  const int i = blockIdx.x;                    // list index (column of the masks)
  const int j = ids ? ids[i] : i;
  const int64_t s0 = sstart[j], n = cnt[j];
  const int64_t b = i >> 6;
  const uint64_t below = (i & 63) ? (~0ull >> (64 - (i & 63))) : 0ull;
  for (int64_t p = threadIdx.x; p < n; p += 256) {
    const int64_t t = term[s0 + p];
    const int64_t pos = toff[t] + blkpre[t * nb + b] + __popcll(mask[t * nb + b] & below);
    G[pos] = make_uint2((uint32_t)j, (uint32_t)p);
  }
}

// Bit j of bits[j / 32] = dirty[j].
__global__ void k_dirty_bits(const uint8_t *dirty, int32_t k, uint32_t *bits) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w * 32 >= k) return;
  uint32_t m = 0;
  for (int i = 0; i < 32 && w * 32 + i < k; ++i) m |= (dirty[w * 32 + i] ? 1u : 0u) << i;
  bits[w] = m;
}

__global__ void k_scan_i32_to_i64(const int32_t *cnt, int64_t n, int64_t *off) {
  // single workgroup of 1024 threads, chunked exclusive scan
  __shared__ int64_t sh[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = min<int64_t>(t * per, n), hi = min(n, lo + per);
  int64_t c = 0;
  for (int64_t i = lo; i < hi; ++i) c += cnt[i];
  sh[t] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t v = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int64_t pos = sh[t] - c;
  for (int64_t i = lo; i < hi; ++i) {
    off[i] = pos;
    pos += cnt[i];
  }
  if (t == 1023) off[n] = sh[1023];
}

// ---------------------------------------------------------------- query

// Index path for the rows in `rows`.  One workgroup per row:
//   1. baseline b = x . c_{a_prev} in FP64 (the current centroid of the previous
//      assignment), b_lo = b - err; level = highest lam with lam * ||x|| <= b_lo;
//   2. cost guard: the query reads sum_t |G[t]| entries; when that exceeds
//      guard * nnz * (centroids the row would otherwise score) the dense scan
//      is cheaper and the row stays dense;
//   3. overlap counts and highest-valued positions in LDS, the candidate test
//      above, candidates ascending into cand[slot * cap ...] (dense fallback
//      when more than cap survive).
// With x.changed (Sec. 3.1 and 3.2 together, the combination the end of
// Sec. 3.2 describes): a row whose previous centroid did not change can only
// move to a changed centroid that beats it, so its candidates are the index's
// candidates that changed (its baseline is the unchanged previous centroid's
// score), and the alternative it is guarded against scores n_ch centroids.
// mode[row] = 2 marks rows finished here (scored by k_index_score).
// Dirty centroids (rebuilt since the last full build) are taken from G2, their
// stale entries in G skipped by a bitmap in LDS.
__global__ __launch_bounds__(256) void k_index_query(IndexArgs x) {
  extern __shared__ uint32_t lds[];
  uint32_t *pmin = lds;                        // k positions
  uint32_t *cnt = lds + x.k;                   // k counts, two 16-bit counts per word
  uint32_t *dbits = cnt + (x.k + 1) / 2;       // dirty bitmap, k bits
  __shared__ double red[256];
  __shared__ int32_t sh_i[256];
  __shared__ int s_level;
  const int64_t slot = blockIdx.x;
  const int64_t row = x.rows ? (int64_t)x.rows[slot] : slot;
  const int64_t b = x.indptr[row], e = x.indptr[row + 1], n = e - b;
  const int32_t ap = x.a_prev ? x.a_prev[row] : 0;
  const bool keep_row = x.changed && x.a_prev && !x.changed[ap];
  // 1. baseline
  double part = 0.0;
  if (x.a_prev)
    for (int64_t q = b + threadIdx.x; q < e; q += 256)
      part = fma((double)x.values[q], x.master[(int64_t)ap * x.D + x.indices[q]], part);
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double base = red[0];
  const double blo = base - exact_err(n, base);
  if (x.base_out && threadIdx.x == 0) x.base_out[slot] = blo;
  const double xn = x.xl2[row] * (1.0 + 0x1p-40);
  // 2. cost guard
  double gsum = 0.0;
  for (int64_t q = b + threadIdx.x; q < e; q += 256) {
    const int32_t t = x.indices[q];
    gsum += (double)(x.toff[t + 1] - x.toff[t]);
    if (x.n_dirty > 0) gsum += (double)(x.toff2[t + 1] - x.toff2[t]);
  }
  __syncthreads();
  red[threadIdx.x] = gsum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int lv = -1;
    for (int l = 0; l < x.n_lambda; ++l)
      if (x.lambda[l] * xn <= blo) lv = l;
    const double alt = keep_row ? (double)x.n_ch : (double)x.k;
    if (x.forced_level >= 0) lv = x.forced_level;
    else if (lv >= 0 && red[0] > x.guard * (double)n * alt) lv = -2;
    s_level = lv;
  }
  __syncthreads();
  const int level = s_level;
  if (level < 0) {
    if (threadIdx.x == 0) {
      x.ncand[slot] = -1;
      atomicAdd(&x.stat[level == -1 ? 5 : 6], 1ull);
    }
    return;
  }
  // 3. counts and best positions
  for (int j = threadIdx.x; j < x.k; j += 256) pmin[j] = 0xFFFFFFFFu;
  for (int j = threadIdx.x; j < (x.k + 1) / 2; j += 256) cnt[j] = 0;
  const bool delta = x.n_dirty > 0;
  if (delta)
    for (int w = threadIdx.x; w < (x.k + 31) / 32; w += 256) dbits[w] = x.dbits[w];
  __syncthreads();
  for (int64_t q = b; q < e; ++q) {
    const int32_t t = x.indices[q];
    for (int64_t g = x.toff[t] + threadIdx.x; g < x.toff[t + 1]; g += 256) {
      const uint2 ent = x.G[g];
      if (delta && ((dbits[ent.x >> 5] >> (ent.x & 31)) & 1u)) continue;
      atomicAdd(&cnt[ent.x >> 1], 1u << (16 * (ent.x & 1)));
      atomicMin(&pmin[ent.x], ent.y);
    }
    if (delta) {
      for (int64_t g = x.toff2[t] + threadIdx.x; g < x.toff2[t + 1]; g += 256) {
        const uint2 ent = x.G2[g];
        atomicAdd(&cnt[ent.x >> 1], 1u << (16 * (ent.x & 1)));
        atomicMin(&pmin[ent.x], ent.y);
      }
    }
  }
  __syncthreads();
  const double lam = x.lambda[level];
  int total = 0;
  for (int j0 = 0; j0 < x.k; j0 += 256) {
    const int j = j0 + threadIdx.x;
    int in = 0;
    const uint32_t cj = j < x.k ? (cnt[j >> 1] >> (16 * (j & 1))) & 0xFFFFu : 0u;
    if (cj > 0 && (!keep_row || x.changed[j])) {
      const int64_t nj = x.cnt[j];
      const int64_t p = pmin[j];
      const int64_t h = min<int64_t>(p + cj, nj);
      const double *Qj = x.Q + x.qstart[j];
      in = (Qj[h] - Qj[p] >= index_threshold(lam, nj, Qj[nj])) ? 1 : 0;
    }
    sh_i[threadIdx.x] = in;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      int v = (int)threadIdx.x >= off ? sh_i[threadIdx.x - off] : 0;
      __syncthreads();
      sh_i[threadIdx.x] += v;
      __syncthreads();
    }
    const int pos = total + sh_i[threadIdx.x] - in;
    if (in && pos < x.cap) x.cand[slot * x.cap + pos] = j;
    total += sh_i[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    x.ncand[slot] = total <= x.cap ? total : -1;
    x.level[slot] = level;
    if (total <= x.cap) {
      if (x.mode) x.mode[row] = 2;
      atomicAdd(&x.stat[2], 1ull);
      atomicAdd(&x.stat[0], (unsigned long long)total + 1ull);
      atomicAdd(&x.stat[3], (unsigned long long)(total + 1) * (unsigned long long)n);
    } else {
      atomicAdd(&x.stat[7], 1ull);
    }
  }
}

// FP64 exact scores of an index row's candidates plus its previous centroid;
// lowest index among the maxima.  One wavefront per row.
__global__ __launch_bounds__(256) void k_index_score(IndexArgs x, int64_t n_slots, int32_t *a_out,
                                                     double *lo_out, double *hi_out) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t slot = (int64_t)blockIdx.x * 4 + wave;
  if (slot >= n_slots) return;
  const int32_t nc = x.ncand[slot];
  if (nc < 0) return;
  const int64_t row = x.rows ? (int64_t)x.rows[slot] : slot;
  const int64_t b = x.indptr[row], e = x.indptr[row + 1];
  const int32_t ap = x.a_prev[row];
  double bs = -INFINITY;
  int bj = 0x7FFFFFFF;
  for (int i = lane; i <= nc; i += kWave) {
    const int j = i < nc ? x.cand[slot * x.cap + i] : ap;
    const double *c = x.master + (int64_t)j * x.D;
    const double s = dot64(b, e, x.indices, x.values, c);
    if (better_d(s, j, bs, bj)) {
      bs = s;
      bj = j;
    }
  }
  wave_best_d(bs, bj);
  if (lane == 0) {
    const double err = exact_err(e - b, bs);
    a_out[row] = bj;
    lo_out[row] = bs - err;
    hi_out[row] = bs + err;
  }
}

// Per term t, the centroid with the largest value at t (lowest index among
// equal values; -1 when no centroid has t), from the index entries: G (the
// centroids not rebuilt since the last full build) and G2.  One wavefront per
// term.
__global__ __launch_bounds__(256) void k_best_centroid(const int64_t *toff, const uint2 *G,
                                                       const int64_t *toff2, const uint2 *G2,
                                                       const uint8_t *dirty, int32_t n_dirty,
                                                       const int64_t *sstart, const uint64_t *key,
                                                       int64_t D, int32_t *best) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= D) return;
  const int lane = lane_id();
  double bv = -INFINITY;
  int bj = 0x7FFFFFFF;
  for (int64_t g = toff[t] + lane; g < toff[t + 1]; g += kWave) {
    const uint2 ent = G[g];
    if (n_dirty > 0 && dirty[ent.x]) continue;
    const double v = __longlong_as_double((long long)~key[sstart[ent.x] + ent.y]);
    if (better_d(v, (int)ent.x, bv, bj)) {
      bv = v;
      bj = (int)ent.x;
    }
  }
  if (n_dirty > 0) {
    for (int64_t g = toff2[t] + lane; g < toff2[t + 1]; g += kWave) {
      const uint2 ent = G2[g];
      const double v = __longlong_as_double((long long)~key[sstart[ent.x] + ent.y]);
      if (better_d(v, (int)ent.x, bv, bj)) {
        bv = v;
        bj = (int)ent.x;
      }
    }
  }
  wave_best_d(bv, bj);
  if (lane == 0) best[t] = bj == 0x7FFFFFFF ? -1 : bj;
}

// Probe centroid of each new row (baseline of the index query): among the
// centroids that are largest at the row's three largest values' terms, the
// one with the highest FP64 score (lowest index among equal scores); 0 when
// none of those terms is in any centroid.  One wavefront per row.
__global__ __launch_bounds__(256) void k_probe(const int64_t *indptr, const int32_t *indices,
                                               const float *values, int64_t n, const int32_t *best,
                                               const double *master, int64_t D, int32_t *probe) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int lane = lane_id();
  const int64_t b = indptr[row], e = indptr[row + 1];
  int cand[3] = {-1, -1, -1};
  int64_t taken[3] = {-1, -1, -1};
  for (int r = 0; r < 3; ++r) {
    // the largest value not yet taken (lowest position among equal values)
    float bv = -INFINITY;
    int64_t bq = INT64_MAX;
    for (int64_t q = b + lane; q < e; q += kWave) {
      if (q == taken[0] || q == taken[1]) continue;
      const float v = values[q];
      if (v > bv || (v == bv && q < bq)) {
        bv = v;
        bq = q;
      }
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
      const float ov = __shfl_xor(bv, m, kWave);
      const int64_t oq = __shfl_xor(bq, m, kWave);
      if (ov > bv || (ov == bv && oq < bq)) {
        bv = ov;
        bq = oq;
      }
    }
    if (bq == INT64_MAX) break;
    taken[r] = bq;
    cand[r] = best[indices[bq]];
  }
  double bs = -INFINITY;
  int bj = 0x7FFFFFFF;
  for (int r = 0; r < 3; ++r) {
    const int j = cand[r];
    if (j < 0 || (r > 0 && j == cand[0]) || (r > 1 && j == cand[1])) continue;
    double t = 0.0;
    for (int64_t q = b + lane; q < e; q += kWave)
      t = fma((double)values[q], master[(int64_t)j * D + indices[q]], t);
    t = wave_sum_d(t);
    if (better_d(t, j, bs, bj)) {
      bs = t;
      bj = j;
    }
  }
  if (lane == 0) probe[row] = bj == 0x7FFFFFFF ? 0 : bj;
}

// Rows whose previous centroid changed, in ascending order (index path).
// Stable compaction of the rows whose previous centroid is flagged in
// `changed` (keep = 0) or not flagged (keep = 1), all rows when changed ==
// nullptr, into an ascending list, in
// three launches: per-block counts, a scan of the block counts, and the
// writes (ballot ranks within a wave, wave counts through LDS).
constexpr int64_t kListBlock = 4096;   // rows per block

__device__ inline bool list_sel(const int32_t *a_prev, const uint8_t *changed, const uint8_t *mode,
                                int64_t i, int32_t keep) {
  return (!changed || (changed[a_prev[i]] != 0) != (keep != 0)) && (!mode || mode[i] != 2);
}

__global__ __launch_bounds__(256) void k_list_count(const int32_t *a_prev, const uint8_t *changed,
                                                    const uint8_t *mode, int32_t keep, int64_t n,
                                                    int32_t *bcnt) {
  __shared__ int32_t ws[4];
  const int64_t lo = (int64_t)blockIdx.x * kListBlock, hi = min(n, lo + kListBlock);
  int c = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256)
    c += list_sel(a_prev, changed, mode, i, keep) ? 1 : 0;
  for (int m = 1; m < kWave; m <<= 1) c += __shfl_xor(c, m, kWave);
  if (lane_id() == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) bcnt[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive scan of the block counts in place; the total into *count.
__global__ __launch_bounds__(1024) void k_list_scan(int32_t *bcnt, int64_t nblk, int32_t *count) {
  __shared__ int32_t wsum[16];
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  int32_t carry = 0;
  for (int64_t i0 = 0; i0 < nblk; i0 += 1024) {
    const int64_t i = i0 + t;
    const int32_t v = i < nblk ? bcnt[i] : 0;
    int32_t incl = v;
    for (int m = 1; m < kWave; m <<= 1) {
      const int32_t y = __shfl_up(incl, m, kWave);
      if (lane >= m) incl += y;
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    int32_t before = 0, step = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wave) before += wsum[w];
      step += wsum[w];
    }
    if (i < nblk) bcnt[i] = carry + before + incl - v;
    carry += step;
    __syncthreads();
  }
  if (t == 0) *count = carry;
}

__global__ __launch_bounds__(256) void k_list_write(const int32_t *a_prev, const uint8_t *changed,
                                                    const uint8_t *mode, int32_t keep, int64_t n,
                                                    const int32_t *boff, int32_t *rows) {
  __shared__ int32_t ws[4];
  const int64_t lo = (int64_t)blockIdx.x * kListBlock, hi = min(n, lo + kListBlock);
  const int wave = threadIdx.x >> 6;
  int32_t pos = boff[blockIdx.x];
  for (int64_t b0 = lo; b0 < hi; b0 += 256) {
    const int64_t i = b0 + threadIdx.x;
    const bool sel = i < hi && list_sel(a_prev, changed, mode, i, keep);
    const uint64_t m = __ballot(sel);
    if (lane_id() == 0) ws[wave] = __popcll(m);
    __syncthreads();
    int32_t before = 0, step = 0;
    for (int w = 0; w < 4; ++w) {
      if (w < wave) before += ws[w];
      step += ws[w];
    }
    if (sel) rows[pos + before + __popcll(m & lanemask_lt())] = (int32_t)i;
    pos += step;
    __syncthreads();
  }
}

}  // namespace

hipError_t index_counts(const double *master, int32_t k, int64_t D, const int32_t *ids,
                        int32_t n, int32_t *cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_centroid_nnz, dim3((unsigned)n), dim3(256), 0, s, master, D, ids, cnt);
  return hipGetLastError();
}

hipError_t index_place(const int32_t *ids, int32_t n, const int32_t *cnt, int64_t base_e,
                       int64_t base_q, int64_t *sstart, int64_t *qstart, int64_t *tot,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_place, dim3(1), dim3(1024), 0, s, ids, (int64_t)n, cnt, base_e, base_q,
                     sstart, qstart, tot);
  return hipGetLastError();
}

int32_t index_run_len() { return kRun; }

hipError_t index_segments(const IndexBuild &ib, const int32_t *ids, int32_t n, const int2 *runs,
                          int64_t n_runs, const int2 *tiles, int64_t n_tiles, int64_t max_len,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_extract, dim3((unsigned)n), dim3(256), 0, s, ib.master, ib.D, ids, ib.sstart,
                     ib.key0, ib.term0);
  if (n_runs > 0)
    hipLaunchKernelGGL(k_sort_runs, dim3((unsigned)n_runs), dim3(256), 0, s, runs, ib.sstart, ib.cnt,
                       ib.key0, ib.term0);
  bool in1 = false;   // the sorted entries are in (key1, term1)
  if (n_tiles > 0) {
    for (int64_t w = kRun; w < max_len; w *= 2) {
      hipLaunchKernelGGL(k_merge_pass, dim3((unsigned)n_tiles), dim3(256), 0, s, tiles, ib.sstart,
                         ib.cnt, w, in1 ? ib.key1 : ib.key0, in1 ? ib.term1 : ib.term0,
                         in1 ? ib.key0 : ib.key1, in1 ? ib.term0 : ib.term1);
      in1 = !in1;
    }
    if (in1)
      hipLaunchKernelGGL(k_copy_tiles, dim3((unsigned)n_tiles), dim3(256), 0, s, tiles, ib.sstart,
                         ib.cnt, ib.key1, ib.term1, ib.key0, ib.term0);
  }
  hipLaunchKernelGGL(k_prefix_sq, dim3((unsigned)n), dim3(256), 0, s, ids, ib.sstart, ib.cnt,
                     ib.qstart, ib.key0, ib.Q);
  return hipGetLastError();
}

hipError_t index_terms(const IndexBuild &ib, hipStream_t s) {
  const int32_t k = ib.k;
  const int64_t D = ib.D, nb = (k + 63) / 64;
  hipLaunchKernelGGL(k_term_masks, dim3((unsigned)nb, (unsigned)((D + 63) / 64)), dim3(256), 0, s,
                     ib.master, (const int32_t *)nullptr, k, D, nb, ib.mask);
  hipLaunchKernelGGL(k_term_prefix, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, ib.mask, D,
                     nb, ib.blkpre, ib.tcnt);
  hipLaunchKernelGGL(k_scan_i32_to_i64, dim3(1), dim3(1024), 0, s, ib.tcnt, D, ib.toff);
  hipLaunchKernelGGL(k_fill_G, dim3((unsigned)k), dim3(256), 0, s, (const int32_t *)nullptr,
                     ib.sstart, ib.cnt, ib.term0, ib.mask, ib.blkpre, ib.toff, nb, ib.G);
  return hipGetLastError();
}

// G2 over the dirty centroids ids[0 .. n) (ascending), built like G over that
// list (the full build's masks and block prefixes are free again once G is
// filled, and hold ceil(k / 64) >= ceil(n / 64) blocks per term): each term's
// entries ascending by centroid, without atomics.
hipError_t index_delta(const IndexBuild &ib, const int32_t *dirty_ids, int32_t n_dirty,
                       const uint8_t *dirty, int64_t *toff2, uint2 *G2, uint32_t *dbits,
                       hipStream_t s) {
  const int64_t D = ib.D, nb2 = (n_dirty + 63) / 64;
  if (n_dirty > 0) {
    hipLaunchKernelGGL(k_term_masks, dim3((unsigned)nb2, (unsigned)((D + 63) / 64)), dim3(256), 0,
                       s, ib.master, dirty_ids, n_dirty, D, nb2, ib.mask);
    hipLaunchKernelGGL(k_term_prefix, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, ib.mask,
                       D, nb2, ib.blkpre, ib.tcnt);
    hipLaunchKernelGGL(k_scan_i32_to_i64, dim3(1), dim3(1024), 0, s, ib.tcnt, D, toff2);
    hipLaunchKernelGGL(k_fill_G, dim3((unsigned)n_dirty), dim3(256), 0, s, dirty_ids, ib.sstart,
                       ib.cnt, ib.term0, ib.mask, ib.blkpre, toff2, nb2, G2);
  }
  hipLaunchKernelGGL(k_dirty_bits, dim3((unsigned)((ib.k + 32 * 256 - 1) / (32 * 256))), dim3(256),
                     0, s, dirty, ib.k, dbits);
  return hipGetLastError();
}

int64_t index_rows_work(int64_t n) { return std::max<int64_t>(1, (n + kListBlock - 1) / kListBlock); }

hipError_t index_rows(const int32_t *a_prev, const uint8_t *changed, int64_t n, int32_t *rows,
                      int32_t *count, int32_t *work, hipStream_t s, int32_t keep,
                      const uint8_t *mode) {
  const int64_t nblk = (n + kListBlock - 1) / kListBlock;
  if (nblk > 0) {
    hipLaunchKernelGGL(k_list_count, dim3((unsigned)nblk), dim3(256), 0, s, a_prev, changed, mode,
                       keep, n, work);
  }
  hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, s, work, nblk, count);
  if (nblk > 0) {
    hipLaunchKernelGGL(k_list_write, dim3((unsigned)nblk), dim3(256), 0, s, a_prev, changed, mode,
                       keep, n, work, rows);
  }
  return hipGetLastError();
}

hipError_t index_query(const IndexArgs &x, int64_t n_slots, hipStream_t s) {
  if (n_slots <= 0) return hipSuccess;
  const size_t lds = index_lds_bytes(x.k);
  hipLaunchKernelGGL(k_index_query, dim3((unsigned)n_slots), dim3(256), lds, s, x);
  return hipGetLastError();
}

hipError_t index_best_centroid(const IndexArgs &x, const uint8_t *dirty, const int64_t *sstart,
                               const uint64_t *key, int32_t *best, hipStream_t s) {
  hipLaunchKernelGGL(k_best_centroid, dim3((unsigned)((x.D + 3) / 4)), dim3(256), 0, s, x.toff, x.G,
                     x.toff2, x.G2, dirty, x.n_dirty, sstart, key, x.D, best);
  return hipGetLastError();
}

hipError_t index_probe(const int64_t *indptr, const int32_t *indices, const float *values,
                       int64_t n, const int32_t *best, const double *master, int64_t D,
                       int32_t *probe, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, indptr, indices,
                     values, n, best, master, D, probe);
  return hipGetLastError();
}

hipError_t index_score(const IndexArgs &x, int64_t n_slots, int32_t *a_out, double *lo_out,
                       double *hi_out, hipStream_t s) {
  if (n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_index_score, dim3((unsigned)((n_slots + 3) / 4)), dim3(256), 0, s, x, n_slots,
                     a_out, lo_out, hi_out);
  return hipGetLastError();
}

}  // namespace skm
