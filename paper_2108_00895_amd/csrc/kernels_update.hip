// Update-side kernels (paper Sec. 2: a centroid is its members' sum divided by
// the sum's length) and the small helpers around them.
//
// The centroid update is atomic-free in its floating point: rows are bucketed
// by cluster with a stable counting sort (integer atomics only for counts), and
// one workgroup owns one cluster's FP64 sum, adding member rows in ascending
// row order.  Unchanged membership therefore reproduces a centroid bit for bit,
// which is what lets Sec. 3.1 skip unchanged centroids exactly.
#include "internal.h"

namespace skm {
namespace {


__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// The update streams dense FP64 rows through once: their loads and stores are
// non-temporal so that they do not evict the lines the scatter-adds reuse.
typedef double v2d __attribute__((ext_vector_type(2)));
unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Block-wide fixed-shape sum over 256 threads (deterministic order).
__device__ inline double block_sum_256(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void k_row_stats(const int64_t *indptr, const int32_t *indices, const float *values,
                            int64_t n_rows, int64_t D, double *xl1, double *xl2, int32_t *bad) {
  const int lane = lane_id();
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n_rows) return;
  const int64_t b = indptr[row], e = indptr[row + 1];
  int flags = 0;
  if (e < b) flags |= 1;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t q = b + lane; q < e; q += kWave) {
    const float v = values[q];
    const int32_t t = indices[q];
    if (!(v > 0.f) || !isfinite(v)) flags |= 2;
    if (t < 0 || t >= D) flags |= 4;
    if (q > b && indices[q - 1] >= t) flags |= 8;
    s1 += (double)v;
    s2 += (double)v * (double)v;
  }
  s1 = wave_sum_d(s1);
  s2 = wave_sum_d(s2);
  for (int m = 1; m < kWave; m <<= 1) flags |= __shfl_xor(flags, m, kWave);
  if (lane == 0) {
    xl1[row] = s1;
    xl2[row] = sqrt(s2);
    if (e > b && fabs(sqrt(s2) - 1.0) > 1e-5) flags |= 16;
    if (e == b) flags |= 32;
    if (flags) atomicOr(bad, flags);
  }
}

// L1 norm per row only (rows already checked on the host).
__global__ void k_row_l1(const int64_t *indptr, const float *values, int64_t n_rows,
                         const int64_t *n_dev, double *xl1) {
  const int lane = lane_id();
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (n_dev ? *n_dev : n_rows)) return;
  double s1 = 0.0;
  for (int64_t q = indptr[row] + lane; q < indptr[row + 1]; q += kWave) s1 += (double)values[q];
  s1 = wave_sum_d(s1);
  if (lane == 0) xl1[row] = s1;
}

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// c_j = x_r / ||x_r|| for r = rows[j]; the master rows are zero beforehand.
__global__ void k_seed(const int64_t *indptr, const int32_t *indices, const float *values,
                       const int32_t *rows, int64_t D, double *master) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  const int64_t r = rows[j];
  const int64_t b = indptr[r], e = indptr[r + 1];
  double ss = 0.0;
  for (int64_t q = b + threadIdx.x; q < e; q += 256) ss += (double)values[q] * (double)values[q];
  const double nrm = sqrt(block_sum_256(ss, sh));
  for (int64_t q = b + threadIdx.x; q < e; q += 256)
    master[(int64_t)j * D + indices[q]] = (double)values[q] / nrm;
}

__global__ void k_fp8_scales(const double *master, int64_t D, const uint8_t *changed, float *scale) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  if (changed && !changed[j]) return;
  double m = 0.0;
  for (int64_t t = threadIdx.x; t < D; t += 256) m = fmax(m, master[(int64_t)j * D + t]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[j] = ldexpf(1.0f, e4m3_scale_exp(sh[0]));
}

// Scoring copy: 64 centroids x 128 terms of the FP64 master per workgroup,
// encoded on load (16-byte loads along each centroid row) and transposed
// through LDS as codes, then written term-major (64 consecutive codes per
// term row).  Workgroups whose 64 centroids are all unchanged exit at once.
template <int P>
struct CodeOf {
  using T = uint32_t;
};
template <>
struct CodeOf<SKM_BF16> {
  using T = uint16_t;
};
template <>
struct CodeOf<SKM_FP8_E4M3> {
  using T = uint8_t;
};

constexpr int kQT = 128;   // terms per quantize tile

template <int P>
__device__ inline typename CodeOf<P>::T encode_code(double c, int e) {
  if (P == SKM_FP32) {
    const float f = (float)c;
    return __float_as_uint(f);
  } else if (P == SKM_BF16) {
    return encode_bf16(c);
  } else {
    return encode_e4m3(ldexp(c, -e));
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_quantize(const double *master, int32_t k, int64_t D,
                                                  const uint8_t *changed, const float *scale,
                                                  uint8_t *tile) {
  using T = typename CodeOf<P>::T;
  constexpr int pitch = kQT + 4 / (int)sizeof(T);   // one 32-bit word of padding per row
  __shared__ T buf[64][pitch];
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int64_t t0 = (int64_t)blockIdx.y * kQT;
  const int tid = threadIdx.x;
  int any = 0;
  if (tid < 64) {
    const int64_t j = j0 + tid;
    any = (j < k) && (changed == nullptr || changed[j]);
  }
  if (!__syncthreads_or(any)) return;
  const bool vec = (D % 2 == 0) && (t0 + kQT <= D);
  // 64 rows x 64 term pairs
#pragma unroll 4
  for (int p = 0; p < 16; ++p) {
    const int idx = p * 256 + tid;
    const int jj = idx >> 6, q = idx & 63;
    const int64_t j = j0 + jj, t = t0 + 2 * q;
    double c0 = 0.0, c1 = 0.0;
    if (j < k) {
      const double *row = master + j * D;
      if (vec) {
        const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(row + t));
        c0 = v.x;
        c1 = v.y;
      } else {
        if (t < D) c0 = row[t];
        if (t + 1 < D) c1 = row[t + 1];
      }
    }
    const int e = (P == SKM_FP8_E4M3 && j < k) ? ilogbf(scale[j]) : 0;
    buf[jj][2 * q] = encode_code<P>(c0, e);
    buf[jj][2 * q + 1] = encode_code<P>(c1, e);
  }
  __syncthreads();
  // term rows: 64 codes each, 8 per thread
  const int64_t ncols = min<int64_t>(64, (int64_t)k - j0);
  for (int p = 0; p < kQT / 32; ++p) {
    const int tt = p * 32 + (tid >> 3);
    const int g = (tid & 7) * 8;
    const int64_t t = t0 + tt;
    if (t >= D) continue;
    T* dst = reinterpret_cast<T *>(tile) + tile_index(t, j0 + g, D);
    if (g + 8 <= ncols) {
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = buf[g + q][tt];
      if (sizeof(T) == 2) {
        uint4 w;
        w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        w.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
        w.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
        w.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
        *reinterpret_cast<uint4 *>(dst) = w;
      } else if (sizeof(T) == 1) {
        uint2 w;
        w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
        w.y = (uint32_t)v[4] | ((uint32_t)v[5] << 8) | ((uint32_t)v[6] << 16) | ((uint32_t)v[7] << 24);
        *reinterpret_cast<uint2 *>(dst) = w;
      } else {
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
        d4[0] = make_uint4(v[0], v[1], v[2], v[3]);
        d4[1] = make_uint4(v[4], v[5], v[6], v[7]);
      }
    } else {
      for (int q = 0; q < 8 && g + q < ncols; ++q) dst[q] = buf[g + q][tt];
    }
  }
}

__global__ void k_count_moved(const int32_t *a, const int32_t *a_prev, int64_t n,
                              unsigned long long *out) {
  int64_t c = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) c += (a[i] != a_prev[i]);
  c = wave_sum_i64(c);
  if (lane_id() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

__global__ void k_mark_changed(const int32_t *a, const int32_t *a_prev, int64_t n, uint8_t *changed) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int32_t x = a[i], y = a_prev[i];
    if (x != y) {
      changed[x] = 1;
      changed[y] = 1;
    }
  }
}

// Ascending list of changed ids: one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_compact_changed(const uint8_t *changed, int32_t k,
                                                          int32_t *ids, int32_t *count) {
  __shared__ int32_t sh[1024];
  const int t = threadIdx.x;
  const int per = (k + 1023) / 1024;
  const int lo = t * per, hi = min(k, lo + per);
  int c = 0;
  for (int j = lo; j < hi; ++j) c += changed[j] ? 1 : 0;
  sh[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // Hillis-Steele inclusive scan
    int v = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int pos = sh[t] - c;
  for (int j = lo; j < hi; ++j)
    if (changed[j]) ids[pos++] = j;
  if (t == 1023) *count = sh[1023];
}

template <typename T>
__global__ void k_gather_tile(const T *tile, int64_t D, const int32_t *ids, int32_t n, T *out) {
  const int64_t t = blockIdx.x;
  for (int o = threadIdx.x; o < n; o += blockDim.x)
    out[tile_index(t, o, D)] = tile[tile_index(t, ids[o], D)];
}

// out[j * n + q] = master[j][terms[q]] (one workgroup per centroid).
__global__ __launch_bounds__(256) void k_centroid_columns(const double *master, int64_t D,
                                                          const int32_t *terms, int32_t n,
                                                          double *out) {
  const int64_t j = blockIdx.x;
  for (int q = threadIdx.x; q < n; q += blockDim.x) out[j * n + q] = master[j * D + terms[q]];
}

// ---- stable counting sort of rows by cluster

__global__ void k_block_hist(const int32_t *a, int64_t n, int32_t k, int64_t blk, int32_t *hist) {
  const int64_t b = blockIdx.x;
  const int64_t lo = b * blk, hi = min(n, lo + blk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&hist[b * k + a[i]], 1);
}

// For each cluster: exclusive prefix over blocks in place, total into counts.
__global__ void k_block_scan(int32_t *hist, int64_t nblk, int32_t k, int32_t *counts) {
  const int64_t j = gtid();
  if (j >= k) return;
  int32_t run = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    const int32_t v = hist[b * k + j];
    hist[b * k + j] = run;
    run += v;
  }
  counts[j] = run;
}

__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t *counts, int32_t k,
                                                      int64_t *offsets) {
  __shared__ int64_t sh[1024];
  const int t = threadIdx.x;
  const int per = (k + 1023) / 1024;
  const int lo = t * per, hi = min(k, lo + per);
  int64_t c = 0;
  for (int j = lo; j < hi; ++j) c += counts[j];
  sh[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int64_t pos = sh[t] - c;
  for (int j = lo; j < hi; ++j) {
    offsets[j] = pos;
    pos += counts[j];
  }
  if (t == 1023) offsets[k] = sh[1023];
}

// One wavefront per block of rows, in row order: rank among equal clusters in
// the 64-row batch by ballots, running per-(block, cluster) counter by atomics
// that only this wavefront touches.
__global__ __launch_bounds__(64) void k_block_scatter(const int32_t *a, int64_t n, int32_t k,
                                                      int64_t blk, int32_t *hist,
                                                      const int64_t *offsets, int32_t *members) {
  const int64_t b = blockIdx.x;
  const int64_t lo = b * blk, hi = min(n, lo + blk);
  const int lane = lane_id();
  for (int64_t base = lo; base < hi; base += kWave) {
    const int64_t i = base + lane;
    const bool valid = i < hi;
    const int32_t cl = valid ? a[i] : -1;
    uint64_t remaining = __ballot(valid);
    uint64_t peers = 0;
    while (remaining) {
      const int leader = __ffsll((unsigned long long)remaining) - 1;
      const int32_t lc = __shfl(cl, leader, kWave);
      const uint64_t m = __ballot(valid && cl == lc);
      if (valid && cl == lc) peers = m;
      remaining &= ~m;
    }
    const int leader = valid ? __ffsll((unsigned long long)peers) - 1 : 0;
    int32_t old = 0;
    if (valid && leader == lane) old = atomicAdd(&hist[b * k + cl], __popcll(peers));
    old = __shfl(old, leader, kWave);
    if (valid) {
      const int rank = __popcll(peers & lanemask_lt());
      members[offsets[cl] + old + rank] = (int32_t)i;
    }
  }
}

// A sum task's destination row: workspace rows are cleared; sum rows S_j are
// all zero already (zeroed at set-up and by the renormalisation that read
// them).  For a task summing straight into S_j the support bitmap of S_j (bit
// t: S_j[t] != 0) is cleared here and set as terms are first added.
__device__ inline void prepare_dst(double *dst, int64_t D, uint32_t *bits, const SumSupport &sp,
                                   const int4 &tk) {
  const int tid = threadIdx.x;
  if (tk.z >= 0) {
    if (D % 2 == 0) {
      v2d *d2 = reinterpret_cast<v2d *>(dst);
      const v2d z = {0.0, 0.0};
      for (int64_t t = tid; t < D / 2; t += 256) __builtin_nontemporal_store(z, d2 + t);
    } else {
      for (int64_t t = tid; t < D; t += 256) dst[t] = 0.0;
    }
  }
  if (bits)
    for (int64_t w = tid; w < sp.W; w += 256) bits[w] = 0u;
}

// dst[t] += v; the first add to an entry (values are positive, so the entry
// was 0.0) sets its support bit.
__device__ inline void add_tracked(double *dst, uint32_t *bits, int32_t t, double v) {
  const double old = dst[t];
  dst[t] = old + v;
  if (bits && old == 0.0) atomicOr(&bits[t >> 5], 1u << (t & 31));
}

__device__ inline void store_tracked(double *dst, uint32_t *bits, int32_t t, double v) {
  dst[t] = v;
  if (bits && v != 0.0) atomicOr(&bits[t >> 5], 1u << (t & 31));
}

// Segmented member sums: task = (cluster, member range [r0, r1), destination).
// A cluster with more members than one segment is split into fixed segments
// whose sums go to partial rows of a workspace (dest >= 0) and are added in
// segment order by k_combine; small clusters sum straight into S_j (dest < 0).
// One workgroup per task adds its member rows in ascending row order (member
// lists are sorted): the entries of one row have distinct terms and rows are
// separated by barriers, so every sum runs in a fixed order without atomics
// and results are reproducible.  The most frequent terms (hot_slot[t] >= 0)
// are summed in LDS and written once at the end; the others go to the FP64
// destination row directly.
__global__ __launch_bounds__(256) void k_sum_tasks(const int64_t *indptr, const int32_t *indices,
                                                   const float *values, const int32_t *members,
                                                   const int4 *tasks, const int64_t *task_r0,
                                                   int64_t D, double *S, double *work,
                                                   const int32_t *hot_slot,
                                                   const int32_t *hot_terms, int32_t n_hot,
                                                   SumSupport sp) {
  __shared__ double hot[kSumHot];
  const int4 tk = tasks[blockIdx.x];   // x = cluster, y = count, z = dest slot (-1: S_j)
  double *dst = tk.z < 0 ? S + (int64_t)tk.x * D : work + (int64_t)tk.z * D;
  uint32_t *bits = (sp.nb && tk.z < 0) ? sp.nb + (int64_t)tk.x * sp.W : nullptr;
  const int tid = threadIdx.x;
  prepare_dst(dst, D, bits, sp, tk);
  for (int h = tid; h < n_hot; h += 256) hot[h] = 0.0;
  // Member row ranges are staged in LDS 256 rows at a time, and each thread's
  // first entry of the next row is loaded before the current row's adds, so
  // those loads overlap the adds and the barrier.
  __shared__ int64_t rb[256], re[256];
  const int64_t r0 = task_r0[blockIdx.x], r1 = r0 + tk.y;
  for (int64_t g0 = r0; g0 < r1; g0 += 256) {
    const int nr = (int)min<int64_t>(256, r1 - g0);
    __syncthreads();   // the zeroing, or the previous group's rows, are done
    if (tid < nr) {
      const int64_t i = members[g0 + tid];
      rb[tid] = indptr[i];
      re[tid] = indptr[i + 1];
    }
    __syncthreads();
    int32_t t1 = 0, h1 = -1;
    double v1 = 0.0;
    bool has1 = rb[0] + tid < re[0];
    if (has1) {
      t1 = indices[rb[0] + tid];
      v1 = (double)values[rb[0] + tid];
      h1 = hot_slot ? hot_slot[t1] : -1;
    }
    for (int q = 0; q < nr; ++q) {
      const int64_t b = rb[q], e = re[q];
      const int32_t t0 = t1, h0 = h1;
      const double v0 = v1;
      const bool has0 = has1;
      has1 = q + 1 < nr && rb[q + 1] + tid < re[q + 1];
      if (has1) {
        t1 = indices[rb[q + 1] + tid];
        v1 = (double)values[rb[q + 1] + tid];
        h1 = hot_slot ? hot_slot[t1] : -1;
      }
      if (has0) {
        if (h0 >= 0) {
          hot[h0] += v0;
        } else {
          add_tracked(dst, bits, t0, v0);
        }
      }
      for (int64_t p = b + 256 + tid; p < e; p += 256) {   // rows longer than 256 entries
        const int32_t t = indices[p];
        const double v = (double)values[p];
        const int32_t h = hot_slot ? hot_slot[t] : -1;
        if (h >= 0) {
          hot[h] += v;
        } else {
          add_tracked(dst, bits, t, v);
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int h = tid; h < n_hot; h += 256) store_tracked(dst, bits, hot_terms[h], hot[h]);
}

// The same sums for corpora of short rows (a few dozen terms or fewer).  A
// step takes as many consecutive member rows as fit in 256 entries, one entry
// per thread; the step's (term, row) keys are sorted in LDS (bitonic) so that
// each term's values form one run in row order, the run's head adds them in
// that order and adds the run's sum to the term's accumulator once.  Terms
// are distinct across runs, so the adds of a step are race-free, and steps
// follow the member order: the sum is a fixed function of the member list.
// Rows of more than 256 entries take a step of their own (their terms are
// distinct).  Requires D < 2^24 (keys pack the term above an 8-bit row index).
__global__ __launch_bounds__(256) void k_sum_tasks_short(const int64_t *indptr,
                                                         const int32_t *indices,
                                                         const float *values,
                                                         const int32_t *members,
                                                         const int4 *tasks, const int64_t *task_r0,
                                                         int64_t D, double *S, double *work,
                                                         const int32_t *hot_slot,
                                                         const int32_t *hot_terms, int32_t n_hot,
                                                         SumSupport sp) {
  __shared__ double hot[kSumHot];
  __shared__ int64_t rb[256];
  __shared__ int32_t plen[257];          // inclusive prefix of the group's row lengths
  __shared__ uint32_t key[256];
  __shared__ double val[256];
  const int4 tk = tasks[blockIdx.x];   // x = cluster, y = count, z = dest slot (-1: S_j)
  double *dst = tk.z < 0 ? S + (int64_t)tk.x * D : work + (int64_t)tk.z * D;
  uint32_t *bits = (sp.nb && tk.z < 0) ? sp.nb + (int64_t)tk.x * sp.W : nullptr;
  const int tid = threadIdx.x;
  prepare_dst(dst, D, bits, sp, tk);
  for (int h = tid; h < n_hot; h += 256) hot[h] = 0.0;
  auto add = [&](int32_t t, double v) {
    const int32_t h = hot_slot ? hot_slot[t] : -1;
    if (h >= 0) {
      hot[h] += v;
    } else {
      add_tracked(dst, bits, t, v);
    }
  };
  const int64_t r0 = task_r0[blockIdx.x], r1 = r0 + tk.y;
  for (int64_t g0 = r0; g0 < r1; g0 += 256) {
    const int nr = (int)min<int64_t>(256, r1 - g0);
    __syncthreads();   // the zeroing, or the previous group's steps, are done
    int32_t len = 0;
    if (tid < nr) {
      const int64_t i = members[g0 + tid];
      rb[tid] = indptr[i];
      len = (int32_t)(indptr[i + 1] - rb[tid]);
    }
    // inclusive scan of the lengths (capped: a long row is a step of its own)
    plen[tid + 1] = len;
    if (tid == 0) plen[0] = 0;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int32_t v = tid + 1 > off ? plen[tid + 1 - off] : 0;
      __syncthreads();
      plen[tid + 1] += v;
      __syncthreads();
    }
    int q0 = 0;
    while (q0 < nr) {
      // rows q0 .. q1 - 1: as many as fit in 256 entries (at least one)
      int q1 = q0 + 1;
      while (q1 < nr && plen[q1 + 1] - plen[q0] <= 256) ++q1;
      const int32_t n_ent = plen[q1] - plen[q0];
      if (q1 - q0 == 1) {
        // one row: its terms are distinct, every thread adds its entries
        for (int32_t e = tid; e < n_ent; e += 256)
          add(indices[rb[q0] + e], (double)values[rb[q0] + e]);
      } else {
        // several rows: sort the step's entries by (term, row)
        uint32_t kk = 0xFFFFFFFFu;
        double vv = 0.0;
        if (tid < n_ent) {
          int q = q0;   // the row holding entry tid of the step
          while (plen[q + 1] - plen[q0] <= tid) ++q;
          const int64_t p = rb[q] + (tid - (plen[q] - plen[q0]));
          kk = ((uint32_t)indices[p] << 8) | (uint32_t)(q - q0);
          vv = (double)values[p];
        }
        key[tid] = kk;
        val[tid] = vv;
        __syncthreads();
        for (int size = 2; size <= 256; size <<= 1) {
          for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int partner = tid ^ stride;
            if (partner > tid) {
              const bool up = (tid & size) == 0;
              const uint32_t a = key[tid], b = key[partner];
              if ((a > b) == up) {
                key[tid] = b;
                key[partner] = a;
                const double x = val[tid];
                val[tid] = val[partner];
                val[partner] = x;
              }
            }
            __syncthreads();
          }
        }
        if (tid < n_ent && (tid == 0 || (key[tid] >> 8) != (key[tid - 1] >> 8))) {
          const uint32_t term = key[tid] >> 8;
          double run = val[tid];
          for (int e = tid + 1; e < n_ent && (key[e] >> 8) == term; ++e) run += val[e];
          add((int32_t)term, run);
        }
      }
      __syncthreads();
      q0 = q1;
    }
  }
  __syncthreads();
  for (int h = tid; h < n_hot; h += 256) store_tracked(dst, bits, hot_terms[h], hot[h]);
}

// S_j = sum of its segment partials, in segment order, and its support bits
// (a wavefront's 64 consecutive terms by ballot).  Block (group, term block).
__global__ __launch_bounds__(256) void k_combine(const int4 *groups, int64_t D, int64_t tblk,
                                                 const double *work, double *S, uint32_t *nb,
                                                 int64_t W) {
  const int4 g = groups[blockIdx.x / tblk];   // x = cluster, y = first slot, z = segments
  const int64_t t0 = (blockIdx.x % tblk) * 4096;
  for (int64_t tw = t0 + (threadIdx.x & ~63); tw < min(D, t0 + 4096); tw += 256) {
    const int64_t t = tw + lane_id();
    double s = 0.0;
    if (t < D) {
      const double *w = work + (int64_t)g.y * D + t;
      int p = 0;
      for (; p + 4 <= g.z; p += 4) {   // four loads in flight, added in segment order
        const double w0 = __builtin_nontemporal_load(w + (int64_t)p * D);
        const double w1 = __builtin_nontemporal_load(w + (int64_t)(p + 1) * D);
        const double w2 = __builtin_nontemporal_load(w + (int64_t)(p + 2) * D);
        const double w3 = __builtin_nontemporal_load(w + (int64_t)(p + 3) * D);
        s += w0;
        s += w1;
        s += w2;
        s += w3;
      }
      for (; p < g.z; ++p) s += __builtin_nontemporal_load(w + (int64_t)p * D);
      __builtin_nontemporal_store(s, S + (int64_t)g.x * D + t);
    }
    if (nb) {
      const uint64_t m = __ballot(s != 0.0);
      if (lane_id() == 0) {
        nb[(int64_t)g.x * W + (tw >> 5)] = (uint32_t)m;
        if ((tw >> 5) + 1 < W) nb[(int64_t)g.x * W + (tw >> 5) + 1] = (uint32_t)(m >> 32);
      }
    }
  }
}

__device__ inline double block_max_256(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] = fmax(sh[t], sh[t + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// c_j = S_j / ||S_j|| (empty clusters keep c_j), with the per-cluster shift
// ||c_j(new) - c_j(old)||^2 and S_j . c_j(old); S_j is left all zero for its
// next sums.  One workgroup per cluster.  The norm is summed over S_j's
// non-zeros as its support bitmap lists them (thread tid takes words tid, tid
// + 256, ..., the set bits of a word ascending, eight loads in flight), so it
// does not depend on which of the two paths below writes the row:
//   - sparse (the master row's support is known and S_j holds fewer than
//     D / 2 non-zeros): only the union of both supports is visited; the new
//     master entries, the shift, S_j . c_j(old) and the scoring codes (FP8:
//     the scale from S_j's largest entry) are written there;
//   - dense: the rows are streamed (a wavefront per 64 consecutive terms),
//     the master's support bitmap built by ballots, and k_quantize encodes
//     the row (qmask).
template <int P>
__global__ __launch_bounds__(256) void k_renorm(double *S, const int32_t *counts,
                                                const int32_t *ids, int64_t D, double *master,
                                                double *snorm, double *shift, double *dot_old,
                                                RenormSupport rs) {
  __shared__ double sh[256];
  const int32_t j = ids[blockIdx.x];
  double *Sj = S + (int64_t)j * D;
  double *Mj = master + (int64_t)j * D;
  const int tid = threadIdx.x;
  if (counts[j] == 0) {
    if (tid == 0) {
      snorm[j] = 0.0;
      shift[j] = 0.0;
      dot_old[j] = 0.0;
      rs.qmask[j] = 0;   // c_j is kept, so are its codes
    }
    return;
  }
  const uint32_t *nbj = rs.nb + (int64_t)j * rs.W;
  double ss = 0.0, smax = 0.0;
  int64_t cnt = 0;
  for (int64_t w = tid; w < rs.W; w += 256) {
    uint32_t m = nbj[w];
    cnt += __popc(m);
    while (m) {
      int64_t t[8];
      int nt = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        t[u] = m ? w * 32 + __builtin_ctz(m) : -1;
        nt += m ? 1 : 0;
        m &= m ? m - 1 : 0u;
      }
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = u < nt ? Sj[t[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < nt) {
          ss += v[u] * v[u];
          smax = fmax(smax, v[u]);
        }
    }
  }
  const double nrm = sqrt(block_sum_256(ss, sh));
  const double total = block_sum_256((double)cnt, sh);
  const bool sparse = rs.mvalid[j] && total * 2.0 < (double)D;
  if (sparse) {
    uint32_t *mbj = rs.mb + (int64_t)j * rs.W;
    int e = 0;
    if (P == SKM_FP8_E4M3) {
      // the new row's largest value is S_j's largest over the norm
      smax = block_max_256(smax, sh);
      e = e4m3_scale_exp(smax / nrm);
      if (tid == 0) rs.scale[j] = ldexpf(1.0f, e);
    }
    using T = typename CodeOf<P>::T;
    T *codes = reinterpret_cast<T *>(rs.tile);
    double sh2 = 0.0, dot = 0.0;
    for (int64_t w = tid; w < rs.W; w += 256) {
      const uint32_t nw = nbj[w];
      uint32_t m = nw | mbj[w];
      while (m) {
        int64_t t[4];
        int nt = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          t[u] = m ? w * 32 + __builtin_ctz(m) : -1;
          nt += m ? 1 : 0;
          m &= m ? m - 1 : 0u;
        }
        double sv[4], o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool in = u < nt && ((nw >> (t[u] & 31)) & 1u);
          sv[u] = in ? Sj[t[u]] : 0.0;
          o[u] = u < nt ? Mj[t[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u >= nt) continue;
          const bool in = (nw >> (t[u] & 31)) & 1u;
          const double c = in ? sv[u] / nrm : 0.0;
          const double d = c - o[u];
          sh2 += d * d;
          dot += sv[u] * o[u];
          Mj[t[u]] = c;
          codes[tile_index(t[u], j, D)] = encode_code<P>(c, e);
          if (in) Sj[t[u]] = 0.0;
        }
      }
      mbj[w] = nw;
    }
    sh2 = block_sum_256(sh2, sh);
    dot = block_sum_256(dot, sh);
    if (tid == 0) {
      snorm[j] = nrm;
      shift[j] = sh2;
      dot_old[j] = dot;
      rs.qmask[j] = 0;
    }
    return;
  }
  double sh2 = 0.0, dot = 0.0;
  uint32_t *mbj = rs.mb + (int64_t)j * rs.W;
  const int lane = lane_id();
  for (int64_t t0 = (int64_t)(tid & ~63); t0 < D; t0 += 256) {
    const int64_t t = t0 + lane;
    double c = 0.0;
    if (t < D) {
      const double sv = __builtin_nontemporal_load(Sj + t);
      const double o = __builtin_nontemporal_load(Mj + t);
      c = sv / nrm;
      const double d = c - o;
      sh2 += d * d;
      dot += sv * o;
      __builtin_nontemporal_store(c, Mj + t);
      if (sv != 0.0) Sj[t] = 0.0;
    }
    const uint64_t m = __ballot(c != 0.0);
    if (lane == 0) {
      mbj[t0 >> 5] = (uint32_t)m;
      if ((t0 >> 5) + 1 < rs.W) mbj[(t0 >> 5) + 1] = (uint32_t)(m >> 32);
    }
  }
  sh2 = block_sum_256(sh2, sh);
  dot = block_sum_256(dot, sh);
  if (tid == 0) {
    snorm[j] = nrm;
    shift[j] = sh2;
    dot_old[j] = dot;
    rs.mvalid[j] = 1;
    rs.qmask[j] = 1;
  }
}

// out[0] = J_A = sum_j S_j . c_j(old), out[1] = J_U = sum_j ||S_j||,
// out[2] = max_j shift_j, all over one workgroup in a fixed order.
__global__ __launch_bounds__(1024) void k_reduce_stats(const uint8_t *changed, const double *snorm,
                                                       const double *shift, const double *dot_old,
                                                       int32_t k, double *out) {
  __shared__ double sa[1024], su[1024], sm[1024];
  const int t = threadIdx.x;
  double ja = 0.0, ju = 0.0, mx = 0.0;
  for (int j = t; j < k; j += 1024) {
    const bool ch = changed[j] != 0;
    ja += ch ? dot_old[j] : snorm[j];
    ju += snorm[j];
    if (ch) mx = fmax(mx, shift[j]);
  }
  sa[t] = ja;
  su[t] = ju;
  sm[t] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) {
      sa[t] += sa[t + w];
      su[t] += su[t + w];
      sm[t] = fmax(sm[t], sm[t + w]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = sa[0];
    out[1] = su[0];
    out[2] = sm[0];
  }
}

}  // namespace

hipError_t launch_row_stats(const int64_t *indptr, const int32_t *indices, const float *values,
                            int64_t n_rows, int64_t D, double *xl1, double *xl2, int32_t *bad,
                            hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_stats, dim3((unsigned)((n_rows + 3) / 4)), dim3(256), 0, s, indptr,
                     indices, values, n_rows, D, xl1, xl2, bad);
  return hipGetLastError();
}

hipError_t launch_row_stats_only(const int64_t *indptr, const int32_t *indices, const float *values,
                                 int64_t n_rows, double *xl1, hipStream_t s, const int64_t *n_dev) {
  (void)indices;
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_l1, dim3((unsigned)((n_rows + 3) / 4)), dim3(256), 0, s, indptr, values,
                     n_rows, n_dev, xl1);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_seed(const int64_t *indptr, const int32_t *indices, const float *values,
                       const int32_t *rows, int32_t k, int64_t D, double *master, hipStream_t s) {
  hipError_t err = launch_fill_f64(master, 0.0, (int64_t)k * D, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_seed, dim3((unsigned)k), dim3(256), 0, s, indptr, indices, values, rows, D,
                     master);
  return hipGetLastError();
}

hipError_t launch_fp8_scales(const double *master, int32_t k, int64_t D, const uint8_t *changed,
                             float *scale, hipStream_t s) {
  hipLaunchKernelGGL(k_fp8_scales, dim3((unsigned)k), dim3(256), 0, s, master, D, changed, scale);
  return hipGetLastError();
}

hipError_t launch_quantize(const double *master, int32_t k, int64_t D, const uint8_t *changed,
                           const float *scale, int prec, uint8_t *tile, hipStream_t s) {
  const dim3 g((unsigned)((k + 63) / 64), (unsigned)((D + kQT - 1) / kQT)), b(256);
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_quantize<SKM_FP32>, g, b, 0, s, master, k, D, changed, scale, tile);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_quantize<SKM_BF16>, g, b, 0, s, master, k, D, changed, scale, tile);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_quantize<SKM_FP8_E4M3>, g, b, 0, s, master, k, D, changed, scale, tile);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_count_moved(const int32_t *a, const int32_t *a_prev, int64_t n,
                              unsigned long long *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_moved, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, a, a_prev, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_mark_changed(const int32_t *a, const int32_t *a_prev, int64_t n, uint8_t *changed,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_changed, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, a, a_prev, n,
                     changed);
  return hipGetLastError();
}

hipError_t launch_compact_changed(const uint8_t *changed, int32_t k, int32_t *ids, int32_t *count,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_compact_changed, dim3(1), dim3(1024), 0, s, changed, k, ids, count);
  return hipGetLastError();
}

hipError_t launch_gather_tile(const uint8_t *tile, int64_t D, int esize, const int32_t *ids,
                              int32_t n, uint8_t *out, hipStream_t s) {
  if (n <= 0 || D <= 0) return hipSuccess;
  const dim3 g((unsigned)D), b(256);
  switch (esize) {
    case 4:
      hipLaunchKernelGGL(k_gather_tile<uint32_t>, g, b, 0, s, (const uint32_t *)tile, D, ids, n,
                         (uint32_t *)out);
      break;
    case 2:
      hipLaunchKernelGGL(k_gather_tile<uint16_t>, g, b, 0, s, (const uint16_t *)tile, D, ids, n,
                         (uint16_t *)out);
      break;
    case 1:
      hipLaunchKernelGGL(k_gather_tile<uint8_t>, g, b, 0, s, tile, D, ids, n, out);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_centroid_columns(const double *master, int32_t k, int64_t D, const int32_t *terms,
                                   int32_t n, double *out, hipStream_t s) {
  if (n <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_centroid_columns, dim3((unsigned)k), dim3(256), 0, s, master, D, terms, n, out);
  return hipGetLastError();
}

hipError_t launch_bucket(const int32_t *a, int64_t n, int32_t k, int64_t blk, int32_t *hist,
                         int32_t *counts, int64_t *offsets, int32_t *members, hipStream_t s) {
  const int64_t nblk = (n + blk - 1) / blk;
  hipError_t err = launch_fill_i32(hist, 0, nblk * k, s);
  if (err != hipSuccess) return err;
  if (n > 0) {
    hipLaunchKernelGGL(k_block_hist, dim3((unsigned)nblk), dim3(256), 0, s, a, n, k, blk, hist);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k_block_scan, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, hist, nblk, k,
                     counts);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, counts, k, offsets);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (n > 0) {
    hipLaunchKernelGGL(k_block_scatter, dim3((unsigned)nblk), dim3(64), 0, s, a, n, k, blk, hist,
                       offsets, members);
    err = hipGetLastError();
  }
  return err;
}

hipError_t launch_sum_tasks(const int64_t *indptr, const int32_t *indices, const float *values,
                            const int32_t *members, const int4 *tasks, const int64_t *task_r0,
                            int32_t n_tasks, int64_t D, double *S, double *work,
                            const int32_t *hot_slot, const int32_t *hot_terms, int32_t n_hot,
                            hipStream_t s, bool short_rows, SumSupport sp) {
  if (n_tasks <= 0) return hipSuccess;
  if (n_hot > kSumHot || (n_hot > 0 && (!hot_slot || !hot_terms))) return hipErrorInvalidValue;
  if (short_rows && D < (int64_t(1) << 24)) {
    hipLaunchKernelGGL(k_sum_tasks_short, dim3((unsigned)n_tasks), dim3(256), 0, s, indptr, indices,
                       values, members, tasks, task_r0, D, S, work,
                       n_hot > 0 ? hot_slot : nullptr, hot_terms, n_hot, sp);
  } else {
    hipLaunchKernelGGL(k_sum_tasks, dim3((unsigned)n_tasks), dim3(256), 0, s, indptr, indices,
                       values, members, tasks, task_r0, D, S, work,
                       n_hot > 0 ? hot_slot : nullptr, hot_terms, n_hot, sp);
  }
  return hipGetLastError();
}

hipError_t launch_combine(const int4 *groups, int32_t n_groups, int64_t D, const double *work,
                          double *S, uint32_t *nb, int64_t W, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  const int64_t tblk = (D + 4095) / 4096;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)(n_groups * tblk)), dim3(256), 0, s, groups, D, tblk,
                     work, S, nb, W);
  return hipGetLastError();
}

hipError_t launch_renorm(double *S, const int32_t *counts, const int32_t *ids, int32_t n_ids,
                         int64_t D, double *master, double *snorm, double *shift, double *dot_old,
                         const RenormSupport &rs, int prec, hipStream_t s) {
  if (n_ids <= 0) return hipSuccess;
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_renorm<SKM_FP32>, dim3((unsigned)n_ids), dim3(256), 0, s, S, counts, ids,
                         D, master, snorm, shift, dot_old, rs);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_renorm<SKM_BF16>, dim3((unsigned)n_ids), dim3(256), 0, s, S, counts, ids,
                         D, master, snorm, shift, dot_old, rs);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_renorm<SKM_FP8_E4M3>, dim3((unsigned)n_ids), dim3(256), 0, s, S, counts,
                         ids, D, master, snorm, shift, dot_old, rs);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_stats(const uint8_t *changed, const double *snorm, const double *shift,
                               const double *dot_old, int32_t k, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(1024), 0, s, changed, snorm, shift, dot_old, k,
                     out);
  return hipGetLastError();
}

}  // namespace skm
