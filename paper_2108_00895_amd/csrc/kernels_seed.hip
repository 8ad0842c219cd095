// k-means++ seeding on the GPU (the initialisation the paper names in Sec. 2;
// D^2 sampling after Arthur and Vassilvitskii, 2007).
//
// For unit rows the squared Euclidean distance to the nearest seed is
// 2 (1 - s), s the highest cosine with a chosen seed, so row i is drawn with
// weight floor(2^32 max(0, 1 - s_i)) (0 once chosen).  Every floating-point
// step is fixed: the cosine with seed r is the row's terms in ascending order
// as one chain of FP64 fused multiply-adds against the seed's values, divided
// by the seed's length (its squared values in the same kind of chain, the
// square root taken on the host); so the integer weights, their sums and the
// draw are exact and independent of the launch shape.  One seed per step:
//   place   - the previous seed's values into a dense FP64 row (the one before
//             it cleared), and its squared length;
//   weights - one lane per row: the cosine, the running maximum, the weight,
//             and per-256-row sums;
//   select  - one workgroup: W = sum of weights, t = draw mod W, the 256-row
//             block and then the row whose cumulative interval holds t (the
//             lowest row not chosen when W = 0).
#include "internal.h"

namespace skm {
namespace {

constexpr int kPPRows = 256;   // rows per weight sum
constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(256) void k_pp_place(const int64_t *__restrict__ indptr,
                                                  const int32_t *__restrict__ indices,
                                                  const float *__restrict__ values, int64_t n,
                                                  const int32_t *__restrict__ rows, int32_t m,
                                                  double *__restrict__ dense,
                                                  double *__restrict__ nrm2) {
  const int tid = threadIdx.x;
  if (m >= 2) {
    const int64_t r0 = rows[m - 2];
    if (r0 >= 0 && r0 < n)
      for (int64_t q = indptr[r0] + tid; q < indptr[r0 + 1]; q += 256) dense[indices[q]] = 0.0;
  }
  __syncthreads();
  const int64_t r = rows[m - 1];
  if (r < 0 || r >= n) {
    if (tid == 0) *nrm2 = -1.0;   // no seed: the host stops
    return;
  }
  const int64_t b = indptr[r], e = indptr[r + 1];
  for (int64_t q = b + tid; q < e; q += 256) dense[indices[q]] = (double)values[q];
  if (tid == 0) {
    double ss = 0.0;
    int64_t q = b;
    for (; q + 8 <= e; q += 8) {   // fixed order, loads issued eight ahead
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = values[q + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) ss = fma((double)x[u], (double)x[u], ss);
    }
    for (; q < e; ++q) {
      const double v = (double)values[q];
      ss = fma(v, v, ss);
    }
    *nrm2 = ss;
  }
}

__global__ __launch_bounds__(kPPRows) void k_pp_weights(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ indices,
    const float *__restrict__ values, int64_t n, const double *__restrict__ dense, double nrm,
    double *__restrict__ best, const uint8_t *__restrict__ chosen, uint64_t *__restrict__ w,
    uint64_t *__restrict__ bsum) {
  __shared__ uint64_t sh[kPPRows];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kPPRows + tid;
  uint64_t wi = 0;
  if (i < n) {
    // the chain's order is fixed; its loads are issued eight terms ahead
    double acc = 0.0;
    int64_t q = indptr[i];
    const int64_t e = indptr[i + 1];
    for (; q + 8 <= e; q += 8) {
      int32_t t[8];
      float x[8];
      double d[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        t[u] = indices[q + u];
        x[u] = values[q + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) d[u] = dense[t[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma((double)x[u], d[u], acc);
    }
    for (; q < e; ++q) acc = fma((double)values[q], dense[indices[q]], acc);
    const double s = acc / nrm;
    const double bi = fmax(best[i], s);
    best[i] = bi;
    const double gap = 1.0 - bi;
    if (!chosen[i]) wi = (uint64_t)floor(ldexp(gap > 0.0 ? gap : 0.0, 32));
    w[i] = wi;
  }
  sh[tid] = wi;
  __syncthreads();
  for (int o = kPPRows / 2; o > 0; o >>= 1) {
    if (tid < o) sh[tid] += sh[tid + o];
    __syncthreads();
  }
  if (tid == 0) bsum[blockIdx.x] = sh[0];
}

// Inclusive prefix sum over the workgroup (kSelThreads values).
__device__ inline uint64_t wg_scan(uint64_t v, uint64_t *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kSelThreads; o <<= 1) {
    const uint64_t x = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  return sh[tid];
}

__global__ __launch_bounds__(kSelThreads) void k_pp_select(const uint64_t *__restrict__ bsum,
                                                           int64_t nb,
                                                           const uint64_t *__restrict__ w,
                                                           int64_t n, uint64_t draw,
                                                           uint8_t *__restrict__ chosen,
                                                           int32_t *__restrict__ rows, int32_t m) {
  __shared__ uint64_t sh[kSelThreads];
  __shared__ int64_t found;
  __shared__ uint64_t found_base;
  const int tid = threadIdx.x;
  uint64_t part = 0;
  for (int64_t b = tid; b < nb; b += kSelThreads) part += bsum[b];
  sh[tid] = part;
  __syncthreads();
  for (int o = kSelThreads / 2; o > 0; o >>= 1) {
    if (tid < o) sh[tid] += sh[tid + o];
    __syncthreads();
  }
  const uint64_t W = sh[0];
  if (tid == 0) found = -1;
  __syncthreads();
  if (W == 0) {
    if (tid == 0) {
      int64_t i = 0;
      while (i < n && chosen[i]) ++i;   // at most m rows are chosen and m < n
      rows[m] = i < n ? (int32_t)i : -1;
      if (i < n) chosen[i] = 1;
    }
    return;
  }
  const uint64_t t = draw % W;
  // the 256-row block whose cumulative interval holds t
  uint64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kSelThreads) {
    const int64_t b = b0 + tid;
    const uint64_t v = b < nb ? bsum[b] : 0;
    const uint64_t incl = wg_scan(v, sh) + carry;
    const uint64_t tile = sh[kSelThreads - 1];
    if (v > 0 && incl - v <= t && t < incl) {
      found = b;
      found_base = incl - v;
    }
    carry += tile;
    __syncthreads();
    if (found >= 0) break;
  }
  if (found < 0) {   // cannot happen: t < W = the sum of the block sums
    if (tid == 0) rows[m] = -1;
    return;
  }
  // the row within that block
  const int64_t base = found * kPPRows;
  const int64_t i = base + tid;
  const uint64_t v = (tid < kPPRows && i < n) ? w[i] : 0;
  const uint64_t incl = wg_scan(v, sh) + found_base;
  if (v > 0 && incl - v <= t && t < incl) {
    rows[m] = (int32_t)i;
    chosen[i] = 1;
  }
}

}  // namespace

hipError_t pp_place(const int64_t *indptr, const int32_t *indices, const float *values, int64_t n,
                    const int32_t *rows, int32_t m, double *dense, double *nrm2, hipStream_t s) {
  hipLaunchKernelGGL(k_pp_place, dim3(1), dim3(256), 0, s, indptr, indices, values, n, rows, m,
                     dense, nrm2);
  return hipGetLastError();
}

hipError_t pp_weights(const int64_t *indptr, const int32_t *indices, const float *values,
                      int64_t n, const double *dense, double nrm, double *best,
                      const uint8_t *chosen, uint64_t *w, uint64_t *bsum, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pp_weights, dim3((unsigned)((n + kPPRows - 1) / kPPRows)), dim3(kPPRows), 0,
                     s, indptr, indices, values, n, dense, nrm, best, chosen, w, bsum);
  return hipGetLastError();
}

hipError_t pp_select(const uint64_t *bsum, const uint64_t *w, int64_t n, uint64_t draw,
                     uint8_t *chosen, int32_t *rows, int32_t m, hipStream_t s) {
  const int64_t nb = (n + kPPRows - 1) / kPPRows;
  hipLaunchKernelGGL(k_pp_select, dim3(1), dim3(kSelThreads), 0, s, bsum, nb, w, n, draw, chosen,
                     rows, m);
  return hipGetLastError();
}

}  // namespace skm
