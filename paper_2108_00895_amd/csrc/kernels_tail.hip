// Per-(chunk, term) lists of non-zero codes for the sparse part of a scoring
// copy (the paper's inverted index G of Sec. 3.2 restricted to non-zero
// entries, kept per 512-centroid chunk).
//
// A term present in few centroids ("tail" term: at most 1/16 of the columns)
// costs a row far less as a list of its non-zero codes than as a full 512-code
// slab row per chunk (bytes and L2 footprint).  The scoring kernels take the
// dense path for head terms and walk these lists, accumulating into LDS, for
// tail terms.
#include "internal.h"

namespace skm {
namespace {

template <int P>
__device__ inline bool code_nonzero(const uint8_t *slab_row, int col) {
  if (P == SKM_FP32) return reinterpret_cast<const uint32_t *>(slab_row)[col] != 0u;
  if (P == SKM_BF16) return reinterpret_cast<const uint16_t *>(slab_row)[col] != 0u;
  return slab_row[col] != 0u;
}

template <int P>
__device__ inline uint32_t code_bits(const uint8_t *slab_row, int col) {
  if (P == SKM_FP32) return reinterpret_cast<const uint32_t *>(slab_row)[col];
  if (P == SKM_BF16) return reinterpret_cast<const uint16_t *>(slab_row)[col];
  return slab_row[col];
}

constexpr int bytes_of(int P) { return P == SKM_FP32 ? 4 : (P == SKM_BF16 ? 2 : 1); }

// One wavefront per term: non-zero codes per chunk and the term's centroid
// count cf_t (into cf and a histogram over cf values).
template <int P>
__global__ __launch_bounds__(256) void k_tail_count(const uint8_t *tile, int64_t D, int32_t ncols,
                                                    uint32_t *cnt, uint32_t *cf_out,
                                                    uint32_t *hist) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= D) return;
  const int lane = lane_id();
  const int nch = (ncols + kChunk - 1) / kChunk;
  int cf = 0;
  for (int cc = 0; cc < nch; ++cc) {
    const uint8_t *row = tile + tile_index(t, (int64_t)cc * kChunk, D) * bytes_of(P);
    int c = 0;
    for (int v = 0; v < kColsPerLane; ++v) {
      const int col = lane * kColsPerLane + v;
      if (cc * kChunk + col < ncols) c += code_nonzero<P>(row, col) ? 1 : 0;
    }
    for (int m = 1; m < kWave; m <<= 1) c += __shfl_xor(c, m, kWave);
    if (lane == 0) cnt[(int64_t)cc * D + t] = (uint32_t)c;
    cf += c;
  }
  if (lane == 0) {
    cf_out[t] = (uint32_t)cf;
    atomicAdd(&hist[cf], 1u);
  }
}

// Threshold v* on cf: terms with cf > v* take the dense path.  v* is the
// smallest value >= ncols / 16 such that at most dense_max terms exceed it.
// A list entry costs about twelve times a dense column on the device (owner
// search, LDS add), so only terms in at most 1/16 of the centroids go to lists.
__global__ __launch_bounds__(1) void k_tail_threshold(const uint32_t *hist, int32_t ncols,
                                                      int64_t dense_max, uint32_t *thr) {
  int64_t above = 0;   // terms with cf > v
  uint32_t v = (uint32_t)ncols;
  const uint32_t vmin = (uint32_t)(ncols / 16);
  while (v > vmin) {
    if (above + hist[v] > dense_max) break;
    above += hist[v];
    --v;
  }
  *thr = v;
}

// Classifies terms and clears the counts of dense terms.
__global__ void k_tail_class(const uint32_t *cf, int64_t D, int32_t ncols, const uint32_t *thr,
                             uint32_t *cnt, uint8_t *tail) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= D) return;
  const bool is_tail = cf[t] <= *thr;
  tail[t] = is_tail ? 1 : 0;
  if (!is_tail) {
    const int nch = (ncols + kChunk - 1) / kChunk;
    for (int cc = 0; cc < nch; ++cc) cnt[(int64_t)cc * D + t] = 0;
  }
}

// Exclusive scan of one chunk's counts over terms (one workgroup per chunk):
// off[cc][t], off[cc][D] = the chunk's total.
__global__ __launch_bounds__(1024) void k_tail_scan(const uint32_t *cnt, int64_t D, uint32_t *off) {
  __shared__ uint32_t sh[1024];
  const int64_t cc = blockIdx.x;
  const uint32_t *c = cnt + cc * D;
  uint32_t *o = off + cc * (D + 1);
  const int t = threadIdx.x;
  const int64_t per = (D + 1023) / 1024;
  const int64_t lo = min<int64_t>(t * per, D), hi = min(D, lo + per);
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += c[i];
  sh[t] = s;
  __syncthreads();
  for (int w = 1; w < 1024; w <<= 1) {
    uint32_t v = t >= w ? sh[t - w] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  uint32_t pos = sh[t] - s;
  for (int64_t i = lo; i < hi; ++i) {
    o[i] = pos;
    pos += c[i];
  }
  if (t == 1023) o[D] = sh[1023];
}

// base[cc] = start of chunk cc's entries; base[nch] = total.
__global__ void k_tail_bases(const uint32_t *off, int64_t D, int nch, uint64_t *base) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t s = 0;
  for (int cc = 0; cc < nch; ++cc) {
    base[cc] = s;
    s += off[(int64_t)cc * (D + 1) + D];
  }
  base[nch] = s;
}

// Entries of tail terms, ascending by column within (chunk, term):
// BF16 / FP8: (column << 16) | code; FP32: (column, code bits) pairs.
template <int P>
__global__ __launch_bounds__(256) void k_tail_fill(const uint8_t *tile, int64_t D, int32_t ncols,
                                                   const uint8_t *tail, const uint32_t *off,
                                                   const uint64_t *base, uint32_t *ent) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= D || !tail[t]) return;
  const int lane = lane_id();
  const int nch = (ncols + kChunk - 1) / kChunk;
  for (int cc = 0; cc < nch; ++cc) {
    const uint8_t *row = tile + tile_index(t, (int64_t)cc * kChunk, D) * bytes_of(P);
    int c = 0;
    for (int v = 0; v < kColsPerLane; ++v) {
      const int col = lane * kColsPerLane + v;
      if (cc * kChunk + col < ncols) c += code_nonzero<P>(row, col) ? 1 : 0;
    }
    int incl = c;   // inclusive prefix over lanes
    for (int m = 1; m < kWave; m <<= 1) {
      const int y = __shfl_up(incl, m, kWave);
      if (lane >= m) incl += y;
    }
    uint64_t pos = base[cc] + off[(int64_t)cc * (D + 1) + t] + (uint64_t)(incl - c);
    for (int v = 0; v < kColsPerLane; ++v) {
      const int col = lane * kColsPerLane + v;
      if (cc * kChunk + col < ncols && code_nonzero<P>(row, col)) {
        const uint32_t bits = code_bits<P>(row, col);
        if (P == SKM_FP32) {
          ent[2 * pos] = (uint32_t)col;
          ent[2 * pos + 1] = bits;
        } else {
          ent[pos] = ((uint32_t)col << 16) | bits;
        }
        ++pos;
      }
    }
  }
}

}  // namespace

hipError_t tail_count(const uint8_t *tile, int64_t D, int32_t ncols, int prec, int64_t dense_max,
                      uint32_t *cnt, uint32_t *cf, uint32_t *hist, uint8_t *tail, uint32_t *off,
                      uint64_t *base, hipStream_t s) {
  const int nch = (ncols + kChunk - 1) / kChunk;
  const dim3 g((unsigned)((D + 3) / 4)), b(256);
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t *>(hist), 0, (int64_t)ncols + 2, s);
  if (e != hipSuccess) return e;
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_tail_count<SKM_FP32>, g, b, 0, s, tile, D, ncols, cnt, cf, hist);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_tail_count<SKM_BF16>, g, b, 0, s, tile, D, ncols, cnt, cf, hist);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_tail_count<SKM_FP8_E4M3>, g, b, 0, s, tile, D, ncols, cnt, cf, hist);
      break;
    default: return hipErrorInvalidValue;
  }
  uint32_t *thr = hist + ncols + 1;
  hipLaunchKernelGGL(k_tail_threshold, dim3(1), dim3(1), 0, s, hist, ncols, dense_max, thr);
  hipLaunchKernelGGL(k_tail_class, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, cf, D, ncols,
                     thr, cnt, tail);
  hipLaunchKernelGGL(k_tail_scan, dim3((unsigned)nch), dim3(1024), 0, s, cnt, D, off);
  hipLaunchKernelGGL(k_tail_bases, dim3(1), dim3(64), 0, s, off, D, nch, base);
  return hipGetLastError();
}

hipError_t tail_fill(const uint8_t *tile, int64_t D, int32_t ncols, int prec, const uint8_t *tail,
                     const uint32_t *off, const uint64_t *base, uint32_t *ent, hipStream_t s) {
  const dim3 g((unsigned)((D + 3) / 4)), b(256);
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_tail_fill<SKM_FP32>, g, b, 0, s, tile, D, ncols, tail, off, base, ent);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_tail_fill<SKM_BF16>, g, b, 0, s, tile, D, ncols, tail, off, base, ent);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_tail_fill<SKM_FP8_E4M3>, g, b, 0, s, tile, D, ncols, tail, off, base, ent);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace skm
