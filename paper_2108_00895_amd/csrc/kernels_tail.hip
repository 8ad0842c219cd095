// Per-(chunk, term) lists of non-zero codes for the sparse part of a scoring
// copy (the paper's inverted index G of Sec. 3.2 restricted to non-zero
// entries, kept per 512-centroid chunk).
//
// A term that few centroids of a chunk contain ("tail" term of that chunk: at
// most 1/16 of the chunk's live columns) costs a row far less as a list of its
// non-zero codes than as the chunk's full 512-code slab row (bytes and L2
// footprint).  The scoring kernels take the slab row for the other terms and
// walk these lists, accumulating into LDS, for tail terms.  The decision is
// made per chunk, so a chunk's lists depend on that chunk's codes alone and
// only the chunks holding changed centroids are rebuilt after an update.
#include "internal.h"

namespace skm {
namespace {

constexpr int bytes_of(int P) { return P == SKM_FP32 ? 4 : (P == SKM_BF16 ? 2 : 1); }

// Non-zero mask of the lane's 8 codes (bit v = column 8*lane + v), columns at
// or past `live` masked off.  One 8-, 16- or 32-byte load per lane.
template <int P>
__device__ inline uint32_t lane_nonzero(const uint8_t *slab_row, int lane, int live,
                                        uint32_t bits_out[8]) {
  uint32_t m = 0;
  if (P == SKM_FP32) {
    const uint4 *p = reinterpret_cast<const uint4 *>(slab_row + lane * 32);
    const uint4 a = p[0], b = p[1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int v = 0; v < 8; ++v) bits_out[v] = w[v];
  } else if (P == SKM_BF16) {
    const uint4 a = *reinterpret_cast<const uint4 *>(slab_row + lane * 16);
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      bits_out[2 * v] = w[v] & 0xFFFFu;
      bits_out[2 * v + 1] = w[v] >> 16;
    }
  } else {
    const uint2 a = *reinterpret_cast<const uint2 *>(slab_row + lane * 8);
    const uint32_t w[2] = {a.x, a.y};
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) bits_out[4 * v + q] = (w[v] >> (8 * q)) & 0xFFu;
  }
#pragma unroll
  for (int v = 0; v < 8; ++v)
    if (bits_out[v] != 0u && lane * kColsPerLane + v < live) m |= 1u << v;
  return m;
}

__device__ inline int live_cols(int32_t ncols, int cc) { return min(kChunk, ncols - cc * kChunk); }

// One wavefront per (term, listed chunk): the chunk's non-zero codes of the
// term; a tail term when at most 1/16 of the live columns hold one.  Counts of
// slab-row terms are stored as 0 so that the scan skips them.
template <int P>
__global__ __launch_bounds__(256) void k_tail_count(const uint8_t *tile, int64_t D, int32_t ncols,
                                                    const int32_t *chunks, uint32_t *cnt,
                                                    uint8_t *tail) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= D) return;
  const int cc = chunks[blockIdx.y];
  const int lane = lane_id();
  const int live = live_cols(ncols, cc);
  uint32_t bits[8];
  const uint8_t *row = tile + tile_index(t, (int64_t)cc * kChunk, D) * bytes_of(P);
  int c = __popc(lane_nonzero<P>(row, lane, live, bits));
  for (int m = 1; m < kWave; m <<= 1) c += __shfl_xor(c, m, kWave);
  if (lane == 0) {
    const bool is_tail = 16 * c <= live;
    tail[(int64_t)cc * D + t] = is_tail ? 1 : 0;
    cnt[(int64_t)cc * D + t] = is_tail ? (uint32_t)c : 0u;
  }
}

// Exclusive scan of each listed chunk's counts over terms: off[cc][t], with
// kListFlag set on the chunk's list terms, and off[cc][D] = the chunk's total
// (also in totals[i] for the i-th listed chunk).  Three launches spread over
// the GPU: sums of blocks of kScanTerms terms, a scan of each chunk's block
// sums, and the writes of each block.
constexpr int kScanTerms = 4096;   // terms per block (256 threads x 16)

__global__ __launch_bounds__(256) void k_tail_bsum(const uint32_t *cnt, int64_t D,
                                                   const int32_t *chunks, int64_t nb,
                                                   uint32_t *bsum) {
  __shared__ uint32_t sh[256];
  const int cc = chunks[blockIdx.y];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTerms;
  const uint32_t *c = cnt + (int64_t)cc * D;
  uint32_t v = 0;
  for (int64_t t = t0 + threadIdx.x; t < min<int64_t>(D, t0 + kScanTerms); t += 256) v += c[t];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[(int64_t)blockIdx.y * nb + blockIdx.x] = sh[0];
}

// Block sums -> exclusive block offsets in place, per listed chunk (a
// handful of blocks: one thread walks them).
__global__ void k_tail_bscan(uint32_t *bsum, int64_t nb, int32_t n_list, const int32_t *chunks,
                             int64_t D, uint32_t *off, uint32_t *totals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_list) return;
  uint32_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const uint32_t v = bsum[(int64_t)i * nb + b];
    bsum[(int64_t)i * nb + b] = run;
    run += v;
  }
  off[(int64_t)chunks[i] * (D + 1) + D] = run;
  totals[i] = run;
}

__global__ __launch_bounds__(256) void k_tail_write(const uint32_t *cnt, const uint8_t *tail,
                                                    int64_t D, const int32_t *chunks, int64_t nb,
                                                    const uint32_t *bsum, uint32_t *off) {
  __shared__ uint32_t sh[256];
  const int cc = chunks[blockIdx.y];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTerms + (int64_t)threadIdx.x * 16;
  const uint32_t *c = cnt + (int64_t)cc * D;
  uint32_t v[16], s = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    v[q] = t0 + q < D ? c[t0 + q] : 0u;
    s += v[q];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t y = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
    __syncthreads();
    sh[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t pos = bsum[(int64_t)blockIdx.y * nb + blockIdx.x] + sh[threadIdx.x] - s;
  uint32_t *o = off + (int64_t)cc * (D + 1);
  const uint8_t *fl = tail + (int64_t)cc * D;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (t0 + q < D) o[t0 + q] = pos | (fl[t0 + q] ? kListFlag : 0u);
    pos += v[q];
  }
}

// Entries of the tail terms of the listed chunks, ascending by column within
// (chunk, term): BF16 / FP8: (column << 16) | code; FP32: (column, code bits).
// Chunk cc's entries start at entry cc * stride.
template <int P>
__global__ __launch_bounds__(256) void k_tail_fill(const uint8_t *tile, int64_t D, int32_t ncols,
                                                   const int32_t *chunks, const uint8_t *tail,
                                                   const uint32_t *off, int64_t stride,
                                                   uint32_t *ent) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= D) return;
  const int cc = chunks[blockIdx.y];
  if (!tail[(int64_t)cc * D + t]) return;
  const int lane = lane_id();
  const int live = live_cols(ncols, cc);
  uint32_t bits[8];
  const uint8_t *row = tile + tile_index(t, (int64_t)cc * kChunk, D) * bytes_of(P);
  const uint32_t m = lane_nonzero<P>(row, lane, live, bits);
  const int c = __popc(m);
  int incl = c;
  for (int s = 1; s < kWave; s <<= 1) {
    const int y = __shfl_up(incl, s, kWave);
    if (lane >= s) incl += y;
  }
  uint64_t pos = (uint64_t)cc * (uint64_t)stride + (off[(int64_t)cc * (D + 1) + t] & ~kListFlag) +
                 (uint64_t)(incl - c);
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    if (m & (1u << v)) {
      const uint32_t col = (uint32_t)(lane * kColsPerLane + v);
      if (P == SKM_FP32) {
        ent[2 * pos] = col;
        ent[2 * pos + 1] = bits[v];
      } else {
        ent[pos] = (col << 16) | bits[v];
      }
      ++pos;
    }
  }
}

__global__ void k_tail_bases(uint64_t *base, int nch, int64_t stride) {
  const int cc = blockIdx.x * blockDim.x + threadIdx.x;
  if (cc <= nch) base[cc] = (uint64_t)cc * (uint64_t)stride;
}

}  // namespace

hipError_t tail_count(const uint8_t *tile, int64_t D, int32_t ncols, int prec,
                      const int32_t *chunks, int32_t n_list, uint32_t *cnt, uint8_t *tail,
                      uint32_t *off, uint32_t *totals, uint32_t *bsum, hipStream_t s) {
  if (n_list <= 0 || D <= 0) return hipSuccess;
  const dim3 g((unsigned)((D + 3) / 4), (unsigned)n_list), b(256);
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_tail_count<SKM_FP32>, g, b, 0, s, tile, D, ncols, chunks, cnt, tail);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_tail_count<SKM_BF16>, g, b, 0, s, tile, D, ncols, chunks, cnt, tail);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_tail_count<SKM_FP8_E4M3>, g, b, 0, s, tile, D, ncols, chunks, cnt, tail);
      break;
    default: return hipErrorInvalidValue;
  }
  const int64_t nb = tail_scan_blocks(D);
  hipLaunchKernelGGL(k_tail_bsum, dim3((unsigned)nb, (unsigned)n_list), dim3(256), 0, s, cnt, D,
                     chunks, nb, bsum);
  hipLaunchKernelGGL(k_tail_bscan, dim3((unsigned)((n_list + 63) / 64)), dim3(64), 0, s, bsum, nb,
                     n_list, chunks, D, off, totals);
  hipLaunchKernelGGL(k_tail_write, dim3((unsigned)nb, (unsigned)n_list), dim3(256), 0, s, cnt, tail,
                     D, chunks, nb, bsum, off);
  return hipGetLastError();
}

int64_t tail_scan_blocks(int64_t D) { return (D + kScanTerms - 1) / kScanTerms; }

hipError_t tail_fill(const uint8_t *tile, int64_t D, int32_t ncols, int prec,
                     const int32_t *chunks, int32_t n_list, const uint8_t *tail,
                     const uint32_t *off, int64_t stride, uint32_t *ent, hipStream_t s) {
  if (n_list <= 0 || D <= 0) return hipSuccess;
  const dim3 g((unsigned)((D + 3) / 4), (unsigned)n_list), b(256);
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_tail_fill<SKM_FP32>, g, b, 0, s, tile, D, ncols, chunks, tail, off,
                         stride, ent);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_tail_fill<SKM_BF16>, g, b, 0, s, tile, D, ncols, chunks, tail, off,
                         stride, ent);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_tail_fill<SKM_FP8_E4M3>, g, b, 0, s, tile, D, ncols, chunks, tail, off,
                         stride, ent);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t tail_bases(uint64_t *base, int32_t nch, int64_t stride, hipStream_t s) {
  hipLaunchKernelGGL(k_tail_bases, dim3((unsigned)((nch + 256) / 256)), dim3(256), 0, s, base, nch,
                     stride);
  return hipGetLastError();
}

}  // namespace skm
