// The dense head of the vocabulary on the matrix cores.
//
// Under a Zipf law the most frequent terms occur in a large share of the rows
// and in nearly every centroid, so their part of the scores s_ij (Sec. 2) is a
// dense product: X_head (rows x H) times C_head^T (H x centroids).  Both sides
// are held in BF16 — the row values rounded once, the centroid side a copy of
// the scoring codes — and multiplied with v_mfma_f32_32x32x16_bf16 into FP32
// head scores, one batch of rows at a time.  The sparse scoring kernel then
// starts every (row, chunk) item from those head scores and adds the row's
// remaining terms; the certified bound accounts for the extra rounding of the
// row values and for the matrix-core accumulation.
#include "internal.h"

namespace skm {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);   // finite, non-negative inputs only
  return (uint16_t)(u >> 16);
}

// Document frequency of every term.
__global__ void k_df(const int32_t *indices, int64_t nnz, uint32_t *df) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&df[indices[q]], 1u);
}

// Per row: the number of non-head terms (into cnt[row]).
__global__ void k_head_count(const int64_t *indptr, const int32_t *indices, int64_t n_rows,
                             const int32_t *slot, int64_t *cnt) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  int64_t c = 0;
  for (int64_t q = indptr[row]; q < indptr[row + 1]; ++q) c += slot[indices[q]] < 0 ? 1 : 0;
  cnt[row] = c;
}

// One wavefront per row: the row's head values (BF16) into its dense X_head
// row, assembled in LDS and written with 16-byte stores, and its other terms
// into the remainder CSR (order kept).
__global__ __launch_bounds__(256) void k_head_split(const int64_t *indptr, const int32_t *indices,
                                                    const float *values, int64_t n_rows,
                                                    const int32_t *slot, int32_t H,
                                                    const int64_t *r_indptr, int32_t *r_indices,
                                                    float *r_values, uint16_t *xh) {
  extern __shared__ uint16_t hrow_all[];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= n_rows) return;
  uint16_t *hrow = hrow_all + (int64_t)wave * H;
  for (int h = lane; h < H; h += kWave) hrow[h] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int64_t b = indptr[row], e = indptr[row + 1];
  int64_t out = r_indptr[row];
  for (int64_t q0 = b; q0 < e; q0 += kWave) {
    const int64_t q = q0 + lane;
    int s = -1;
    int32_t t = 0;
    float v = 0.f;
    if (q < e) {
      t = indices[q];
      v = values[q];
      s = slot[t];
    }
    if (s >= 0) hrow[s] = bf16_rne(v);
    const bool rest = q < e && s < 0;
    const uint64_t m = __ballot(rest);
    if (rest) {
      const int64_t o = out + __popcll(m & lanemask_lt());
      r_indices[o] = t;
      r_values[o] = v;
    }
    out += __popcll(m);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint4 *src = reinterpret_cast<const uint4 *>(hrow);
  uint4 *dst = reinterpret_cast<uint4 *>(xh + row * (int64_t)H);
  for (int i = lane; i < H / 8; i += kWave) dst[i] = src[i];
}

// C_head[j][h] = centroid j at head term h as BF16: for BF16 scoring the code
// itself; for FP8 scoring the BF16 rounding of the FP64 master value divided
// by the centroid's power-of-two scale (the head part of an FP8 score thus
// carries BF16 accuracy; the scale is applied with the rest of the score).
// Rows j >= k are zero.  A 64 x 64 block is transposed through LDS so that the
// C_head writes are coalesced.
template <int P>
__global__ __launch_bounds__(256) void k_head_codes(const uint8_t *tile, const double *master,
                                                    const float *scale, int64_t D, int32_t k,
                                                    const int32_t *terms, int32_t H,
                                                    int32_t k_pad, uint16_t *ch) {
  __shared__ uint16_t t_sh[64][65];
  const int j0 = blockIdx.x * 64, h0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int h = h0 + r, j = j0 + tx;
    uint16_t v = 0;
    if (h < H && j < k) {
      if (P == SKM_BF16) {
        v = reinterpret_cast<const uint16_t *>(tile)[tile_index(terms[h], j, D)];
      } else {
        v = encode_bf16(ldexp(master[(int64_t)j * D + terms[h]], -ilogbf(scale[j])));
      }
    }
    t_sh[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r, h = h0 + tx;
    if (j < k_pad && h < H) ch[(int64_t)j * H + h] = t_sh[tx][r];
  }
}

// Rows of head codes of the listed centroids (16-byte copies; H % 8 == 0).
__global__ __launch_bounds__(256) void k_gather_head(const uint16_t *ch, int32_t H,
                                                     const int32_t *ids, uint16_t *out) {
  const uint4 *src = reinterpret_cast<const uint4 *>(ch + (int64_t)ids[blockIdx.x] * H);
  uint4 *dst = reinterpret_cast<uint4 *>(out + (int64_t)blockIdx.x * H);
  for (int i = threadIdx.x; i < H / 8; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------------ GEMM
// hs[r][j] = sum_h xh[row0 + r][h] * ch[j][h] for r < nb, j < ncp (ch already
// offset to the first column).
// Workgroup tile (64 WM) rows x 256 centroids, K step GK through LDS in two
// stages; WM x 2 wavefronts, each computing 64 x 128 with 2 x 4 MFMA 32x32x16
// blocks.  The launch uses WM = 4, GK = 64 (144 KiB of LDS, one workgroup per
// CU); WM = 2, GK = 32 (60 KiB, two workgroups per CU, so that one's first
// loads and final stores overlap the other's products) measured 10 % slower
// on the head batches of a 2e6-row corpus.  Operand rows are padded by 16
// bytes so that the 16-byte operand reads of consecutive rows fall on distinct
// banks.  Lane layout of v_mfma_f32_32x32x16_bf16: A operand lane l
// holds row l%32, k = 8*(l/32) .. +8; B operand lane l holds column l%32, same
// k; the FP32 result element (8g + 4*(l/32) + e, l%32) sits in accumulator
// 4g + e.
constexpr int kGN = 256;
constexpr int64_t kXcdCols = 2;   // column tiles (of 256) per XCD

// Column-tile counts the XCD-aware placement covers: a power of two that
// splits into at most 8 groups of kXcdCols (or fewer) tiles.
__host__ __device__ inline bool xcd_placement(int64_t ncb) {
  return ncb >= 1 && ncb <= 8 * kXcdCols && (ncb & (ncb - 1)) == 0;
}

// Workgroups of one head product launch with row tiles of gm rows.
inline int64_t gemm_blocks(int64_t nb, int64_t ncb, int64_t gm) {
  const int64_t nrb = (nb + gm - 1) / gm;
  if (!xcd_placement(ncb)) return nrb * ncb;
  const int64_t cpx = ncb < kXcdCols ? ncb : kXcdCols;
  const int64_t gr = 8 / (ncb / cpx);
  return 8 * ((nrb + gr - 1) / gr) * cpx;
}

template <int GK, int WM>
__global__ __launch_bounds__(WM * 128) void k_head_gemm(const uint16_t *__restrict__ xh, int32_t H,
                                                        int64_t row0, int64_t nb,
                                                        const int32_t *__restrict__ rows,
                                                        const uint16_t *__restrict__ ch,
                                                        int64_t ncp, float *__restrict__ hs,
                                                        int64_t ldh) {
  constexpr int kT = WM * 128;           // threads
  constexpr int kGM = WM * 64;           // rows of the tile
  constexpr int kRow = GK * 2 + 16;      // LDS bytes per tile row
  constexpr int kPPR = GK / 8;           // 16-byte pieces per tile row
  constexpr int kRPP = kT / kPPR;        // tile rows moved per pass of the workgroup
  constexpr int kNA = kGM / kRPP;        // passes per A tile
  constexpr int kNB = kGN / kRPP;        // passes per B tile
  static_assert(kNA >= 1 && kNB >= 1 && kGM % kRPP == 0 && kGN % kRPP == 0, "tile shape");
  __shared__ __attribute__((aligned(16))) uint8_t lds_a[2][kGM * kRow];
  __shared__ __attribute__((aligned(16))) uint8_t lds_b[2][kGN * kRow];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 31, kg = lane >> 5;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t ncb = ncp / kGN;
  int64_t rb, cb;
  if (xcd_placement(ncb)) {
    // XCD-aware placement: workgroups are dealt to the 8 XCDs round-robin;
    // XCD x takes kXcdCols column tiles (their B tiles stay in its L2) and
    // every (8 / groups)-th row tile, the column tiles of one row tile on
    // consecutive slots so that its A tile is fetched into that L2 once.
    const int64_t cpx = ncb < kXcdCols ? ncb : kXcdCols;
    const int64_t gc = ncb / cpx, gr = 8 / gc;
    const int64_t x = blockIdx.x % 8, slot = blockIdx.x / 8;
    cb = (x % gc) * cpx + slot % cpx;
    rb = (slot / cpx) * gr + x / gc;
    if (rb * kGM >= nb) return;
  } else {
    rb = blockIdx.x / ncb;
    cb = blockIdx.x - rb * ncb;
  }
  const int64_t r_base = rb * kGM, c_base = cb * kGN;

  // global -> register staging: thread t moves piece (row pr + kRPP u, k
  // offset 8 kq) of the A tile (u < kNA) and of the B tile (u < kNB)
  const int pr = tid / kPPR, kq = tid % kPPR;
  const int so = pr * kRow + kq * 16;   // LDS offset of piece u: so + kRPP u rows
  // Rows at or past nb read row nb - 1 instead: their results are never
  // stored, and every output row depends on its own A row only.
  const v4u *xv = reinterpret_cast<const v4u *>(xh);
  const v4u *cv = reinterpret_cast<const v4u *>(ch);
  const int64_t h8 = H / 8;
  int64_t oa[kNA], ob[kNB];
#pragma unroll
  for (int u = 0; u < kNA; ++u) {
    const int64_t r = row0 + min<int64_t>(r_base + pr + kRPP * u, nb - 1);
    oa[u] = (rows ? (int64_t)rows[r] : r) * h8 + kq;
  }
#pragma unroll
  for (int u = 0; u < kNB; ++u) ob[u] = (c_base + pr + kRPP * u) * h8 + kq;
  v4u ra[kNA], rbv[kNB];
#pragma unroll
  for (int u = 0; u < kNA; ++u) ra[u] = xv[oa[u]];
#pragma unroll
  for (int u = 0; u < kNB; ++u) rbv[u] = cv[ob[u]];

  f32x16_t acc[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int n4 = 0; n4 < 4; ++n4)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mb][n4][i] = 0.f;

  const int nk = H / GK;
#pragma unroll
  for (int u = 0; u < kNA; ++u) *reinterpret_cast<v4u *>(&lds_a[0][so + kRPP * u * kRow]) = ra[u];
#pragma unroll
  for (int u = 0; u < kNB; ++u) *reinterpret_cast<v4u *>(&lds_b[0][so + kRPP * u * kRow]) = rbv[u];
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      const int q = (kt + 1) * kPPR;
#pragma unroll
      for (int u = 0; u < kNA; ++u) ra[u] = xv[oa[u] + q];
#pragma unroll
      for (int u = 0; u < kNB; ++u) rbv[u] = cv[ob[u] + q];
    }
#pragma unroll
    for (int ks = 0; ks < GK / 16; ++ks) {
      bf16x8_t a[2], b[4];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
        a[mb] = *reinterpret_cast<const bf16x8_t *>(
            &lds_a[cur][(wm * 64 + mb * 32 + li) * kRow + ks * 32 + kg * 16]);
#pragma unroll
      for (int n4 = 0; n4 < 4; ++n4)
        b[n4] = *reinterpret_cast<const bf16x8_t *>(
            &lds_b[cur][(wn * 128 + n4 * 32 + li) * kRow + ks * 32 + kg * 16]);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int n4 = 0; n4 < 4; ++n4)
          acc[mb][n4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mb], b[n4], acc[mb][n4], 0, 0, 0);
    }
    if (kt + 1 < nk) {
#pragma unroll
      for (int u = 0; u < kNA; ++u)
        *reinterpret_cast<v4u *>(&lds_a[cur ^ 1][so + kRPP * u * kRow]) = ra[u];
#pragma unroll
      for (int u = 0; u < kNB; ++u)
        *reinterpret_cast<v4u *>(&lds_b[cur ^ 1][so + kRPP * u * kRow]) = rbv[u];
    }
    __syncthreads();
  }

#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = r_base + wm * 64 + mb * 32 + 8 * g + 4 * kg + e;
        if (r < nb) {
          float *o = hs + r * ldh + c_base + wn * 128 + li;
          // written once, read by the sparse kernel much later: non-temporal
#pragma unroll
          for (int n4 = 0; n4 < 4; ++n4)
            __builtin_nontemporal_store(acc[mb][n4][4 * g + e], o + n4 * 32);
        }
      }
}

// Shape of the head product: K step (H is a multiple of 64, so of either
// step) and wavefront rows.
constexpr int kHeadGK = 64, kHeadWM = 4;

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of n int64 values into out[0..n] (out[n] = total):
// per-block sums, one block scans them, then each block writes its outputs.
constexpr int kScanBlock = 1024, kScanPer = 16;

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const int64_t *in, int64_t n,
                                                          int64_t *bsum) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanPer;
  int64_t s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t q = base + (int64_t)i * kScanBlock + threadIdx.x;
    if (q < n) s += in[q];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kScanBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_bsums(int64_t *bsum, int64_t nblk,
                                                           int64_t *total) {
  __shared__ int64_t sh[kScanBlock];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nblk; c0 += kScanBlock) {
    const int64_t q = c0 + threadIdx.x;
    const int64_t v = q < nblk ? bsum[q] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < kScanBlock; w <<= 1) {
      const int64_t y = (int)threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
      __syncthreads();
      sh[threadIdx.x] += y;
      __syncthreads();
    }
    if (q < nblk) bsum[q] = carry + sh[threadIdx.x] - v;
    carry += sh[kScanBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_write(const int64_t *in, int64_t n,
                                                           const int64_t *bsum, int64_t *out) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanPer;
  int64_t carry = bsum[blockIdx.x];
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t q = base + (int64_t)i * kScanBlock + threadIdx.x;
    const int64_t v = q < n ? in[q] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < kScanBlock; w <<= 1) {
      const int64_t y = (int)threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
      __syncthreads();
      sh[threadIdx.x] += y;
      __syncthreads();
    }
    if (q < n) out[q] = carry + sh[threadIdx.x] - v;
    carry += sh[kScanBlock - 1];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_df(const int32_t *indices, int64_t nnz, uint32_t *df, int64_t D, hipStream_t s) {
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t *>(df), 0, D, s);
  if (e != hipSuccess || nnz == 0) return e;
  const int64_t g = std::min<int64_t>((nnz + 255) / 256, 65536);
  hipLaunchKernelGGL(k_df, dim3((unsigned)g), dim3(256), 0, s, indices, nnz, df);
  return hipGetLastError();
}

hipError_t launch_head_split(const int64_t *indptr, const int32_t *indices, const float *values,
                             int64_t n_rows, const int32_t *slot, int32_t H, int64_t *cnt,
                             int64_t *scan_work, int64_t *r_indptr, int32_t *r_indices,
                             float *r_values, uint16_t *xh, hipStream_t s) {
  if (n_rows <= 0) return launch_fill_i32(reinterpret_cast<int32_t *>(r_indptr), 0, 2, s);
  hipLaunchKernelGGL(k_head_count, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s, indptr,
                     indices, n_rows, slot, cnt);
  const int64_t nblk = (n_rows + (int64_t)kScanBlock * kScanPer - 1) / ((int64_t)kScanBlock * kScanPer);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nblk), dim3(kScanBlock), 0, s, cnt, n_rows, scan_work);
  hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kScanBlock), 0, s, scan_work, nblk, r_indptr + n_rows);
  hipLaunchKernelGGL(k_scan_write, dim3((unsigned)nblk), dim3(kScanBlock), 0, s, cnt, n_rows,
                     scan_work, r_indptr);
  const size_t lds = sizeof(uint16_t) * 4 * (size_t)H;
  hipLaunchKernelGGL(k_head_split, dim3((unsigned)((n_rows + 3) / 4)), dim3(256), lds, s, indptr,
                     indices, values, n_rows, slot, H, (const int64_t *)r_indptr, r_indices,
                     r_values, xh);
  return hipGetLastError();
}

int64_t head_split_scan_blocks(int64_t n_rows) {
  return (n_rows + (int64_t)kScanBlock * kScanPer - 1) / ((int64_t)kScanBlock * kScanPer) + 1;
}

hipError_t launch_head_codes(const uint8_t *tile, const double *master, const float *scale,
                             int64_t D, int32_t k, int prec, const int32_t *terms, int32_t H,
                             int32_t k_pad, uint16_t *ch, hipStream_t s) {
  const dim3 g((unsigned)((k_pad + 63) / 64), (unsigned)((H + 63) / 64)), b(256);
  switch (prec) {
    case SKM_BF16:
      hipLaunchKernelGGL(k_head_codes<SKM_BF16>, g, b, 0, s, tile, master, scale, D, k, terms, H,
                         k_pad, ch);
      break;
    case SKM_FP8_E4M3:
      if (!master || !scale) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_head_codes<SKM_FP8_E4M3>, g, b, 0, s, tile, master, scale, D, k, terms,
                         H, k_pad, ch);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_head_gemm(const uint16_t *xh, int32_t H, int64_t row0, int64_t nb,
                            const int32_t *rows, const uint16_t *ch, int64_t col0, int64_t ncols,
                            float *hs, int64_t ldh, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (H % 64 != 0 || ncols % kGN != 0 || ldh < ncols) return hipErrorInvalidValue;
  const int64_t blocks = gemm_blocks(nb, ncols / kGN, 64 * kHeadWM);
  hipLaunchKernelGGL((k_head_gemm<kHeadGK, kHeadWM>), dim3((unsigned)blocks), dim3(128 * kHeadWM),
                     0, s, xh, H, row0, nb, rows, ch + col0 * (int64_t)H, ncols, hs, ldh);
  return hipGetLastError();
}

hipError_t launch_gather_head(const uint16_t *ch, int32_t H, const int32_t *ids, int32_t n,
                              uint16_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_head, dim3((unsigned)n), dim3(256), 0, s, ch, H, ids, out);
  return hipGetLastError();
}

}  // namespace skm
