// Assignment kernels: low-precision gather-FMA scoring with a fused top-two
// argmax (FP8: a fused summary of certified bounds) and certification (paper
// Sec. 2, Sec. 3.1), and the exact FP64 tier.
//
// Layout: the scoring copy of the centroids is term-major, codes[t * ld + j],
// so one term's codes for 512 consecutive centroids are contiguous: a wavefront
// scores one row against a 512-centroid chunk, lane l holding centroids
// [8l, 8l + 8) of the chunk, and walks the row's terms; each step is one
// coalesced 16 B (BF16), 32 B (FP32) or 8 B (FP8) load per lane plus eight FMAs.
// Row terms are broadcast with v_readlane from a 64-term register batch.
#include <algorithm>

#include "internal.h"

namespace skm {
namespace {

template <int P>
struct Codes;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

// Raw buffer loads: the resource (slab base and size) lives in scalar
// registers, the term row's byte offset is a scalar offset and the lane's
// column offset a 32-bit vector offset.  Reads past the slab return zero.
template <>
struct Codes<SKM_FP32> {
  static constexpr int kBytes = 4;
  static constexpr int kEntWords = 2;
  __device__ static void entry(const uint32_t *e, int &col, float &v) {
    col = (int)e[0];
    v = __uint_as_float(e[1]);
  }
  struct raw_t {
    float4 a, b;
  };
  __device__ static raw_t load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    const v4i x = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
    const v4i y = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16, soff, 0);
    return raw_t{make_float4(__int_as_float(x[0]), __int_as_float(x[1]), __int_as_float(x[2]),
                             __int_as_float(x[3])),
                 make_float4(__int_as_float(y[0]), __int_as_float(y[1]), __int_as_float(y[2]),
                             __int_as_float(y[3]))};
  }
  __device__ static void fma8(const raw_t &r, float x, float acc[8]) {
    acc[0] = fmaf(x, r.a.x, acc[0]);
    acc[1] = fmaf(x, r.a.y, acc[1]);
    acc[2] = fmaf(x, r.a.z, acc[2]);
    acc[3] = fmaf(x, r.a.w, acc[3]);
    acc[4] = fmaf(x, r.b.x, acc[4]);
    acc[5] = fmaf(x, r.b.y, acc[5]);
    acc[6] = fmaf(x, r.b.z, acc[6]);
    acc[7] = fmaf(x, r.b.w, acc[7]);
  }
};

template <>
struct Codes<SKM_BF16> {
  static constexpr int kBytes = 2;
  static constexpr int kEntWords = 1;
  __device__ static void entry(const uint32_t *e, int &col, float &v) {
    col = (int)(e[0] >> 16);
    v = __uint_as_float(e[0] << 16);
  }
  using raw_t = uint4;
  __device__ static raw_t load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    const v4i x = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
    return make_uint4((uint32_t)x[0], (uint32_t)x[1], (uint32_t)x[2], (uint32_t)x[3]);
  }
  __device__ static void fma8(const raw_t &r, float x, float acc[8]) {
    // little-endian: the lower half-word is the lower column
    acc[0] = fmaf(x, __uint_as_float(r.x << 16), acc[0]);
    acc[1] = fmaf(x, __uint_as_float(r.x & 0xFFFF0000u), acc[1]);
    acc[2] = fmaf(x, __uint_as_float(r.y << 16), acc[2]);
    acc[3] = fmaf(x, __uint_as_float(r.y & 0xFFFF0000u), acc[3]);
    acc[4] = fmaf(x, __uint_as_float(r.z << 16), acc[4]);
    acc[5] = fmaf(x, __uint_as_float(r.z & 0xFFFF0000u), acc[5]);
    acc[6] = fmaf(x, __uint_as_float(r.w << 16), acc[6]);
    acc[7] = fmaf(x, __uint_as_float(r.w & 0xFFFF0000u), acc[7]);
  }
};

template <>
struct Codes<SKM_FP8_E4M3> {
  static constexpr int kBytes = 1;
  static constexpr int kEntWords = 1;
  __device__ static void entry(const uint32_t *e, int &col, float &v) {
    col = (int)(e[0] >> 16);
    v = __builtin_amdgcn_cvt_pk_f32_fp8((int)(e[0] & 0xFFu), false)[0];
  }
  using raw_t = uint2;
  __device__ static raw_t load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    const v2i x = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
    return make_uint2((uint32_t)x[0], (uint32_t)x[1]);
  }
  __device__ static void fma8(const raw_t &r, float x, float acc[8]) {
    // v_cvt_pk_f32_fp8 decodes two OCP E4M3 bytes (word_sel picks bytes 2,3)
    auto p0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r.x, false);
    auto p1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r.x, true);
    auto p2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r.y, false);
    auto p3 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r.y, true);
    acc[0] = fmaf(x, p0[0], acc[0]);
    acc[1] = fmaf(x, p0[1], acc[1]);
    acc[2] = fmaf(x, p1[0], acc[2]);
    acc[3] = fmaf(x, p1[1], acc[3]);
    acc[4] = fmaf(x, p2[0], acc[4]);
    acc[5] = fmaf(x, p2[1], acc[5]);
    acc[6] = fmaf(x, p3[0], acc[6]);
    acc[7] = fmaf(x, p3[1], acc[7]);
  }
};

__device__ inline int64_t uniform64(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int32_t uniform32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// acc[c] += sum over the row's terms of x_t * code(t, c0 + 8*lane + c).
// Head terms: one slab-row load per term (8 loads in flight per lane) and
// eight FMAs into registers.  Tail terms of the chunk: the term's list of
// non-zero codes in this chunk, lanes over entries, products added into the
// wave's 512-float LDS accumulator lacc, folded into acc at the end.  A term's
// list word (entry offset, kListFlag = a tail term of this chunk) gives both
// the choice and the list, so the list walk waits for no further load.  The
// order of the sum differs from the term order; the error bound allows any
// order (at most two roundings per term plus the final merge).  Lanes whose
// columns all lie at or past nvalid (a ragged or narrow compacted chunk) issue
// no loads.
template <int P>
__device__ inline void score_chunk(int64_t b, int64_t e, const int32_t *__restrict__ indices,
                                   const float *__restrict__ values, const uint8_t *__restrict__ tile,
                                   int64_t D, int64_t c0, int64_t nvalid, float acc[8],
                                   const TailView &tv, float *lacc) {
  using C = Codes<P>;
  const int lane = lane_id();
  const bool act = (int64_t)lane * kColsPerLane < nvalid;
  const int64_t cc = c0 / kChunk;
  // chunk slab [D][512] as a buffer resource in scalar registers
  const uint8_t *slab = reinterpret_cast<const uint8_t *>(
      uniform64(reinterpret_cast<int64_t>(tile + tile_index(0, c0, D) * C::kBytes)));
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(slab), 0, (int)(D * kChunk * C::kBytes), 0x00020000);
  const int voff = lane * kColsPerLane * C::kBytes;
  constexpr int rowbytes = kChunk * C::kBytes;
  const uint32_t *toff = tv.off ? tv.off + cc * (D + 1) : nullptr;
  const uint32_t *tent = tv.off ? tv.ent + (int64_t)tv.base[cc] * C::kEntWords : nullptr;
  bool used_lds = false;
  for (int64_t q0 = b; q0 < e; q0 += kWave) {
    const int cnt = (int)((e - q0) < kWave ? (e - q0) : kWave);
    int my_t = 0;
    float my_x = 0.f;
    uint32_t w0 = 0, w1 = 0;
    if (lane < cnt) {
      // streamed once per (row, chunk): non-temporal, to leave L2 to the codes
      my_t = __builtin_nontemporal_load(indices + q0 + lane);
      my_x = __builtin_nontemporal_load(values + q0 + lane);
      if (toff) {
        w0 = toff[my_t];
        w1 = toff[my_t + 1];
      }
    }
    const bool my_tail = (w0 & kListFlag) != 0u;
    uint64_t dmask = __ballot(lane < cnt && !my_tail);
    const uint64_t tmask = __ballot(my_tail);
    while (__popcll(dmask) >= 8) {
      int u[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        u[v] = __builtin_ctzll(dmask);
        dmask &= dmask - 1;
      }
      int so[8];
      float xs[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        so[v] = __builtin_amdgcn_readlane(my_t, u[v]) * rowbytes;
        xs[v] = readlane_f(my_x, u[v]);
      }
      if (act) {
        typename C::raw_t r[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) r[v] = C::load(rs, voff, so[v]);
#pragma unroll
        for (int v = 0; v < 8; ++v) C::fma8(r[v], xs[v], acc);
      }
    }
    while (dmask) {
      const int u = __builtin_ctzll(dmask);
      dmask &= dmask - 1;
      const int so0 = __builtin_amdgcn_readlane(my_t, u) * rowbytes;
      const float x0 = readlane_f(my_x, u);
      if (act) {
        typename C::raw_t r0 = C::load(rs, voff, so0);
        C::fma8(r0, x0, acc);
      }
    }
    if (tmask) {
      // All tail terms of the batch at once: lane l owns list [o0, o0 + len)
      // of its term; the lists are flattened and each lane takes one entry
      // per step, finding its owner by a binary search over the prefix sums.
      used_lds = true;
      const uint32_t o0 = w0 & ~kListFlag;
      const uint32_t len = my_tail ? (w1 & ~kListFlag) - o0 : 0u;
      uint32_t incl = len;
#pragma unroll
      for (int m = 1; m < kWave; m <<= 1) {
        const uint32_t y = __shfl_up(incl, m, kWave);
        if (lane >= m) incl += y;
      }
      const uint32_t excl = incl - len;
      const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
      for (uint32_t f0 = 0; f0 < total; f0 += 2 * kWave) {
        int col[2];
        float v[2], x[2];
        bool ok[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t f = f0 + h * kWave + lane;
          ok[h] = f < total;
          int own = 0;
#pragma unroll
          for (int step = 32; step > 0; step >>= 1) {
            const uint32_t pv = __shfl(incl, own + step - 1, kWave);
            if (pv <= f) own += step;
          }
          own = own > kWave - 1 ? kWave - 1 : own;
          const uint32_t ou = __shfl(o0, own, kWave);
          const uint32_t eu = __shfl(excl, own, kWave);
          x[h] = __shfl(my_x, own, kWave);
          col[h] = 0;
          v[h] = 0.f;
          if (ok[h]) C::entry(tent + (int64_t)(ou + (f - eu)) * C::kEntWords, col[h], v[h]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (ok[h]) atomicAdd(&lacc[col[h]], x[h] * v[h]);
      }
    }
  }
  if (used_lds) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      acc[v] += lacc[lane * kColsPerLane + v];
      lacc[lane * kColsPerLane + v] = 0.f;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

__device__ inline void zero_lacc(float *lacc) {
  for (int i = lane_id(); i < kChunk; i += kWave) lacc[i] = 0.f;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

struct RowPlan {
  const uint8_t *tile;
  int32_t ncols;
  const int32_t *colmap;   // column -> centroid id, nullptr = identity
  bool ncc;
  int32_t ap;
  bool done;               // finished by the index path
  const TailView *tv;
};

__device__ inline RowPlan plan_row(const ScoreArgs &a, int64_t row, bool allow_ncc) {
  RowPlan p{a.tile, a.k, nullptr, false, -1, false, &a.tv};
  if (a.mode && a.mode[row] == 2) {
    p.ncols = 0;
    p.done = true;
    return p;
  }
  if (allow_ncc && a.a_prev) {
    const int32_t ap = a.a_prev[row];
    if (!a.changed[ap]) {
      p.tile = a.tile_ch;
      p.ncols = a.n_ch;
      p.colmap = a.ch_ids;
      p.ncc = true;
      p.ap = ap;
      p.tv = &a.tv_ch;
    }
  }
  return p;
}

// Certified bound |s^ - s| <= kap * s^ + A of the scores behind the chunk
// partials (head product plus sparse terms when head scores were used).
__device__ inline void part_bound(const ScoreArgs &a, int64_t row, int64_t n, double &kap,
                                  double &A) {
  const double l1 = a.xl1[row];
  if (a.head_H > 0) {
    kap = bound_kappa_head(n, a.head_H, a.uq);
    A = bound_abs(n, l1, a.abs_coef) + bound_abs_head(a.head_H, l1, a.abs_coef);
  } else {
    kap = bound_kappa(n, a.uq);
    A = bound_abs(n, l1, a.abs_coef);
  }
}

// Per-(row, chunk) top-two of the low-precision scores (FP8: bound summary,
// see Partial).  The grid is
// persistent and walks items chunk-major (item = chunk * n_rows + row), so all
// wavefronts sweep the same 512-centroid slice of the codes at the same time
// and its hot term rows stay in L2 / the Infinity Cache instead of being
// re-fetched from HBM for every row.  BF16 / FP8: built for the register
// budget of eight waves per SIMD (the eight loads in flight still fit); FP32
// would spill there.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == SKM_FP32 ? 1 : 8)))
void k_score_part(ScoreArgs a, Partial *__restrict__ part, int64_t n_items) {
  __shared__ float lacc_all[4][kChunk];
  const int wave = uniform32(threadIdx.x >> 6);
  const int lane = lane_id();
  float *lacc = lacc_all[wave];
  zero_lacc(lacc);
  const int64_t stride = (int64_t)gridDim.x * 4;
  const int64_t nb = a.n_dev ? uniform64(*a.n_dev) : a.nb;
  if (a.n_dev) n_items = (int64_t)a.c_count * nb;
  for (int64_t it = (int64_t)blockIdx.x * 4 + wave; it < n_items; it += stride) {
    const int64_t ci = uniform64(it / nb);
    const int64_t r = uniform64(it - ci * nb);
    const int64_t row = a.row_list ? uniform64((int64_t)a.row_list[a.row0 + r]) : a.row0 + r;
    const int64_t c = a.c_first + ci;
    const RowPlan pl = plan_row(a, row, true);
    if (a.ncc_only && !pl.ncc) continue;
    const int64_t c0 = c * kChunk;
    if (c0 >= pl.ncols) continue;
    const int64_t b = uniform64(a.sc_indptr[row]);
    const int64_t e = uniform64(a.sc_indptr[row + 1]);
    // FP32 / BF16: the sparse terms are added onto the head scores of these 8
    // columns (kernels_head.hip).  FP8: the head part (BF16 head codes) and
    // the sparse part (FP8 codes) are summed apart and added once, so that
    // each part keeps its own bound.
    constexpr bool kSplit = P == SKM_FP8_E4M3;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float hh[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    auto load_head = [&](float *dst) {
      const float4 *h = reinterpret_cast<const float4 *>(a.hs + r * a.hs_ld + ci * kChunk +
                                                         lane * kColsPerLane);
      // streamed once: non-temporal loads, to leave L2 to the codes
      const v4f h0 = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(h));
      const v4f h1 = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(h) + 1);
      dst[0] = h0.x;
      dst[1] = h0.y;
      dst[2] = h0.z;
      dst[3] = h0.w;
      dst[4] = h1.x;
      dst[5] = h1.y;
      dst[6] = h1.z;
      dst[7] = h1.w;
    };
    if (!kSplit && a.hs) load_head(acc);
    score_chunk<P>(b, e, a.sc_indices, a.sc_values, pl.tile, a.D, c0, pl.ncols - c0, acc, *pl.tv,
                   lacc);
    if (kSplit && a.hs) load_head(hh);   // read after the sparse loop: no registers held
    if constexpr (kSplit) {
      // certified bounds per column (float arithmetic, inflated so that every
      // rounding leaves them conservative): E = kh h + ks r + 2^-24 (h + r) + A,
      // then lb = s - E - M and ub = s + E + M with M = 2^-21 (s + E)
      const int64_t n_s = e - b;
      const float ks = f_up(bound_kappa(n_s, a.uq));
      const float kh = a.hs ? f_up(bound_kappa_head_bf16(a.head_H)) : 0.f;
      const float A = f_up((bound_abs(n_s, a.xl1[row], a.abs_coef) +
                            (a.hs ? (double)a.head_H * 0x1p-120 : 0.0)) * (1.0 + 0x1p-20));
      float lb = -INFINITY, ubl = -INFINITY, u1 = -INFINITY, u2 = -INFINITY;
      int jl = 0x7FFFFFFF, j1 = 0x7FFFFFFF, j2 = 0x7FFFFFFF;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t col = c0 + lane * kColsPerLane + q;
        if (col < pl.ncols) {
          const int j = pl.colmap ? pl.colmap[col] : (int)col;
          const float sc = a.scale[j];
          const float hq = hh[q] * sc, rq = acc[q] * sc;
          const float sf = (hh[q] + acc[q]) * sc;
          float E = fmaf(kh, hq, fmaf(ks, rq, 0x1p-24f * (hq + rq)));
          E = fmaf(E, 1.0f + 0x1p-20f, A);
          const float M = 0x1p-21f * (sf + E);
          const float lq = sf - E - M, uq = sf + E + M;
          if (better(lq, j, lb, jl)) {
            lb = lq;
            jl = j;
            ubl = uq;
          }
          ub_insert(uq, j, u1, j1, u2, j2);
        }
      }
      wave_bound_summary(lb, jl, ubl, u1, j1, u2, j2);
      if (lane == 0) {
        float4 *dst = reinterpret_cast<float4 *>(&part[c * a.n_rows + row]);
        dst[0] = make_float4(lb, __int_as_float(jl), ubl, __int_as_float(jl));
        dst[1] = make_float4(u1, __int_as_float(j1), u2, __int_as_float(j2));
      }
    } else {
      float b1 = -INFINITY, b2 = -INFINITY;
      int j1 = 0x7FFFFFFF;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t col = c0 + lane * kColsPerLane + q;
        if (col < pl.ncols) {
          const int j = pl.colmap ? pl.colmap[col] : (int)col;
          float s = acc[q];
          if (a.scale) s *= a.scale[j];
          if (better(s, j, b1, j1)) {
            b2 = b1;
            b1 = s;
            j1 = j;
          } else if (s > b2) {
            b2 = s;
          }
        }
      }
      wave_top2(b1, j1, b2);
      if (lane == 0) {
        // the first two entries only (16 bytes)
        float4 *dst = reinterpret_cast<float4 *>(&part[c * a.n_rows + row]);
        *dst = make_float4(b1, __int_as_float(j1), b2, __int_as_float(0x7FFFFFFF));
      }
    }
  }
}

// Sec. 3.1 with few changed centroids (n_ch <= 8 * NG <= kNarrowMax): a row
// whose previous centroid is unchanged scores only the compacted changed
// centroids, here without the head product.  One wavefront per row; lanes
// take the row's terms (all of them), each loading its term's n_ch codes from
// the compacted copy and accumulating them, and a butterfly over the wave
// adds the lane sums (any summation order is inside the bound).  Writes the
// row's partial of compacted chunk 0; rows whose previous centroid changed
// are left to the full pass.
template <int P, int NG>
__global__ __launch_bounds__(256) void k_score_narrow(ScoreArgs a, Partial *__restrict__ part) {
  using C = Codes<P>;
  const int lane = lane_id();
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.n_rows) return;
  const RowPlan pl = plan_row(a, row, true);
  if (!pl.ncc || pl.done) return;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(a.tile_ch), 0, (int)(a.D * kChunk * C::kBytes), 0x00020000);
  float acc[NG * 8];
#pragma unroll
  for (int c = 0; c < NG * 8; ++c) acc[c] = 0.f;
  const int64_t b = uniform64(a.indptr[row]), e = uniform64(a.indptr[row + 1]);
  for (int64_t q = b + lane; q < e; q += kWave) {
    const int t = a.indices[q];
    const float x = a.values[q];
    const int vo = t * (kChunk * C::kBytes);
    typename C::raw_t r[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) r[g] = C::load(rs, vo + g * 8 * C::kBytes, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) C::fma8(r[g], x, acc + 8 * g);
  }
#pragma unroll
  for (int c = 0; c < NG * 8; ++c) {
    float v = acc[c];
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
    acc[c] = v;
  }
  if (lane != 0) return;
  const int n_ch = a.n_ch;
  if (a.top == kTop) {
    // FP8 bound summary (every term from the FP8 codes)
    const int64_t n = e - b;
    const double ks = bound_kappa(n, a.uq), A = bound_abs(n, a.xl1[row], a.abs_coef);
    float lb = -INFINITY, ubl = -INFINITY, u1 = -INFINITY, u2 = -INFINITY;
    int jl = 0x7FFFFFFF, j1 = 0x7FFFFFFF, j2 = 0x7FFFFFFF;
#pragma unroll
    for (int c = 0; c < NG * 8; ++c) {
      if (c < n_ch) {
        const int j = a.ch_ids[c];
        const float sc = a.scale ? a.scale[j] : 1.f;
        const float sf = acc[c] * sc;
        const double E = bound_split(0.0, (double)sf, 0.0, ks, A);
        const float lq = f_down((double)sf - E), uq = f_up((double)sf + E);
        if (better(lq, j, lb, jl)) {
          lb = lq;
          jl = j;
          ubl = uq;
        }
        ub_insert(uq, j, u1, j1, u2, j2);
      }
    }
    Partial p;
    p.e[0].s = lb;
    p.e[0].j = jl;
    p.e[1].s = ubl;
    p.e[1].j = jl;
    p.e[2].s = u1;
    p.e[2].j = j1;
    p.e[3].s = u2;
    p.e[3].j = j2;
    part[row] = p;
  } else {
    float b1 = -INFINITY, b2 = -INFINITY;
    int j1 = 0x7FFFFFFF;
#pragma unroll
    for (int c = 0; c < NG * 8; ++c) {
      if (c < n_ch) {
        const int j = a.ch_ids[c];
        float s = acc[c];
        if (a.scale) s *= a.scale[j];
        if (better(s, j, b1, j1)) {
          b2 = b1;
          b1 = s;
          j1 = j;
        } else if (s > b2) {
          b2 = s;
        }
      }
    }
    *reinterpret_cast<float4 *>(&part[row]) =
        make_float4(b1, __int_as_float(j1), b2, __int_as_float(0x7FFFFFFF));
  }
}

// Merges a row's chunk partials in chunk order and certifies the winner:
// certain when the winner's lower bound exceeds every other candidate's upper
// bound; otherwise the row goes to the exact tier with L = the certified lower
// bound of the maximum.  One thread per row.
__global__ __launch_bounds__(256) void k_finalize(ScoreArgs a, const Partial *__restrict__ part) {
  __shared__ unsigned long long sh[4][256];
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n_rows = a.n_dev ? *a.n_dev : a.n_rows;
  unsigned long long n_cols = 0, n_prod = 0, n_ncc = 0, n_sp = 0;
  const RowPlan pl = row < n_rows ? plan_row(a, row, true) : RowPlan{};
  if (row < n_rows && !pl.done) {
    const int64_t b = a.indptr[row], e = a.indptr[row + 1];
    const int64_t n = e - b;
    const int64_t nch = (pl.ncols + kChunk - 1) / kChunk;
    int win;
    double wlo, whi, L;
    bool certain;
    if (a.top == kTop) {
      // FP8: the chunk summaries hold certified bounds.  The winner is the
      // column with the best lower bound; it is certain when that bound
      // exceeds every other column's upper bound.
      float lbw = -INFINITY, ubw = -INFINITY, g1 = -INFINITY, g2 = -INFINITY;
      int jw = 0x7FFFFFFF, gj1 = 0x7FFFFFFF, gj2 = 0x7FFFFFFF;
      for (int64_t c = 0; c < nch; ++c) {
        const Partial p = part[c * a.n_rows + row];
        if (better(p.e[0].s, p.e[0].j, lbw, jw)) {
          lbw = p.e[0].s;
          jw = p.e[0].j;
          ubw = p.e[1].s;
        }
        ub_insert(p.e[2].s, p.e[2].j, g1, gj1, g2, gj2);
        ub_insert(p.e[3].s, p.e[3].j, g1, gj1, g2, gj2);
      }
      const double other = gj1 != jw ? (double)g1 : (double)g2;   // best other upper bound
      if (!pl.ncc) {
        win = jw;
        wlo = lbw;
        whi = ubw;
        certain = (double)lbw > other;
        L = lbw;
      } else {
        const double plo = a.prev_lo[row], phi = a.prev_hi[row];
        if (nch == 0) {
          win = pl.ap;
          wlo = plo;
          whi = phi;
          certain = true;
          L = plo;
        } else if (plo >= (double)lbw) {
          win = pl.ap;
          wlo = plo;
          whi = phi;
          certain = plo > (double)g1;
          L = plo;
        } else {
          win = jw;
          wlo = lbw;
          whi = ubw;
          certain = (double)lbw > fmax(phi, other);
          L = lbw;
        }
      }
    } else {
      float b1 = -INFINITY, b2 = -INFINITY;
      int j1 = 0x7FFFFFFF;
      for (int64_t c = 0; c < nch; ++c) {
        const Partial p = part[c * a.n_rows + row];
        if (better(p.e[0].s, p.e[0].j, b1, j1)) {
          b2 = fmaxf(b1, p.e[1].s);
          b1 = p.e[0].s;
          j1 = p.e[0].j;
        } else {
          b2 = fmaxf(b2, p.e[0].s);
        }
      }
      double kap, A;
      part_bound(a, row, n, kap, A);
      auto lo_of = [&](float s) { return s == -INFINITY ? -INFINITY : (double)s - (kap * (double)s + A); };
      auto hi_of = [&](float s) { return s == -INFINITY ? -INFINITY : (double)s + (kap * (double)s + A); };
      if (!pl.ncc) {
        win = j1;
        wlo = lo_of(b1);
        whi = hi_of(b1);
        certain = wlo > hi_of(b2);
        L = wlo;
      } else {
        const double plo = a.prev_lo[row], phi = a.prev_hi[row];
        if (b1 == -INFINITY) {
          win = pl.ap;
          wlo = plo;
          whi = phi;
          certain = true;
          L = plo;
        } else if (plo >= lo_of(b1)) {
          win = pl.ap;
          wlo = plo;
          whi = phi;
          certain = plo > hi_of(b1);
          L = plo;
        } else {
          win = j1;
          wlo = lo_of(b1);
          whi = hi_of(b1);
          certain = wlo > fmax(phi, hi_of(b2));
          L = wlo;
        }
      }
    }
    n_cols = (unsigned long long)pl.ncols;
    n_prod = (unsigned long long)pl.ncols * (unsigned long long)n;
    n_ncc = pl.ncc ? 1ull : 0ull;
    if (a.head_H > 0)   // narrow NCC rows (no head product) scored every term
      n_sp = (unsigned long long)pl.ncols *
             (unsigned long long)(pl.ncc && pl.ncols <= kNarrowMax
                                      ? n
                                      : a.sc_indptr[row + 1] - a.sc_indptr[row]);
    if (certain || a.no_exact) {
      a.a_out[row] = win;
      a.lo_out[row] = wlo;
      a.hi_out[row] = whi;
    } else {
      const int f = atomicAdd(&a.counters[0], 1);
      a.flag_rows[f] = (int32_t)row;
      a.flag_L[f] = L;
      a.flag_mode[f] = pl.ncc ? 1 : 0;
    }
  }
  sh[0][threadIdx.x] = n_cols;
  sh[1][threadIdx.x] = n_prod;
  sh[2][threadIdx.x] = n_ncc;
  sh[3][threadIdx.x] = n_sp;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
      sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
      sh[3][threadIdx.x] += sh[3][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&a.stat[0], sh[0][0]);
    atomicAdd(&a.stat[3], sh[1][0]);
    if (sh[2][0]) atomicAdd(&a.stat[1], sh[2][0]);
    if (a.head_H > 0) atomicAdd(&a.stat[8], sh[3][0]);   // products of the sparse pass
  }
}

// Exact tier.  For each flagged row: first the FP64 scores of the
// low-precision winner (and, for an NCC row, of the previous centroid); the
// best of them, less its FP64 error, is a lower bound of the true maximum at
// least as high as the row's certified L and narrows the band.  Then recompute
// the low-precision scores, keep the band of candidates whose upper bound
// reaches that bound (every centroid that can be the true maximum) and decide
// among them in FP64 against the FP64 centroids (lowest index on ties).  The
// band is collected in LDS and scored whenever the buffer could overflow, so
// its size is not limited.
template <int P>
__global__ __launch_bounds__(256) void k_exact(ExactArgs x) {
  __shared__ int32_t band_all[4][kBandCap];
  __shared__ float lacc_all[4][kChunk];
  const ScoreArgs &a = x.s;
  const int wave = uniform32(threadIdx.x >> 6);
  const int lane = lane_id();
  int32_t *band = band_all[wave];
  float *lacc = lacc_all[wave];
  zero_lacc(lacc);
  const int32_t n_flag = uniform32(*(volatile int32_t *)&a.counters[0]);
  for (int64_t f = (int64_t)blockIdx.x * 4 + wave; f < n_flag; f += (int64_t)gridDim.x * 4) {
    const int64_t row = uniform64(a.flag_rows[f]);
    const bool ncc_row = a.flag_mode[f] == 1;
    const int64_t b = uniform64(a.indptr[row]);
    const int64_t e = uniform64(a.indptr[row + 1]);
    const int64_t n = e - b;
    RowPlan pl{a.tile, a.k, nullptr, false, -1, false, &a.tv};
    if (ncc_row) {
      pl.tv = &a.tv_ch;
      pl.tile = a.tile_ch;
      pl.ncols = a.n_ch;
      pl.colmap = a.ch_ids;
      pl.ncc = true;
      pl.ap = a.a_prev[row];
    }
    const int64_t nch = (pl.ncols + kChunk - 1) / kChunk;
    // seeds: the merged low-precision winner and the previous centroid
    float w1 = -INFINITY;
    int wj = 0x7FFFFFFF;
    for (int64_t c = 0; c < nch; ++c) {
      const Partial p = x.part[c * a.n_rows + row];
      if (better(p.e[0].s, p.e[0].j, w1, wj)) {
        w1 = p.e[0].s;
        wj = p.e[0].j;
      }
    }
    // (each seed's FP64 dot product by the whole wavefront, lanes over terms)
    double bs = -INFINITY;
    int bj = 0x7FFFFFFF;
    double L = a.flag_L[f];
    for (int q = 0; q < 2; ++q) {
      const int seed = q == 0 ? (w1 == -INFINITY ? -1 : wj) : (pl.ncc ? pl.ap : -1);
      if (seed < 0) continue;
      const double *crow = x.master + (int64_t)seed * x.D;
      double t = 0.0;
      for (int64_t k = b + lane; k < e; k += kWave) t = fma((double)a.values[k], crow[a.indices[k]], t);
      t = wave_sum_d(t);
      L = fmax(L, t - exact_err(n, t));
      if (lane == q && better_d(t, seed, bs, bj)) {
        bs = t;
        bj = seed;
      }
    }
    // bound of the rescoring below (all terms, sparse path)
    const double kap = bound_kappa(n, a.uq);
    const double A = bound_abs(n, a.xl1[row], a.abs_coef);
    // bound of the partials of the scoring pass
    double pkap, pA;
    part_bound(a, row, n, pkap, pA);
    auto phi_of = [&](float s) {
      return s == -INFINITY ? -INFINITY : (double)s + (pkap * (double)s + pA);
    };
    int nb = 0;           // members in the buffer
    int64_t total = 0;    // band size
    auto flush = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int i = lane; i < nb; i += kWave) {
        const int j = band[i];
        const double s = dot64(b, e, a.indices, a.values, x.master + (int64_t)j * x.D);
        if (better_d(s, j, bs, bj)) {
          bs = s;
          bj = j;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      total += nb;
      nb = 0;
    };
    for (int64_t c0 = 0; c0 < pl.ncols; c0 += kChunk) {
      if (nb + kChunk > kBandCap) flush();
      // A chunk whose kept entries show that at most one column can reach L
      // contributes that column without being rescored: with two kept
      // scores, when the second one's upper bound misses L; with FP8 bound
      // summaries, when the second largest upper bound misses L (every
      // column but the one with the largest lies at or below it).
      const Partial p = x.part[(c0 / kChunk) * a.n_rows + row];
      if (a.top == kTop) {
        if ((double)p.e[3].s < L) {
          if ((double)p.e[2].s >= L) {
            if (lane == 0) band[nb] = p.e[2].j;
            nb += 1;
          }
          continue;
        }
      } else if (phi_of(p.e[1].s) < L) {
        if (phi_of(p.e[0].s) >= L) {
          if (lane == 0) band[nb] = p.e[0].j;
          nb += 1;
        }
        continue;
      }
      float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      score_chunk<P>(b, e, a.indices, a.values, pl.tile, a.D, c0, pl.ncols - c0, acc, *pl.tv, lacc);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int64_t col = c0 + lane * kColsPerLane + c;
        bool in = false;
        int j = 0;
        if (col < pl.ncols) {
          j = pl.colmap ? pl.colmap[col] : (int)col;
          double s = acc[c];
          if (a.scale) s *= (double)a.scale[j];
          in = s + (kap * s + A) >= L;
        }
        const uint64_t m = __ballot(in);
        if (in) band[nb + __popcll(m & lanemask_lt())] = j;
        nb += __popcll(m);
      }
    }
    flush();
    wave_best_d(bs, bj);
    if (lane == 0) {
      const double err = exact_err(n, bs);
      a.a_out[row] = bj;
      a.lo_out[row] = bs - err;
      a.hi_out[row] = bs + err;
      if (total > kBandCap) atomicAdd(&a.counters[1], 1);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Dense low-precision score matrix (diagnostic): one wave per row.
template <int P>
__global__ __launch_bounds__(256) void k_score_dense(const int64_t *indptr, const int32_t *indices,
                                                     const float *values, int64_t n_rows,
                                                     const uint8_t *tile, int64_t D, int32_t k,
                                                     const float *scale, TailView tv,
                                                     const float *hs, int64_t hs_ld, float *out,
                                                     float *out_head) {
  __shared__ float lacc_all[4][kChunk];
  const int wave = uniform32(threadIdx.x >> 6);
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= n_rows) return;
  const int lane = lane_id();
  float *lacc = lacc_all[wave];
  zero_lacc(lacc);
  const int64_t b = uniform64(indptr[row]);
  const int64_t e = uniform64(indptr[row + 1]);
  for (int64_t c0 = 0; c0 < k; c0 += kChunk) {
    // the head scores and the sparse terms combined as the scoring kernel
    // does: added onto the head scores (FP32 / BF16), or summed apart and
    // added once (FP8)
    constexpr bool kSplit = P == SKM_FP8_E4M3;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float hh[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (hs) {
#pragma unroll
      for (int c = 0; c < 8; ++c) hh[c] = hs[row * hs_ld + c0 + lane * kColsPerLane + c];
      if constexpr (!kSplit) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = hh[c];
      }
    }
    score_chunk<P>(b, e, indices, values, tile, D, c0, k - c0, acc, tv, lacc);
    for (int c = 0; c < 8; ++c) {
      const int64_t col = c0 + lane * kColsPerLane + c;
      if (col < k) {
        const float sc = scale ? scale[col] : 1.f;
        out[row * k + col] = (kSplit ? hh[c] + acc[c] : acc[c]) * sc;
        if (out_head) out_head[row * k + col] = hh[c] * sc;
      }
    }
  }
}

// FP64 dot product of each row with its assigned centroid: one wave per row,
// lanes over terms, fixed-shape wave sum.
__global__ __launch_bounds__(256) void k_exact_scores(const int64_t *indptr, const int32_t *indices,
                                                      const float *values, int64_t n_rows,
                                                      const int64_t *n_dev, const int32_t *asg,
                                                      const double *master, int64_t D,
                                                      double *out) {
  const int wave = uniform32(threadIdx.x >> 6);
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= (n_dev ? *n_dev : n_rows)) return;
  const int lane = lane_id();
  const int64_t b = indptr[row], e = indptr[row + 1];
  const double *c = master + (int64_t)asg[row] * D;
  double s = 0.0;
  for (int64_t q = b + lane; q < e; q += kWave) s = fma((double)values[q], c[indices[q]], s);
  s = wave_sum_d(s);
  if (lane == 0) out[row] = s;
}

// Workgroups of k_score_part<P> resident per CU at its register and LDS use.
template <int P>
int occupancy_t() {
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_score_part<P>, 256, 0) != hipSuccess ||
        n <= 0)
      n = 4;
    (void)hipGetLastError();
    return n;
  }();
  return per_cu;
}

template <int P>
hipError_t launch_score_part_t(const ScoreArgs &a, Partial *part, int n_cu, int wpc, hipStream_t s) {
  if (a.n_rows <= 0) return hipSuccess;
  // By default the persistent grid is exactly one wave of resident
  // workgroups, so no workgroup starts late and sweeps the chunks out of step
  // with the rest; wpc > 0 overrides the workgroups per CU (autotuning).
  const int per_cu = wpc > 0 ? wpc : occupancy_t<P>();
  // with a device row count, nb is the capacity the grid is sized for
  const int64_t n_items = (int64_t)a.c_count * a.nb;
  const int64_t need = (n_items + 3) / 4;
  if (need <= 0) return hipSuccess;
  const int g = (int)std::min<int64_t>((int64_t)n_cu * per_cu, need);
  hipLaunchKernelGGL(k_score_part<P>, dim3((unsigned)g), dim3(256), 0, s, a, part, n_items);
  return hipGetLastError();
}

template <int P>
hipError_t launch_exact_t(const ExactArgs &x, hipStream_t s) {
  hipLaunchKernelGGL(k_exact<P>, dim3((unsigned)x.max_waves / 4), dim3(256), 0, s, x);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_score_part(const ScoreArgs &a, Partial *part, int n_cu, int prec, hipStream_t s,
                             int wpc) {
  switch (prec) {
    case SKM_FP32: return launch_score_part_t<SKM_FP32>(a, part, n_cu, wpc, s);
    case SKM_BF16: return launch_score_part_t<SKM_BF16>(a, part, n_cu, wpc, s);
    case SKM_FP8_E4M3: return launch_score_part_t<SKM_FP8_E4M3>(a, part, n_cu, wpc, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
hipError_t launch_score_narrow_t(const ScoreArgs &a, Partial *part, hipStream_t s) {
  const dim3 g((unsigned)((a.n_rows + 3) / 4)), b(256);
  if (a.n_ch <= 8) {
    hipLaunchKernelGGL((k_score_narrow<P, 1>), g, b, 0, s, a, part);
  } else if (a.n_ch <= 16) {
    hipLaunchKernelGGL((k_score_narrow<P, 2>), g, b, 0, s, a, part);
  } else if (a.n_ch <= 32) {
    hipLaunchKernelGGL((k_score_narrow<P, 4>), g, b, 0, s, a, part);
  } else {
    hipLaunchKernelGGL((k_score_narrow<P, 8>), g, b, 0, s, a, part);
  }
  return hipGetLastError();
}

hipError_t launch_score_narrow(const ScoreArgs &a, Partial *part, int prec, hipStream_t s) {
  if (a.n_rows <= 0 || a.n_ch <= 0) return hipSuccess;
  if (a.n_ch > kNarrowMax || !a.tile_ch || !a.ch_ids || !a.a_prev || !a.changed ||
      a.D * kChunk * 4 > INT32_MAX)
    return hipErrorInvalidValue;
  switch (prec) {
    case SKM_FP32: return launch_score_narrow_t<SKM_FP32>(a, part, s);
    case SKM_BF16: return launch_score_narrow_t<SKM_BF16>(a, part, s);
    case SKM_FP8_E4M3: return launch_score_narrow_t<SKM_FP8_E4M3>(a, part, s);
  }
  return hipErrorInvalidValue;
}

int score_occupancy(int prec) {
  switch (prec) {
    case SKM_FP32: return occupancy_t<SKM_FP32>();
    case SKM_BF16: return occupancy_t<SKM_BF16>();
    default: return occupancy_t<SKM_FP8_E4M3>();
  }
}

hipError_t launch_finalize(const ScoreArgs &a, const Partial *part, hipStream_t s) {
  if (a.n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((a.n_rows + 255) / 256)), dim3(256), 0, s, a, part);
  return hipGetLastError();
}

hipError_t launch_score(const ScoreArgs &a, Partial *part, int n_cu, int prec, hipStream_t s,
                        int wpc) {
  hipError_t e = launch_score_part(a, part, n_cu, prec, s, wpc);
  if (e != hipSuccess) return e;
  return launch_finalize(a, part, s);
}

hipError_t launch_exact(const ExactArgs &x, int prec, hipStream_t s) {
  switch (prec) {
    case SKM_FP32: return launch_exact_t<SKM_FP32>(x, s);
    case SKM_BF16: return launch_exact_t<SKM_BF16>(x, s);
    case SKM_FP8_E4M3: return launch_exact_t<SKM_FP8_E4M3>(x, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_score_dense(const int64_t *indptr, const int32_t *indices, const float *values,
                              int64_t n_rows, const uint8_t *tile, int64_t D, int32_t k,
                              const float *scale, const TailView &tv, int prec, const float *hs,
                              int64_t hs_ld, float *out, hipStream_t s, float *out_head) {
  if (n_rows <= 0) return hipSuccess;
  const dim3 g((unsigned)((n_rows + 3) / 4)), blk(256);
  switch (prec) {
    case SKM_FP32:
      hipLaunchKernelGGL(k_score_dense<SKM_FP32>, g, blk, 0, s, indptr, indices, values, n_rows, tile,
                         D, k, nullptr, tv, hs, hs_ld, out, out_head);
      break;
    case SKM_BF16:
      hipLaunchKernelGGL(k_score_dense<SKM_BF16>, g, blk, 0, s, indptr, indices, values, n_rows, tile,
                         D, k, nullptr, tv, hs, hs_ld, out, out_head);
      break;
    case SKM_FP8_E4M3:
      hipLaunchKernelGGL(k_score_dense<SKM_FP8_E4M3>, g, blk, 0, s, indptr, indices, values, n_rows,
                         tile, D, k, scale, tv, hs, hs_ld, out, out_head);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_exact_scores(const int64_t *indptr, const int32_t *indices, const float *values,
                               int64_t n_rows, const int32_t *asg, const double *master, int64_t D,
                               double *out, hipStream_t s, const int64_t *n_dev) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exact_scores, dim3((unsigned)((n_rows + 3) / 4)), dim3(256), 0, s, indptr,
                     indices, values, n_rows, n_dev, asg, master, D, out);
  return hipGetLastError();
}

}  // namespace skm
