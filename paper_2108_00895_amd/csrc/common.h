// Device helpers shared by the kernels of libskm: wavefront primitives, the
// scoring-copy encodings and the certified error bound.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "../../include/skm.h"

namespace skm {

constexpr int kWave = 64;
constexpr int kColsPerLane = 8;
constexpr int kChunk = kWave * kColsPerLane;  // centroid columns per wave pass
constexpr int kBandCap = 1024;                // exact-tier band buffer in LDS per wave (>= 2 chunks)

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Scoring copies are blocked by 512-centroid chunks: chunk c is a contiguous
// [D][512] slab, so one chunk's term rows are consecutive 512-code pieces.  A
// plain [D][k] layout would put a chunk's pieces at a stride of k codes, which
// for the k of interest is a multiple of 4 KiB and folds every piece of a
// chunk onto the same few L2 channels and sets.
__host__ __device__ inline int64_t tile_index(int64_t t, int64_t j, int64_t D) {
  return ((j / kChunk) * D + t) * kChunk + (j % kChunk);
}

// ---------------------------------------------------------------- wave helpers

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ inline uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ inline double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, kWave);
}

// Lexicographic "better": higher score, then lower index.
__device__ inline bool better(float s, int j, float bs, int bj) {
  return s > bs || (s == bs && j < bj);
}
__device__ inline bool better_d(double s, int j, double bs, int bj) {
  return s > bs || (s == bs && j < bj);
}

// Merges (b1, j1, b2) top-two summaries across the wave; every lane ends with
// the wave's result.  b2 is the best score among all candidates other than j1.
__device__ inline void wave_top2(float &b1, int &j1, float &b2) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) {
    float o1 = __shfl_xor(b1, m, kWave);
    int oj = __shfl_xor(j1, m, kWave);
    float o2 = __shfl_xor(b2, m, kWave);
    if (better(o1, oj, b1, j1)) {
      b2 = fmaxf(b1, o2);
      b1 = o1;
      j1 = oj;
    } else {
      b2 = fmaxf(b2, o1);
    }
  }
}

// FP8 chunk summaries kept as certified bounds: the column with the best
// lower bound (ties: lower index) with its upper bound, and the two largest
// upper bounds (ties: lower index) with their columns.
__device__ inline void ub_insert(float u, int j, float &u1, int &j1, float &u2, int &j2) {
  // selects only (branches on the references make the compiler spill them)
  const bool f = better(u, j, u1, j1), g = better(u, j, u2, j2);
  const float nu2 = f ? u1 : (g ? u : u2);
  const int nj2 = f ? j1 : (g ? j : j2);
  u1 = f ? u : u1;
  j1 = f ? j : j1;
  u2 = nu2;
  j2 = nj2;
}

// Butterfly merge of bound summaries (the two halves hold disjoint columns);
// every lane ends with the wave's summary.
__device__ inline void wave_bound_summary(float &lb, int &jl, float &ubl, float &u1, int &j1,
                                          float &u2, int &j2) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) {
    const float olb = __shfl_xor(lb, m, kWave), oubl = __shfl_xor(ubl, m, kWave);
    const int ojl = __shfl_xor(jl, m, kWave);
    const float ou1 = __shfl_xor(u1, m, kWave), ou2 = __shfl_xor(u2, m, kWave);
    const int oj1 = __shfl_xor(j1, m, kWave), oj2 = __shfl_xor(j2, m, kWave);
    if (better(olb, ojl, lb, jl)) {
      lb = olb;
      jl = ojl;
      ubl = oubl;
    }
    ub_insert(ou1, oj1, u1, j1, u2, j2);
    ub_insert(ou2, oj2, u1, j1, u2, j2);
  }
}

// Float bounds that keep a double bound's direction: the largest float <= x,
// the smallest float >= x.
__device__ inline float f_down(double x) {
  const float f = (float)x;
  return (double)f > x ? nextafterf(f, -INFINITY) : f;
}
__device__ inline float f_up(double x) {
  const float f = (float)x;
  return (double)f < x ? nextafterf(f, INFINITY) : f;
}

__device__ inline void wave_best_d(double &s, int &j) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) {
    double os = shfl_xor_d(s, m);
    int oj = __shfl_xor(j, m, kWave);
    if (better_d(os, oj, s, j)) {
      s = os;
      j = oj;
    }
  }
}

// FP64 dot product of a row with one centroid row, by one lane: eight
// interleaved partial sums (fixed order) so that eight gathers are in flight.
__device__ inline double dot64(int64_t b, int64_t e, const int32_t *__restrict__ indices,
                               const float *__restrict__ values, const double *__restrict__ crow) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t q = b;
  for (; q + 8 <= e; q += 8) {
    double c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = crow[indices[q + u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] = fma((double)values[q + u], c[u], s[u]);
  }
  for (; q < e; ++q) s[0] = fma((double)values[q], crow[indices[q]], s[0]);
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += shfl_xor_d(v, m);
  return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// ------------------------------------------------------- scoring-copy encodings
// All conversions start from the FP64 centroid value and round once, to nearest
// with ties to even.  Centroid values are >= 0.

// bfloat16: 8 significant bits, binary32's exponent range.
__host__ __device__ inline uint16_t encode_bf16(double c) {
  if (!(c > 0.0)) return 0;
  if (c < 0x1p-126) {                       // subnormal: spacing 2^-133
    double m = rint(ldexp(c, 133));
    return (uint16_t)m;                     // m == 128 encodes 2^-126 correctly
  }
  int ex;
  double m = frexp(c, &ex);                 // c = m * 2^ex, m in [0.5, 1)
  double q = rint(m * 256.0);               // 8 significant bits
  if (q == 256.0) {
    q = 128.0;
    ex += 1;
  }
  int e_field = ex - 1 + 127;
  if (e_field >= 255) return 0x7F80;        // overflow to +inf (not reached: c <= 1)
  return (uint16_t)((e_field << 7) | ((int)q - 128));
}

// FP8 E4M3 (OCP): bias 7, 3 mantissa bits, max 448, subnormal spacing 2^-9.
// v must already be divided by the centroid's power-of-two scale.
__host__ __device__ inline uint8_t encode_e4m3(double v) {
  if (!(v > 0.0)) return 0;
  if (v < 0x1p-6) {
    double m = rint(v * 512.0);             // m == 8 encodes 2^-6 correctly
    return (uint8_t)m;
  }
  int ex;
  double m = frexp(v, &ex);
  double q = rint(m * 16.0);                // 4 significant bits
  if (q == 16.0) {
    q = 8.0;
    ex += 1;
  }
  int e_field = ex - 1 + 7;
  int code = (e_field << 3) | ((int)q - 8);
  return (uint8_t)(code > 0x7E ? 0x7E : code);   // saturate at 448
}

// Least e with cmax <= 448 * 2^e (0 for cmax == 0).
__host__ __device__ inline int e4m3_scale_exp(double cmax) {
  if (!(cmax > 0.0)) return 0;
  int e;
  frexp(cmax / 448.0, &e);
  e += 1;
  while (cmax <= ldexp(448.0, e - 1)) e -= 1;
  while (cmax > ldexp(448.0, e)) e += 1;
  return e;
}

// ------------------------------------------------------------- error bound
// A low-precision score s^ = fl32(sum_t x_t * c^_t) of a row with n terms,
// where |c^_t - c_t| <= u_q * c_t + a (a: absolute term of the encoding, scaled),
// and the FP32 sum runs in at most 2n + 2 roundings (fused multiply-adds on the
// dense path, a rounded product plus an add on the list path, one final merge):
//   |s^ - S^| <= g_m * S^,   g_m = m u / (1 - m u), m = 2n + 2, u = 2^-24
//   |S^ - s|  <= u_q * s + a * ||x||_1
// which gives |s^ - s| <= kappa * s^ + A with
//   kappa = (g_m + u_q / (1 - u_q)) / (1 - g_m),  A = a ||x||_1 / (1 - u_q).
// Both are inflated slightly so the FP64 evaluation of the test stays safe.
__host__ __device__ inline double bound_kappa(int64_t n, double uq) {
  const double u = 0x1p-24;
  // each term costs at most two roundings (a product rounded before an LDS
  // add on the list path), plus the final merge of the two partial sums
  double nn = 2.0 * (double)(n > 0 ? n : 1) + 2.0;
  double g = nn * u / (1.0 - nn * u);
  double k = (g + uq / (1.0 - uq)) / (1.0 - g);
  return k * (1.0 + 0x1p-20) + 0x1p-60;
}

// The same bound when the first part of the score came from the head product
// (kernels_head.hip): H head terms with the row values rounded to BF16 (unit
// 2^-8) and summed on the matrix cores, each of whose accumulation steps is
// counted as two roundings; the sum then joins the sparse path's chain.  Every
// product sees at most 2n + 2H + 4 roundings, and its inputs carry the
// combined unit u' = u_x + u_q + u_x u_q.
__host__ __device__ inline double bound_kappa_head(int64_t n, int64_t H, double uq) {
  const double u = 0x1p-24, ux = 0x1p-8;
  const double up = ux + uq + ux * uq;
  double nn = 2.0 * (double)(n > 0 ? n : 1) + 2.0 * (double)H + 4.0;
  double g = nn * u / (1.0 - nn * u);
  double k = (g + up / (1.0 - up)) / (1.0 - g);
  return k * (1.0 + 0x1p-20) + 0x1p-60;
}

// Relative bound of a head sum alone when the head codes are BF16 roundings of
// the FP64 master (FP8 scoring copies): H products of BF16 row values and
// BF16 codes (combined unit 2^-8 + 2^-8 + 2^-16), each accumulation step on the
// matrix cores counted as two roundings.
__host__ __device__ inline double bound_kappa_head_bf16(int64_t H) {
  const double u = 0x1p-24, up = 0x1p-8 + 0x1p-8 + 0x1p-16;
  double nn = 2.0 * (double)(H > 0 ? H : 1) + 4.0;
  double g = nn * u / (1.0 - nn * u);
  double k = (g + up / (1.0 - up)) / (1.0 - g);
  return k * (1.0 + 0x1p-20) + 0x1p-60;
}

// Bound on an FP8 score whose head part hs and sparse part rs (both >= 0, in
// score units) were summed separately and added once:
//   |s^ - s| <= kh hs + ks rs + 2^-24 (hs + rs) + A,
// kh from bound_kappa_head_bf16, ks and A those of the n_s sparse terms, plus
// the matrix cores' flush term.
__host__ __device__ inline double bound_split(double hs, double rs, double kh, double ks,
                                              double A) {
  return (kh * hs + ks * rs + 0x1p-24 * (hs + rs)) * (1.0 + 0x1p-20) + A;
}

// Absolute part for head scores: the encoding term grows with the rounded row
// values (|x^| <= x (1 + 2^-8)), and values or partial sums below 2^-126 that
// the matrix cores flush cost at most 2^-126 per head step.
__host__ __device__ inline double bound_abs_head(int64_t H, double l1, double abs_coef) {
  return abs_coef * l1 * 0x1p-7 + (double)H * 0x1p-120;
}

__host__ __device__ inline double bound_abs(int64_t n, double l1, double abs_coef) {
  return abs_coef * l1 + (double)(n > 0 ? n : 1) * 0x1p-140;
}

// Bound on |fl64(sum_t x_t c_t) - s| for the FP64 rescoring (n products).
__host__ __device__ inline double exact_err(int64_t n, double s) {
  double nn = (double)(n > 0 ? n : 1) + 2.0;
  return nn * 0x1p-52 * fabs(s) + 0x1p-1000;
}

}  // namespace skm
