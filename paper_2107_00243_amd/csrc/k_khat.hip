// Matrix-free W = K_hat V with kernel tiles built on the fly (the product inside
// every CG iteration; Section 4.4 and its complexity paragraph: O(n^2) per
// product, never storing K_hat).
//
// Each workgroup owns 64*RG rows (four waves of 16*RG rows) and streams one column
// range (split-K) in steps of 32 columns.  Per step and per 16 x 16 sub-tile:
//   1. MFMA distance product in the transposed orientation, D[j][i] = x'_j . x'_i,
//      accumulated on top of the per-row term (C operand) -> the lane holding
//      column i of D owns 4 consecutive j of that row i;
//   2. the kernel map in registers (exp2 of the log2-domain argument for RBF,
//      sqrt/exp2/polynomial for Matern), the exact diagonal on diagonal tiles;
//   3. those 4 + 4 values are exactly one row-slice of the A operand of the
//      second MFMA (tile x V) under a fixed permutation of the 32 contraction
//      indices, which the staged V fragments share.
// Operands are pre-arranged "fragment-major" in global memory so that every LDS
// read is one contiguous 16-byte (or 4/8-byte) slot per lane.
//
// Precisions: BF16X3 splits every operand into bf16 hi + lo; the distance uses
// the (hi, hi, lo, lo) x (hi, lo, hi, lo) K-concatenation (all four cross
// products), the tile x V product the three products hi.hi + hi.lo + lo.hi, all
// with FP32 accumulation.  FP32 uses v_mfma_f32_16x16x4_f32, FP64 uses
// v_mfma_f64_16x16x4_f64.
#include "gpmll_impl.h"

#include <algorithm>

#ifndef GPMLL_KHAT_PART
#define GPMLL_KHAT_PART 0
#endif

namespace gpmll {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr float kLog2e = 1.4426950408889634f;

// Row (within a 16-row block) of accumulator slot v in lane group g = lane/16 for
// the 16x16x4 MFMA outputs: FP32 holds rows 4g + v, FP64 holds rows g + 4v.
template <typename T>
__device__ __host__ constexpr int acc_row(int g, int v) {
  return sizeof(T) == 8 ? g + 4 * v : 4 * g + v;
}

__device__ inline uint32_t pack_bf16(float a, float b) {
  f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// hi = RNE(a), lo = RNE(a - hi) for a pair; returns packed hi and lo words
__device__ inline void split_pair(float a, float b, uint32_t* hi, uint32_t* lo) {
  uint32_t h = pack_bf16(a, b);
  float ha = __builtin_bit_cast(float, h << 16);
  float hb = __builtin_bit_cast(float, h & 0xffff0000u);
  *hi = h;
  *lo = pack_bf16(a - ha, b - hb);
}

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint32_t pack_f16(float a, float b) {
  f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}

// FP16 split of a pair: hi = RNE(a), lo = RNE(a - hi)
__device__ inline void split_pair_f16(float a, float b, uint32_t* hi, uint32_t* lo) {
  const uint32_t h = pack_f16(a, b);
  const f32x2 hf = __builtin_convertvector(__builtin_bit_cast(f16x2, h), f32x2);
  *hi = h;
  *lo = pack_f16(a - hf[0], b - hf[1]);
}

__device__ inline float bf16_lo_f(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ inline float bf16_hi_f(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

// kernel value of the split-precision tiles from the MFMA argument q: RBF
// q = log2 k; Matern q = rho^2 with rho = a log2(e) r (a = sqrt3, sqrt5), so
// exp(-a r) = exp2(-rho) and a r = ln2 rho:
//   3/2: s (1 + ln2 rho) exp2(-rho),  5/2: s (1 + ln2 rho + (ln2 rho)^2 / 3) exp2(-rho)
// (|q| guards the rounding of q = 0 to a tiny negative number).  Rational
// quadratic: q = r^2 / (2 alpha) (x staged times 1/sqrt(alpha)), s (1 + q)^-alpha.
template <int KIND>
__device__ inline float map_split(float q, float s, float alpha) {
  if (KIND == GP_KERNEL_RBF) {
    return __builtin_amdgcn_exp2f(q);
  } else if (KIND == GP_KERNEL_RATQUAD) {
    return s * __builtin_amdgcn_exp2f(-alpha * __builtin_amdgcn_logf(1.0f + fabsf(q)));
  } else {
    const float ln2 = 0.6931471805599453f;
    const float rho = __builtin_amdgcn_sqrtf(fabsf(q));
    const float e = __builtin_amdgcn_exp2f(-rho);
    float poly;
    if (KIND == GP_KERNEL_MATERN32) poly = fmaf(s * ln2, rho, s);
    else poly = fmaf(fmaf(s * (ln2 * ln2 / 3.0f), rho, s * ln2), rho, s);
    return poly * e;
  }
}

// kernel value from the MFMA argument q (FP32 tiles): RBF q = log2 k; otherwise q = r^2
template <int KIND>
__device__ inline float map32(float q, float s, float alpha) {
  if (KIND == GP_KERNEL_RBF) {
    return __builtin_amdgcn_exp2f(q);
  } else if (KIND == GP_KERNEL_RATQUAD) {
    return s * __builtin_amdgcn_exp2f(-alpha * __builtin_amdgcn_logf(fmaf(fmaxf(q, 0.0f), 0.5f / alpha, 1.0f)));
  } else if (KIND == GP_KERNEL_MATERN32) {
    const float a = 1.7320508075688772f;
    float r = __builtin_amdgcn_sqrtf(fmaxf(q, 0.0f));
    float e = __builtin_amdgcn_exp2f(-a * kLog2e * r);
    return s * fmaf(a, r, 1.0f) * e;
  } else {
    const float a = 2.23606797749979f;
    float q0 = fmaxf(q, 0.0f);
    float r = __builtin_amdgcn_sqrtf(q0);
    float e = __builtin_amdgcn_exp2f(-a * kLog2e * r);
    return s * fmaf(5.0f / 3.0f, q0, fmaf(a, r, 1.0f)) * e;
  }
}

template <int KIND>
__device__ inline double map64(double q, double s, double alpha) {
  q = q > 0.0 ? q : 0.0;
  return s * kappa64(KIND, q, alpha);
}

// ---------------------------------------------------------------------------
// Tile kernels
// ---------------------------------------------------------------------------

struct TileArgs {
  int64_t n_pad;
  int64_t n_valid;          // rows/columns >= n_valid carry zero operands
  int64_t cols_per_split;   // multiple of 32
  int tp;                   // leading dimension of the partial output
  int ntt;                  // 16-column tiles of right-hand sides staged for this launch
  int xc;                   // split precisions: 1 = one more column on the vector ALU
  int vp;                   // BF16x3: pieces of the staged search directions (2 or 3)
  float s32;
  double s64;
  float alpha32;            // rational quadratic shape
  double alpha64;
};

// cooperative copy of `count` 16-byte units from three contiguous sources into LDS
__device__ inline void copy_units(u32x4* dst, const u32x4* a, int na, const u32x4* b, int nb, const u32x4* c,
                                  int nc, int tid, int nthreads) {
  const int total = na + nb + nc;
  for (int e = tid; e < total; e += nthreads) {
    u32x4 v;
    if (e < na) v = a[e];
    else if (e < na + nb) v = b[e - na];
    else v = c[e - na - nb];
    dst[e] = v;
  }
}

#if GPMLL_KHAT_PART == 0
// ---------------------------------------------------------------------------
// Staging of the inputs x~ into the MFMA fragment layouts, and the row and
// column terms of the distance expansion.  RBF: x' = sqrt(log2 e) x~ on both
// sides, q = x'_i.x'_j - |x'_i|^2/2 - |x'_j|^2/2 + log2 s = log2 k.  Matern:
// x'_B = sqrt2 x~, x'_A = -x'_B, q = |x'_i|^2/2 + |x'_j|^2/2 - x'_i.x'_j = r^2;
// the split-precision tiles stage x' = sqrt2 a log2(e) x~ instead (a = sqrt3 or
// sqrt5), so that sqrt(q) = a log2(e) r is directly the exponent of exp2.
// FP64 and the derivative sweep: as Matern, q = r^2.  Norms are those of the
// represented (rounded) operands, so q is a true squared distance of slightly
// perturbed points.
// ---------------------------------------------------------------------------

// rbf_add: added to the RBF row term (log2 s for BF16X3 tiles; 15 for FP16X3 tiles,
// whose kernel values are 2^15 kappa)
__global__ void k_stage_x_bf16(const double* __restrict__ xs, int64_t n_pad, int d, int dq, int nkc, int kind,
                               double alpha, float rbf_add, u32x4* __restrict__ xfa, u32x4* __restrict__ xfb,
                               float* __restrict__ rowterm, float* __restrict__ colterm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  const bool rbf = kind == GP_KERNEL_RBF;
  // RBF: sqrt(log2 e); Matern: sqrt2 * a * log2 e with a = sqrt3 (3/2) or sqrt5 (5/2);
  // rational quadratic: 1/sqrt(alpha), so that q = r^2 / (2 alpha)
  const double scale = rbf ? 1.2011224087864498
                           : (kind == GP_KERNEL_RATQUAD
                                  ? 1.0 / sqrt(alpha)
                                  : 1.4142135623730951 * 1.4426950408889634 *
                                        (kind == GP_KERNEL_MATERN32 ? 1.7320508075688772 : 2.23606797749979));
  uint16_t hi[GP_MAX_D], lo[GP_MAX_D];
  double nrm = 0.0;
  for (int q = 0; q < dq; ++q) {
    float x = q < d ? (float)(scale * xs[i * d + q]) : 0.0f;
    uint32_t h, l;
    split_pair(x, 0.0f, &h, &l);
    hi[q] = (uint16_t)(h & 0xffffu);
    lo[q] = (uint16_t)(l & 0xffffu);
    double rep = (double)bf16_lo_f(hi[q]) + (double)bf16_lo_f(lo[q]);
    nrm += rep * rep;
  }
  const uint16_t sgn = rbf ? 0 : 0x8000;
  const int kd = nkc * 32;
  const int64_t tile = i / 16;
  const int li = (int)(i % 16);
  for (int kc = 0; kc < nkc; ++kc) {
    for (int g = 0; g < 4; ++g) {
      uint32_t wa[4], wb[4];
      for (int w = 0; w < 4; ++w) {
        uint16_t ea[2], eb[2];
        for (int h2 = 0; h2 < 2; ++h2) {
          int k = kc * 32 + g * 8 + w * 2 + h2;
          int seg = k / dq, q = k % dq;
          ea[h2] = eb[h2] = 0;
          if (k < 4 * dq && k < kd) {
            // A side: [hi | hi | lo | lo], B side: [hi | lo | hi | lo]
            uint16_t va = (seg < 2) ? hi[q] : lo[q];
            uint16_t vb = (seg % 2 == 0) ? hi[q] : lo[q];
            ea[h2] = (va & 0x7fff) == 0 ? 0 : (uint16_t)(va ^ sgn);
            eb[h2] = vb;
          }
        }
        wa[w] = (uint32_t)ea[0] | ((uint32_t)ea[1] << 16);
        wb[w] = (uint32_t)eb[0] | ((uint32_t)eb[1] << 16);
      }
      const int64_t slot = (tile * nkc + kc) * 64 + li + 16 * g;
      xfa[slot] = u32x4{wa[0], wa[1], wa[2], wa[3]};
      xfb[slot] = u32x4{wb[0], wb[1], wb[2], wb[3]};
    }
  }
  if (rbf) {
    rowterm[i] = (float)(-0.5 * nrm + (double)rbf_add);
    colterm[i] = (float)(-0.5 * nrm);
  } else {
    rowterm[i] = (float)(0.5 * nrm);
    colterm[i] = (float)(0.5 * nrm);
  }
}

// log2form: RBF in the log2 domain (FP32 forward tiles); otherwise q = r^2
template <typename T>
__global__ void k_stage_x_fp(const double* __restrict__ xs, int64_t n_pad, int d, int nk4, int log2form,
                             double log2s, T* __restrict__ xfa, T* __restrict__ xfb, T* __restrict__ rowterm,
                             T* __restrict__ colterm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  const bool rbf32 = log2form != 0;
  const double scale = rbf32 ? 1.2011224087864498 : 1.4142135623730951;
  const int64_t tile = i / 16;
  const int li = (int)(i % 16);
  double nrm = 0.0;
  for (int q = 0; q < nk4 * 4; ++q) {
    T x = q < d ? (T)(scale * xs[i * d + q]) : (T)0;
    double rep = (double)x;
    nrm += rep * rep;
    const int64_t slot = (tile * nk4 + q / 4) * 64 + li + 16 * (q % 4);
    xfb[slot] = x;
    xfa[slot] = rbf32 ? x : -x;
  }
  if (rbf32) {
    rowterm[i] = (T)(-0.5 * nrm + log2s);
    colterm[i] = (T)(-0.5 * nrm);
  } else {
    rowterm[i] = (T)(0.5 * nrm);
    colterm[i] = (T)(0.5 * nrm);
  }
}

// V (rows < nrows of an FP64 row-major array with leading dimension ldv) ->
// fragment-major tile-precision copy of ncols staged columns; staged column c
// holds source column colmap[c] (c itself when colmap is null; nothing, i.e.
// zeros, when the entry is negative).  Everything else is zero.
__device__ inline int staged_source(const int* __restrict__ colmap, int col, int ncols) {
  if (col >= ncols) return -1;
  return colmap != nullptr ? colmap[col] : col;
}

// BF16: fragment (jb, tt, piece) lane l holds rows jb*32 + perm(l/16, s), s < 8,
// perm(g, s) = 4g + s (s < 4) or 16 + 4g + s - 4, column tt*16 + l%16.
__global__ void k_stage_v_bf16(const double* __restrict__ V, int64_t nrows, int ldv, int ncols,
                               const int* __restrict__ colmap, int64_t n_pad, int ntt, int NP,
                               u32x4* __restrict__ vfrag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (jb, tt, lane)
  const int64_t total = (n_pad / 32) * ntt * 64;
  if (e >= total) return;
  const int lane = (int)(e % 64);
  const int tt = (int)((e / 64) % ntt);
  const int64_t jb = e / (64 * ntt);
  const int g = lane / 16, col = tt * 16 + lane % 16;
  const int src = staged_source(colmap, col, ncols);
  // FP64 -> hi + lo (+ lo2 when NP = 3): hi = RNE(v), lo = RNE(v - hi),
  // lo2 = RNE(v - hi - lo), the remainders taken in FP64
  uint32_t h[4], l[4], m[4];
  for (int w = 0; w < 4; ++w) {
    int64_t j0 = jb * 32 + (2 * w < 4 ? 4 * g + 2 * w : 16 + 4 * g + (2 * w - 4));
    int64_t j1 = j0 + 1;
    double a = (j0 < nrows && src >= 0) ? V[j0 * ldv + src] : 0.0;
    double b = (j1 < nrows && src >= 0) ? V[j1 * ldv + src] : 0.0;
    uint32_t hh = pack_bf16((float)a, (float)b);
    double ra = a - (double)bf16_lo_f(hh), rb = b - (double)bf16_hi_f(hh);
    h[w] = hh;
    l[w] = pack_bf16((float)ra, (float)rb);
    m[w] = pack_bf16((float)(ra - (double)bf16_lo_f(l[w])), (float)(rb - (double)bf16_hi_f(l[w])));
  }
  vfrag[((jb * ntt + tt) * NP + 0) * 64 + lane] = u32x4{h[0], h[1], h[2], h[3]};
  vfrag[((jb * ntt + tt) * NP + 1) * 64 + lane] = u32x4{l[0], l[1], l[2], l[3]};
  if (NP == 3) vfrag[((jb * ntt + tt) * NP + 2) * 64 + lane] = u32x4{m[0], m[1], m[2], m[3]};
}

// column maxima of |V| as float bit patterns (non-negative floats order like their
// bits, so the integer maximum is exact and order-independent)
__global__ void k_colmax(const double* __restrict__ V, int64_t nrows, int ldv, int ncols,
                         const int* __restrict__ colmap, uint32_t* __restrict__ cm, int64_t rows_per_block) {
  // block: 64 staged columns x 4 row lanes over rows_per_block rows (each row's columns
  // read together); blocks combine with atomicMax
  __shared__ uint32_t red[4][64];
  const int cl = threadIdx.x % 64, lane4 = threadIdx.x / 64;
  const int c = blockIdx.y * 64 + cl;
  const int src = staged_source(colmap, c, ncols);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(nrows, r0 + rows_per_block);
  uint32_t m = 0;
  if (src >= 0) {
    for (int64_t r = r0 + lane4; r < r1; r += 4) {
      const uint32_t b = __builtin_bit_cast(uint32_t, fabsf((float)V[r * ldv + src]));
      m = b > m ? b : m;
    }
  }
  red[lane4][cl] = m;
  __syncthreads();
  if (lane4 == 0 && src >= 0) atomicMax(cm + c, max(max(red[0][cl], red[1][cl]), max(red[2][cl], red[3][cl])));
}

__global__ void k_zero_u32(uint32_t* p, int count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0;
}

// power-of-two scale that brings a column's maximum into [2^13, 2^14)
__device__ __host__ inline float f16_col_scale(uint32_t maxbits) {
  const float m = __builtin_bit_cast(float, maxbits);
  if (!(m > 0.0f)) return 1.0f;
  int e;
  frexpf(m, &e);  // m = f * 2^e, f in [0.5, 1)
  return ldexpf(1.0f, 14 - e);
}

// as k_stage_v_bf16 with FP16 hi + lo of (scale_c * V)
__global__ void k_stage_v_f16(const double* __restrict__ V, int64_t nrows, int ldv, int ncols,
                              const int* __restrict__ colmap, int64_t n_pad, int ntt, const uint32_t* __restrict__ cm,
                              u32x4* __restrict__ vfrag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (jb, tt, lane)
  const int64_t total = (n_pad / 32) * ntt * 64;
  if (e >= total) return;
  const int lane = (int)(e % 64);
  const int tt = (int)((e / 64) % ntt);
  const int64_t jb = e / (64 * ntt);
  const int g = lane / 16, col = tt * 16 + lane % 16;
  const int src = staged_source(colmap, col, ncols);
  const double sc = (col < ncols) ? (double)f16_col_scale(cm[col]) : 1.0;
  uint32_t h[4], l[4];
  for (int w = 0; w < 4; ++w) {
    int64_t j0 = jb * 32 + (2 * w < 4 ? 4 * g + 2 * w : 16 + 4 * g + (2 * w - 4));
    int64_t j1 = j0 + 1;
    double a = (j0 < nrows && src >= 0) ? sc * V[j0 * ldv + src] : 0.0;
    double b = (j1 < nrows && src >= 0) ? sc * V[j1 * ldv + src] : 0.0;
    const uint32_t hh = pack_f16((float)a, (float)b);
    const f32x2 hf = __builtin_convertvector(__builtin_bit_cast(f16x2, hh), f32x2);
    h[w] = hh;
    l[w] = pack_f16((float)(a - (double)hf[0]), (float)(b - (double)hf[1]));
  }
  vfrag[((jb * ntt + tt) * 2 + 0) * 64 + lane] = u32x4{h[0], h[1], h[2], h[3]};
  vfrag[((jb * ntt + tt) * 2 + 1) * 64 + lane] = u32x4{l[0], l[1], l[2], l[3]};
}

// the extra column of the split-precision tiles: FP32 values of staged column
// xcol (times its FP16 power-of-two scale when cm is given), zero past nrows
__global__ void k_stage_vx(const double* __restrict__ V, int64_t nrows, int ldv, int xcol, int ncols,
                           const int* __restrict__ colmap, int64_t n_pad, const uint32_t* __restrict__ cm,
                           float* __restrict__ vx) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_pad) return;
  const int src = staged_source(colmap, xcol, ncols);
  const double sc = cm != nullptr ? (double)f16_col_scale(cm[xcol]) : 1.0;
  vx[j] = (j < nrows && src >= 0) ? (float)(sc * V[j * ldv + src]) : 0.0f;
}

// FP32/FP64: fragment (j16, tt, v) lane l holds row j16*16 + acc_row(l/16, v), column tt*16 + l%16
template <typename T>
__global__ void k_stage_v_fp(const double* __restrict__ V, int64_t nrows, int ldv, int ncols,
                             const int* __restrict__ colmap, int64_t n_pad, int ntt, T* __restrict__ vfrag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (j16, tt, v, lane)
  const int64_t total = (n_pad / 16) * ntt * 4 * 64;
  if (e >= total) return;
  const int lane = (int)(e % 64);
  const int v = (int)((e / 64) % 4);
  const int tt = (int)((e / 256) % ntt);
  const int64_t j16 = e / (256 * ntt);
  const int64_t j = j16 * 16 + acc_row<T>(lane / 16, v);
  const int src = staged_source(colmap, tt * 16 + lane % 16, ncols);
  vfrag[e] = (j < nrows && src >= 0) ? (T)V[j * ldv + src] : (T)0;
}

// W[i][c] = sum_s wpart[s][i][c] + sigma^2 V[i][c] (FP64, fixed order), rows < nrows,
// columns < ncols; optionally per-block partial dots V[:,c].W[:,c].  Block: 64 rows x
// kRedCols columns, 320 threads = 20 column quads x 16 row lanes: a thread reads four
// consecutive partial columns with one vector load per split and row (a wave covers
// about three whole 80-column partial rows per load), for the rows rl, rl + 16,
// rl + 32 and rl + 48 of the block, all loads in flight before the sums.  The 16 row
// lanes' dot sums are added in a fixed order and the block shape is fixed, so a
// column's partial dot has the same summation order however many columns are active.
constexpr int kRedCols = 80;
constexpr int kRedQuads = kRedCols / 4;
constexpr int kRedLanes = 16;
constexpr int kRedThreads = kRedQuads * kRedLanes;
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_khat_reduce(const T* __restrict__ wpart, int nsplit, int64_t n_pad,
                                                             int tp, const double* __restrict__ V, int ldv,
                                                             double* __restrict__ W, int ldw, int64_t nrows, int ncols,
                                                             const int* __restrict__ colmap, int ldpart, double s2,
                                                             double* __restrict__ dot_part,
                                                             const int* __restrict__ nactive,
                                                             const uint32_t* __restrict__ colmax, double fac_s) {
  if (nactive != nullptr && *nactive == 0) return;
  typedef T T4 __attribute__((ext_vector_type(4)));
  __shared__ double red[kRedLanes][kRedCols];
  const int cq = threadIdx.x % kRedQuads, rl = threadIdx.x / kRedQuads;
  // staged column c0 + v carries source column src[v] (results go back to that column)
  const int c0 = blockIdx.y * kRedCols + 4 * cq;
  int src[4];
  double fac[4];
  bool any = false;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    src[v] = staged_source(colmap, c0 + v, ncols);
    // FP16X3 partials carry the factors 2^15 / s (kernel values) and scale_c (column)
    fac[v] = (colmax != nullptr && src[v] >= 0) ? fac_s / (double)f16_col_scale(colmax[c0 + v]) : 1.0;
    any = any || src[v] >= 0;
  }
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  double dot[4] = {0.0, 0.0, 0.0, 0.0};
  // an active column lies below ncols <= tp, so a quad with one is inside the partial row
  if (any) {
    double w[4][4];
    bool rin[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      rin[q] = r0 + rl + 16 * q < nrows;
#pragma unroll
      for (int v = 0; v < 4; ++v) w[q][v] = 0.0;
    }
    // the V values first (clamped addresses, then a select), so they are in flight
    // with the partial-sum loads
    double vvp[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool in = rin[q] && src[v] >= 0;
        const double t = V[in ? (r0 + rl + 16 * q) * ldv + src[v] : 0];
        vvp[q][v] = in ? t : 0.0;
      }
    // partial rows exist up to n_pad >= 64 * gridDim.x, so the loads need no row
    // condition (rows past nrows are summed and never used)
    for (int s = 0; s < nsplit; ++s) {
      T4 pv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        pv[q] = *reinterpret_cast<const T4*>(wpart + ((int64_t)s * n_pad + r0 + rl + 16 * q) * tp + c0);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) w[q][v] += (double)pv[q][v];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!rin[q]) continue;
      const int64_t r = r0 + rl + 16 * q;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (src[v] < 0) continue;
        const double vv = vvp[q][v];
        const double ww = w[q][v] * fac[v] + s2 * vv;
        W[r * ldw + src[v]] = ww;
        dot[v] += vv * ww;
      }
    }
  }
  if (dot_part == nullptr) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) red[rl][4 * cq + v] = dot[v];
  __syncthreads();
  if (rl == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (src[v] < 0) continue;
      double t = 0.0;
      for (int l = 0; l < kRedLanes; ++l) t += red[l][4 * cq + v];
      dot_part[(int64_t)blockIdx.x * ldpart + src[v]] = t;
    }
  }
}

#endif  // part 0

#if GPMLL_KHAT_PART == 1 || GPMLL_KHAT_PART == 4
// Software-pipelined BF16x3 tile kernel.  Per wave (RG row groups of 16 rows)
// and per 32-column step j:
//   distance MFMAs of step j+1          (16 MFMAs for d <= 16)
//   tile x V MFMAs of step j            (3 * NTT * RG MFMAs)
//   kernel map + hi/lo split of step j+1 (VALU), interleaved with the MFMAs above
// so the matrix pipe and the vector ALU of one wave work at the same time.  Stage
// data (distance A fragments, V fragments, column terms) rotate through three LDS
// buffers: step j reads V of stage j and A of stage j+1 while stage j+2 lands.

// distance accumulators of one step: dd[rg][js] (lane = row i, 4 consecutive j)
template <int NKC, int RG>
__device__ __forceinline__ void bf16_distance(const u32x4* __restrict__ A, const u32x4 (&xbv)[RG][NKC],
                                              const f32x4 (&rt)[RG], f32x4 (&dd)[RG][2], int lane) {
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int js = 0; js < 2; ++js) dd[rg][js] = rt[rg];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
      for (int js = 0; js < 2; ++js)
        dd[rg][js] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[(js * NKC + kc) * 64 + lane]),
                                                             __builtin_bit_cast(bf16x8, xbv[rg][kc]), dd[rg][js], 0,
                                                             0, 0);
}

// kernel map and hi/lo split of one step: dd -> (ph, pl); DIAG puts s on i == j.
// XC: the FP32 kernel values also meet the extra column (its 32 values follow the
// column terms in the stage), yacc[rg][js] += sum_v kv[v] y[j(v)] in FP32.
template <int KIND, int RG, bool DIAG, bool F16, int XC>
__device__ __forceinline__ void bf16_map(const f32x4 (&dd)[RG][2], const float* __restrict__ ct, u32x4 (&ph)[RG],
                                         u32x4 (&pl)[RG], float (&yacc)[RG][2], int lane, int64_t row0, int64_t c,
                                         float s32, float alpha) {
  const int g = lane >> 4, li = lane & 15;
  const f32x4 ct0 = *reinterpret_cast<const f32x4*>(ct + 4 * g);
  const f32x4 ct1 = *reinterpret_cast<const f32x4*>(ct + 16 + 4 * g);
  f32x4 yv0{}, yv1{};
  if constexpr (XC != 0) {
    yv0 = *reinterpret_cast<const f32x4*>(ct + 32 + 4 * g);
    yv1 = *reinterpret_cast<const f32x4*>(ct + 48 + 4 * g);
  }
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int js = 0; js < 2; ++js) {
      const f32x4 ctv = js ? ct1 : ct0;
      float kv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) kv[v] = map_split<KIND>(dd[rg][js][v] + ctv[v], s32, alpha);
      if constexpr (DIAG) {
        const int64_t i = row0 + rg * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) kv[v] = (i == c + js * 16 + 4 * g + v) ? s32 : kv[v];
      }
      if constexpr (XC != 0) {
        const f32x4 yv = js ? yv1 : yv0;
#pragma unroll
        for (int v = 0; v < 4; ++v) yacc[rg][js] = fmaf(kv[v], yv[v], yacc[rg][js]);
      }
      uint32_t h0, l0, h1, l1;
      if constexpr (F16) {
        split_pair_f16(kv[0], kv[1], &h0, &l0);
        split_pair_f16(kv[2], kv[3], &h1, &l1);
      } else {
        split_pair(kv[0], kv[1], &h0, &l0);
        split_pair(kv[2], kv[3], &h1, &l1);
      }
      ph[rg][2 * js] = h0;
      ph[rg][2 * js + 1] = h1;
      pl[rg][2 * js] = l0;
      pl[rg][2 * js + 1] = l1;
    }
}

// tile x V MFMAs of one step: acc += P V with P = hi + lo, V = hi + lo (3 products)
template <bool F16>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                   0);
}

template <int NTT, int RG, bool F16, int NTA, int NP>
__device__ __forceinline__ void bf16_tile_v(const u32x4* __restrict__ Vf, const u32x4 (&ph)[RG], const u32x4 (&pl)[RG],
                                            f32x4 (&acc)[RG][NTA], int lane) {
  if constexpr (F16) {
#pragma unroll
    for (int tt = 0; tt < NTT; ++tt) {
      const u32x4 vh = Vf[(tt * 2 + 0) * 64 + lane];
      const u32x4 vl = Vf[(tt * 2 + 1) * 64 + lane];
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) acc[rg][tt] = mfma16<true>(ph[rg], vh, acc[rg][tt]);
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) acc[rg][tt] = mfma16<true>(ph[rg], vl, acc[rg][tt]);
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) acc[rg][tt] = mfma16<true>(pl[rg], vh, acc[rg][tt]);
    }
    return;
  }
#pragma unroll
  for (int tt = 0; tt < NTT; ++tt) {
    const bf16x8 vh = __builtin_bit_cast(bf16x8, Vf[(tt * NP + 0) * 64 + lane]);
    const bf16x8 vl = __builtin_bit_cast(bf16x8, Vf[(tt * NP + 1) * 64 + lane]);
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
      acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ph[rg]), vh, acc[rg][tt], 0, 0, 0);
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
      acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ph[rg]), vl, acc[rg][tt], 0, 0, 0);
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
      acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, pl[rg]), vh, acc[rg][tt], 0, 0, 0);
    if constexpr (NP == 3) {
      // the third piece of the search direction: hi x lo2
      const bf16x8 vm = __builtin_bit_cast(bf16x8, Vf[(tt * NP + 2) * 64 + lane]);
#pragma unroll
      for (int rg = 0; rg < RG; ++rg)
        acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ph[rg]), vm, acc[rg][tt], 0, 0,
                                                              0);
    }
  }
}

// interleave: one MFMA, then two VALU instructions, for the tile x V MFMAs
template <int NMFMA>
__device__ __forceinline__ void bf16_interleave_hint() {
#pragma unroll
  for (int i = 0; i < NMFMA; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // VALU
  }
}

// Stage for one 32-column step, copied global -> LDS without registers
// (global_load_lds_dwordx4: each wave instruction moves one contiguous 1 KB
// chunk): [A fragments 2 x NKC | V fragments NTT x {hi, lo} | column terms].
// The last chunk holds the 32 column terms (units 0-7) and, with XC, the 32 FP32
// values of the extra right-hand side column (units 8-15).
template <int NKC, int NTT, int XC, int NP>
__device__ __forceinline__ void bf16_issue_stage(u32x4* dst, const u32x4* __restrict__ xfa,
                                                 const u32x4* __restrict__ vfrag, const float* __restrict__ colterm,
                                                 const float* __restrict__ vx, int64_t c, int wave, int lane) {
  constexpr int NCH = 2 * NKC + NP * NTT + 1;
  // the chunk walk is the same for the whole wave: keep it on the scalar unit
  for (int ch = __builtin_amdgcn_readfirstlane(wave); ch < NCH; ch += 4) {
    const u32x4* src;
    if (ch < 2 * NKC) src = xfa + (c / 16) * NKC * 64 + ch * 64 + lane;
    else if (ch < 2 * NKC + NP * NTT) src = vfrag + (c / 32) * NTT * NP * 64 + (ch - 2 * NKC) * 64 + lane;
    else if (XC && lane >= 8 && lane < 16) src = reinterpret_cast<const u32x4*>(vx + c) + (lane - 8);
    else src = reinterpret_cast<const u32x4*>(colterm + c) + (lane < 8 ? lane : 7);
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(dst + ch * 64), 16, 0, 0);
  }
}

// NTT 16-column tiles of right-hand sides on the matrix cores and, with XC = 1,
// one more column (staged column 16 NTT) contracted on the vector ALU from the
// FP32 kernel values: a column count of 16 m + 1 (y and 16 m probes) then needs
// no mostly-empty sixteen-column tile.  VP: pieces of the BF16 search directions
// (2, or 3 with the extra hi x lo2 product).
template <int KIND, int NKC, int NTT, int RG, bool F16, int XC, int VP>
__global__ __launch_bounds__(256, 2) void k_khat_bf16(const u32x4* __restrict__ xfa, const u32x4* __restrict__ xfb,
                                                      const float* __restrict__ rowterm,
                                                      const float* __restrict__ colterm,
                                                      const u32x4* __restrict__ vfrag, const float* __restrict__ vx,
                                                      float* __restrict__ wpart, TileArgs a,
                                                      const int* __restrict__ nactive) {
  if (nactive != nullptr && *nactive == 0) return;
  constexpr int NTA = NTT > 0 ? NTT : 1;  // accumulator array extent
  constexpr int NP = F16 ? 2 : VP;  // pieces of each staged V value
  constexpr int A_U = 2 * NKC * 64, V_U = NTT * NP * 64, C_U = 64;
  constexpr int STAGE = A_U + V_U + C_U;
  __shared__ u32x4 lds[3][STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * RG) + wave * (16 * RG);
  const int64_t c_begin = (int64_t)blockIdx.y * a.cols_per_split;
  const int64_t c_end = min(a.n_pad, c_begin + a.cols_per_split);
  if (c_begin >= c_end) return;
  const int nsteps = (int)((c_end - c_begin) / 32);

  u32x4 xbv[RG][NKC];
  f32x4 rt[RG];
  f32x4 acc[RG][NTA];
  float yacc[RG][2];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) xbv[rg][kc] = xfb[((row0 / 16 + rg) * NKC + kc) * 64 + lane];
    const float r = rowterm[row0 + rg * 16 + li];
    rt[rg] = f32x4{r, r, r, r};
#pragma unroll
    for (int tt = 0; tt < NTA; ++tt) acc[rg][tt] = f32x4{0.f, 0.f, 0.f, 0.f};
    yacc[rg][0] = yacc[rg][1] = 0.f;
  }
  auto is_diag = [&](int64_t c) { return (c + 32 > row0) && (c < row0 + 16 * RG); };

  // prologue: stages 0 and 1 in flight, P of step 0
  bf16_issue_stage<NKC, NTT, XC, NP>(lds[0], xfa, vfrag, colterm, vx, c_begin, wave, lane);
  if (nsteps > 1) bf16_issue_stage<NKC, NTT, XC, NP>(lds[1], xfa, vfrag, colterm, vx, c_begin + 32, wave, lane);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  u32x4 ph[RG], pl[RG];
  {
    f32x4 dd[RG][2];
    bf16_distance<NKC, RG>(lds[0], xbv, rt, dd, lane);
    const float* ct = reinterpret_cast<const float*>(lds[0] + A_U + V_U);
    if (is_diag(c_begin))
      bf16_map<KIND, RG, true, F16, XC>(dd, ct, ph, pl, yacc, lane, row0, c_begin, a.s32, a.alpha32);
    else
      bf16_map<KIND, RG, false, F16, XC>(dd, ct, ph, pl, yacc, lane, row0, c_begin, a.s32, a.alpha32);
  }
  int cur = 0;
  for (int j = 0; j + 1 < nsteps; ++j) {
    const int nxt = cur == 2 ? 0 : cur + 1;
    const int far = nxt == 2 ? 0 : nxt + 1;
    const int64_t cn = c_begin + (int64_t)(j + 1) * 32;
    if (j + 2 < nsteps) bf16_issue_stage<NKC, NTT, XC, NP>(lds[far], xfa, vfrag, colterm, vx, cn + 32, wave, lane);
    f32x4 dd[RG][2];
    bf16_distance<NKC, RG>(lds[nxt], xbv, rt, dd, lane);
    u32x4 nph[RG], npl[RG];
    const float* ctn = reinterpret_cast<const float*>(lds[nxt] + A_U + V_U);
    if (is_diag(cn)) {
      bf16_tile_v<NTT, RG, F16, NTA, NP>(lds[cur] + A_U, ph, pl, acc, lane);
      bf16_map<KIND, RG, true, F16, XC>(dd, ctn, nph, npl, yacc, lane, row0, cn, a.s32, a.alpha32);
    } else {
      bf16_tile_v<NTT, RG, F16, NTA, NP>(lds[cur] + A_U, ph, pl, acc, lane);
      bf16_map<KIND, RG, false, F16, XC>(dd, ctn, nph, npl, yacc, lane, row0, cn, a.s32, a.alpha32);
    }
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      ph[rg] = nph[rg];
      pl[rg] = npl[rg];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur = nxt;
  }
  bf16_tile_v<NTT, RG, F16, NTA, NP>(lds[cur] + A_U, ph, pl, acc, lane);

  float* out = wpart + (int64_t)blockIdx.y * a.n_pad * a.tp;
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int tt = 0; tt < NTT; ++tt)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(row0 + rg * 16 + 4 * g + v) * a.tp + tt * 16 + li] = acc[rg][tt][v];
  if constexpr (XC != 0) {
    // row i = li of each row group: the four lane groups hold disjoint column
    // subsets; combine them in a fixed order ((g0 + g1) + (g2 + g3))
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      float y = yacc[rg][0] + yacc[rg][1];
      y += __shfl_xor(y, 16);
      y += __shfl_xor(y, 32);
      if (g == 0) out[(row0 + rg * 16 + li) * a.tp + 16 * NTT] = y;
    }
  }
}

#endif  // parts 1, 4

#if GPMLL_KHAT_PART == 2 || GPMLL_KHAT_PART == 3
// FP32 / FP64 tiles with v_mfma_{f32,f64}_16x16x4.  The accumulator -> operand
// hand-off: the lane holding D[j = acc_row(l/16, v)][i = l%16] supplies the A
// operand of MFMA number v, whose K index l/16 stands for that j.
template <typename T>
struct FpMfma;
template <>
struct FpMfma<float> {
  typedef f32x4 acc_t;
  __device__ static acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct FpMfma<double> {
  typedef f64x4 acc_t;
  __device__ static acc_t mfma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

template <typename T, int KIND, int NK4, int NTT, int RG>
__global__ __launch_bounds__(256, 2) void k_khat_fp(const T* __restrict__ xfa, const T* __restrict__ xfb,
                                                    const T* __restrict__ rowterm, const T* __restrict__ colterm,
                                                    const T* __restrict__ vfrag, T* __restrict__ wpart, TileArgs a,
                                                    const int* __restrict__ nactive, const int4* __restrict__ items,
                                                    const int* __restrict__ item_gate,
                                                    const int* __restrict__ gate_count) {
  if (nactive != nullptr && *nactive == 0) return;
  // work items whose group (problem) has no active column left are skipped
  if (item_gate != nullptr && gate_count[item_gate[blockIdx.x]] == 0) return;
  typedef typename FpMfma<T>::acc_t acc_t;
  // stage of 16 columns: A fragments NK4*64, V fragments NTT*4*64, column terms 16
  constexpr int A_E = NK4 * 64, V_E = NTT * 4 * 64, C_E = 16;
  constexpr int STAGE = A_E + V_E + C_E;
  constexpr int PER = (STAGE + 255) / 256;
  __shared__ T lds[2][STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  // block -> (first row, column range, output slot): the regular grid, or one
  // entry of a work-item table (ragged batches: every item stays inside one
  // problem's diagonal block)
  int64_t row0, c_begin, c_end, slot;
  if (items != nullptr) {
    const int4 it = items[blockIdx.x];
    row0 = (int64_t)it.x + wave * (16 * RG);
    c_begin = it.y;
    c_end = it.z;
    slot = it.w;
  } else {
    row0 = (int64_t)blockIdx.x * (64 * RG) + wave * (16 * RG);
    c_begin = (int64_t)blockIdx.y * a.cols_per_split;
    c_end = min(a.n_pad, c_begin + a.cols_per_split);
    slot = blockIdx.y;
  }
  if (c_begin >= c_end) return;

  T xb[RG][NK4];
  acc_t rt[RG];
  acc_t acc[RG][NTT];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
    for (int kc = 0; kc < NK4; ++kc) xb[rg][kc] = xfb[((row0 / 16 + rg) * NK4 + kc) * 64 + lane];
    T r = rowterm[row0 + rg * 16 + li];
    rt[rg] = acc_t{r, r, r, r};
#pragma unroll
    for (int tt = 0; tt < NTT; ++tt) acc[rg][tt] = acc_t{0, 0, 0, 0};
  }
  auto load = [&](int64_t c, int e) -> T {
    if (e < A_E) return xfa[(c / 16) * NK4 * 64 + e];
    if (e < A_E + V_E) return vfrag[(c / 16) * NTT * 4 * 64 + (e - A_E)];
    return colterm[c + (e - A_E - V_E)];
  };
  for (int e = tid; e < STAGE; e += 256) lds[0][e] = load(c_begin, e);
  __syncthreads();
  int buf = 0;
  for (int64_t c = c_begin; c < c_end; c += 16) {
    const bool has_next = c + 16 < c_end;
    T pre[PER];
    if (has_next) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        int e = tid + q * 256;
        if (e < STAGE) pre[q] = load(c + 16, e);
      }
    }
    const T* A = lds[buf];
    const T* Vf = A + A_E;
    const T* ct = A + A_E + V_E;
    const bool diag = (c + 16 > row0) && (c < row0 + 16 * RG);
    T ctv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) ctv[v] = ct[acc_row<T>(g, v)];
    T kv[RG][4];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      acc_t dd = rt[rg];
#pragma unroll
      for (int kc = 0; kc < NK4; ++kc) dd = FpMfma<T>::mfma(A[kc * 64 + lane], xb[rg][kc], dd);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T q = dd[v] + ctv[v];
        if constexpr (sizeof(T) == 4) kv[rg][v] = map32<KIND>(q, a.s32, a.alpha32);
        else kv[rg][v] = map64<KIND>(q, a.s64, a.alpha64);
      }
      if (diag) {
        const int64_t i = row0 + rg * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (i == c + acc_row<T>(g, v)) kv[rg][v] = (sizeof(T) == 4) ? (T)a.s32 : (T)a.s64;
      }
    }
#pragma unroll
    for (int tt = 0; tt < NTT; ++tt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T bv = Vf[(tt * 4 + v) * 64 + lane];
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) acc[rg][tt] = FpMfma<T>::mfma(kv[rg][v], bv, acc[rg][tt]);
      }
    }
    if (has_next) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        int e = tid + q * 256;
        if (e < STAGE) lds[buf ^ 1][e] = pre[q];
      }
    }
    __syncthreads();
    buf ^= 1;
  }
  T* out = wpart + slot * a.n_pad * a.tp;
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int tt = 0; tt < NTT; ++tt)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(row0 + rg * 16 + acc_row<T>(g, v)) * a.tp + tt * 16 + li] = acc[rg][tt][v];
}

#endif  // parts 2, 3

// ---------------------------------------------------------------------------
// dispatch: NTT = tp / 16 takes the values of kSupportedNtt; the distance
// K-extent takes 1..4 chunks of 32 (BF16) or 1, 2, 4, 8 chunks of 4 (FP32/FP64).
// Each precision is compiled in its own translation unit (GPMLL_KHAT_PART).
// ---------------------------------------------------------------------------

hipError_t khat_tiles_bf16x3(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact);
hipError_t khat_tiles_f16x3(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact);
hipError_t khat_tiles_fp32(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact,
                           const ItemTable& it = ItemTable{});
hipError_t khat_tiles_fp64(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact,
                           const ItemTable& it = ItemTable{});

#define GPMLL_NTT_CASES(M) M(1) M(2) M(3) M(4) M(5) M(6) M(8) M(12) M(16)
// split-precision tiles with the extra vector-ALU column: 16 NTT + 1 columns
#define GPMLL_XC_NTT_CASES(M) M(0) M(1) M(2) M(3) M(4)
// BF16x3 tiles with three-piece search directions (at most eight tiles)
#define GPMLL_V3_NTT_CASES(M) M(1) M(2) M(3) M(4) M(5) M(6) M(8)

#if GPMLL_KHAT_PART == 1 || GPMLL_KHAT_PART == 4
namespace {
constexpr bool kF16 = GPMLL_KHAT_PART == 4;
template <int KIND, int NKC, int NTT, int XC, int VP>
hipError_t run_bf16(const Ctx& c, const TileArgs& ta, const int* nact) {
  const Layout& L = *c.lay;
  constexpr int RG = NTT <= 5 ? 4 : (NTT <= 8 ? 2 : 1);
  dim3 grid((unsigned)(L.n_pad / (64 * RG)), (unsigned)L.nsplit);
  hipLaunchKernelGGL((k_khat_bf16<KIND, NKC, NTT, RG, kF16, XC, VP>), grid, dim3(256), 0, c.st, c.at<u32x4>(L.xfa),
                     c.at<u32x4>(L.xfb), c.at<float>(L.rowterm), c.at<float>(L.colterm), c.at<u32x4>(L.vfrag),
                     c.at<float>(L.vx), c.at<float>(L.wpart), ta, nact);
  return hipGetLastError();
}
template <int KIND, int NKC>
hipError_t sel_bf16_ntt(const Ctx& c, const TileArgs& ta, const int* nact) {
  if (!kF16 && ta.vp == 3) {
    if (ta.xc != 0) {
      switch (ta.ntt) {
#define CASE(N) case N: return run_bf16<KIND, NKC, N, 1, 3>(c, ta, nact);
        GPMLL_XC_NTT_CASES(CASE)
#undef CASE
      }
      return hipErrorInvalidValue;
    }
    switch (ta.ntt) {
#define CASE(N) case N: return run_bf16<KIND, NKC, N, 0, 3>(c, ta, nact);
      GPMLL_V3_NTT_CASES(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
  }
  if (ta.xc != 0) {
    switch (ta.ntt) {
#define CASE(N) case N: return run_bf16<KIND, NKC, N, 1, 2>(c, ta, nact);
      GPMLL_XC_NTT_CASES(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
  }
  switch (ta.ntt) {
#define CASE(N) case N: return run_bf16<KIND, NKC, N, 0, 2>(c, ta, nact);
    GPMLL_NTT_CASES(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}
template <int KIND>
hipError_t sel_bf16(const Ctx& c, const TileArgs& ta, const int* nact) {
  const Layout& L = *c.lay;
  switch (L.kd / 32) {
    case 1: return sel_bf16_ntt<KIND, 1>(c, ta, nact);
    case 2: return sel_bf16_ntt<KIND, 2>(c, ta, nact);
    case 3: return sel_bf16_ntt<KIND, 3>(c, ta, nact);
    case 4: return sel_bf16_ntt<KIND, 4>(c, ta, nact);
  }
  return hipErrorInvalidValue;
}
}  // namespace
#if GPMLL_KHAT_PART == 1
hipError_t khat_tiles_bf16x3(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact) {
#else
hipError_t khat_tiles_f16x3(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact) {
#endif
  switch (h.kind) {
    case GP_KERNEL_RBF: return sel_bf16<GP_KERNEL_RBF>(c, ta, nact);
    case GP_KERNEL_MATERN32: return sel_bf16<GP_KERNEL_MATERN32>(c, ta, nact);
    case GP_KERNEL_RATQUAD: return sel_bf16<GP_KERNEL_RATQUAD>(c, ta, nact);
    default: return sel_bf16<GP_KERNEL_MATERN52>(c, ta, nact);
  }
}
#endif

#if GPMLL_KHAT_PART == 2 || GPMLL_KHAT_PART == 3
namespace {
template <typename T, int KIND, int NK4, int NTT>
hipError_t run_fp(const Ctx& c, const TileArgs& ta, const int* nact, const ItemTable& it) {
  const Layout& L = *c.lay;
  constexpr int RG = fp_row_groups(sizeof(T), NTT);
  dim3 grid = it.items != nullptr ? dim3((unsigned)it.nitems)
                                  : dim3((unsigned)(L.n_pad / (64 * RG)), (unsigned)L.nsplit);
  hipLaunchKernelGGL((k_khat_fp<T, KIND, NK4, NTT, RG>), grid, dim3(256), 0, c.st, c.at<T>(L.xfa), c.at<T>(L.xfb),
                     c.at<T>(L.rowterm), c.at<T>(L.colterm), c.at<T>(L.vfrag), c.at<T>(L.wpart), ta, nact, it.items,
                     it.gate, it.gate_count);
  return hipGetLastError();
}
template <typename T, int KIND, int NK4>
hipError_t sel_fp_ntt(const Ctx& c, const TileArgs& ta, const int* nact, int ntt, const ItemTable& it) {
  switch (ntt) {
#define CASE(N) case N: return run_fp<T, KIND, NK4, N>(c, ta, nact, it);
    GPMLL_NTT_CASES(CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}
template <typename T, int KIND>
hipError_t sel_fp(const Ctx& c, const TileArgs& ta, const int* nact, const ItemTable& it) {
  const Layout& L = *c.lay;
  const int ntt = ta.ntt;
  switch (L.kd / 4) {
    case 1: return sel_fp_ntt<T, KIND, 1>(c, ta, nact, ntt, it);
    case 2: return sel_fp_ntt<T, KIND, 2>(c, ta, nact, ntt, it);
    case 4: return sel_fp_ntt<T, KIND, 4>(c, ta, nact, ntt, it);
    case 8: return sel_fp_ntt<T, KIND, 8>(c, ta, nact, ntt, it);
  }
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t khat_tiles_fp(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact, const ItemTable& it) {
  switch (h.kind) {
    case GP_KERNEL_RBF: return sel_fp<T, GP_KERNEL_RBF>(c, ta, nact, it);
    case GP_KERNEL_MATERN32: return sel_fp<T, GP_KERNEL_MATERN32>(c, ta, nact, it);
    case GP_KERNEL_RATQUAD: return sel_fp<T, GP_KERNEL_RATQUAD>(c, ta, nact, it);
    default: return sel_fp<T, GP_KERNEL_MATERN52>(c, ta, nact, it);
  }
}
}  // namespace
#if GPMLL_KHAT_PART == 2
hipError_t khat_tiles_fp32(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact, const ItemTable& it) {
  return khat_tiles_fp<float>(c, h, ta, nact, it);
}
#else
hipError_t khat_tiles_fp64(const Ctx& c, const Hyper& h, const TileArgs& ta, const int* nact, const ItemTable& it) {
  return khat_tiles_fp<double>(c, h, ta, nact, it);
}
#endif
#endif

#if GPMLL_KHAT_PART == 0
hipError_t launch_stage_x(const Ctx& c, const Hyper& h) {
  const Layout& L = *c.lay;
  const unsigned nb = (unsigned)((L.n_pad + 255) / 256);
  if (L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3) {
    const int dq = (L.d + 7) / 8 * 8;
    const float rbf_add = L.prec == GP_PREC_FP16X3 ? 15.0f : (float)h.log2s;
    hipLaunchKernelGGL(k_stage_x_bf16, dim3(nb), dim3(256), 0, c.st, c.at<double>(L.xs), L.n_pad, L.d, dq,
                       L.kd / 32, h.kind, h.alpha, rbf_add, c.at<u32x4>(L.xfa), c.at<u32x4>(L.xfb),
                       c.at<float>(L.rowterm), c.at<float>(L.colterm));
  } else if (L.prec == GP_PREC_FP32) {
    hipLaunchKernelGGL(k_stage_x_fp<float>, dim3(nb), dim3(256), 0, c.st, c.at<double>(L.xs), L.n_pad, L.d,
                       L.kd / 4, h.kind == GP_KERNEL_RBF ? 1 : 0, h.log2s, c.at<float>(L.xfa), c.at<float>(L.xfb),
                       c.at<float>(L.rowterm), c.at<float>(L.colterm));
  } else {
    hipLaunchKernelGGL(k_stage_x_fp<double>, dim3(nb), dim3(256), 0, c.st, c.at<double>(L.xs), L.n_pad, L.d,
                       L.kd / 4, 0, h.log2s, c.at<double>(L.xfa), c.at<double>(L.xfb), c.at<double>(L.rowterm),
                       c.at<double>(L.colterm));
  }
  return hipGetLastError();
}

// distance operands of the derivative sweep (always q = r^2)
hipError_t launch_stage_x_bwd(const Ctx& c, const Hyper& h) {
  const Layout& L = *c.lay;
  (void)h;
  if (L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3) return hipSuccess;  // reused by the split sweep
  const unsigned nb = (unsigned)((L.n_pad + 255) / 256);
  if (L.bprec == GP_PREC_FP64)
    hipLaunchKernelGGL(k_stage_x_fp<double>, dim3(nb), dim3(256), 0, c.st, c.at<double>(L.xs), L.n_pad, L.d,
                       L.bkd / 4, 0, 0.0, c.at<double>(L.bxa), c.at<double>(L.bxb), c.at<double>(L.brt),
                       c.at<double>(L.bct));
  else
    hipLaunchKernelGGL(k_stage_x_fp<float>, dim3(nb), dim3(256), 0, c.st, c.at<double>(L.xs), L.n_pad, L.d,
                       L.bkd / 4, 0, 0.0, c.at<float>(L.bxa), c.at<float>(L.bxb), c.at<float>(L.brt),
                       c.at<float>(L.bct));
  return hipGetLastError();
}

TilePlan tile_plan(const Layout& L, int ncols) {
  static const int ok[] = {1, 2, 3, 4, 5, 6, 8, 12, 16};
  const int full = L.tp / 16;
  const bool split = L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3;
  ncols = std::max(1, std::min(ncols, L.tp));
  // 16 m + 1 columns: m tiles on the matrix cores, the last column on the vector ALU
  if (split && ncols % 16 == 1 && ncols / 16 <= 4) return TilePlan{ncols / 16, 1};
  for (int v : ok)
    if (16 * v >= ncols && v <= full) return TilePlan{v, 0};
  return TilePlan{full, 0};
}

hipError_t launch_stage_v(const Ctx& c, const double* V, int ldv, int ncols, const Hyper& h, const int* colmap,
                          TilePlan plan) {
  const Layout& L = *c.lay;
  (void)h;
  int ntt = plan.ntt;
  if (ntt < 0) ntt = L.tp / 16;
  const int xcol = plan.xc != 0 ? 16 * ntt : -1;
  if (plan.xc != 0 && L.prec != GP_PREC_BF16X3 && L.prec != GP_PREC_FP16X3) return hipErrorInvalidValue;
  const unsigned nbx = (unsigned)((L.n_pad + 255) / 256);
  if (L.prec == GP_PREC_FP16X3) {
    uint32_t* cm = c.at<uint32_t>(L.vscale);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, c.st, cm, L.tp);
    const int64_t rpb = 256;
    hipLaunchKernelGGL(k_colmax, dim3((unsigned)((L.n + rpb - 1) / rpb), (unsigned)((ncols + 63) / 64)), dim3(256), 0,
                       c.st, V, L.n, ldv, ncols, colmap, cm, rpb);
    const int64_t total = (L.n_pad / 32) * ntt * 64;
    if (total > 0)
      hipLaunchKernelGGL(k_stage_v_f16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.st, V, L.n, ldv,
                         ncols, colmap, L.n_pad, ntt, cm, c.at<u32x4>(L.vfrag));
    if (xcol >= 0)
      hipLaunchKernelGGL(k_stage_vx, dim3(nbx), dim3(256), 0, c.st, V, L.n, ldv, xcol, ncols, colmap, L.n_pad, cm,
                         c.at<float>(L.vx));
  } else if (L.prec == GP_PREC_BF16X3) {
    const int64_t total = (L.n_pad / 32) * ntt * 64;
    if (total > 0)
      hipLaunchKernelGGL(k_stage_v_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.st, V, L.n, ldv,
                         ncols, colmap, L.n_pad, ntt, plan.vp == 3 && bf16_v3_fits(ntt) ? 3 : 2,
                         c.at<u32x4>(L.vfrag));
    if (xcol >= 0)
      hipLaunchKernelGGL(k_stage_vx, dim3(nbx), dim3(256), 0, c.st, V, L.n, ldv, xcol, ncols, colmap, L.n_pad,
                         (const uint32_t*)nullptr, c.at<float>(L.vx));
  } else if (L.prec == GP_PREC_FP32) {
    const int64_t total = (L.n_pad / 16) * ntt * 256;
    hipLaunchKernelGGL(k_stage_v_fp<float>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.st, V, L.n, ldv,
                       ncols, colmap, L.n_pad, ntt, c.at<float>(L.vfrag));
  } else {
    const int64_t total = (L.n_pad / 16) * ntt * 256;
    hipLaunchKernelGGL(k_stage_v_fp<double>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.st, V, L.n,
                       ldv, ncols, colmap, L.n_pad, ntt, c.at<double>(L.vfrag));
  }
  return hipGetLastError();
}

hipError_t launch_khat_tiles(const Ctx& c, const Hyper& h, const int* nact, TilePlan plan) {
  const Layout& L = *c.lay;
  TileArgs ta;
  ta.n_pad = L.n_pad;
  ta.n_valid = L.n;
  ta.cols_per_split = L.cols_per_split;
  ta.tp = L.tp;
  ta.ntt = plan.ntt >= 0 ? plan.ntt : L.tp / 16;
  ta.xc = plan.xc;
  ta.vp = (plan.vp == 3 && bf16_v3_fits(ta.ntt)) ? 3 : 2;
  ta.s32 = (float)h.s;
  ta.s64 = h.s;
  ta.alpha32 = (float)h.alpha;
  ta.alpha64 = h.alpha;
  if (L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3) {
    // FP16X3 kernel values are 2^15 kappa: the tile carries no outputscale
    if (L.prec == GP_PREC_FP16X3) {
      ta.s32 = 32768.0f;
      return khat_tiles_f16x3(c, h, ta, nact);
    }
    return khat_tiles_bf16x3(c, h, ta, nact);
  }
  if (ta.xc != 0) return hipErrorInvalidValue;
  if (L.prec == GP_PREC_FP32) return khat_tiles_fp32(c, h, ta, nact);
  return khat_tiles_fp64(c, h, ta, nact);
}

hipError_t launch_khat_tiles_items(const Ctx& c, const Hyper& h, const ItemTable& it, const int* nact) {
  const Layout& L = *c.lay;
  if (it.nitems == 0) return hipSuccess;
  TileArgs ta;
  ta.n_pad = L.n_pad;
  ta.n_valid = L.n;
  ta.cols_per_split = L.cols_per_split;
  ta.tp = L.tp;
  ta.ntt = L.tp / 16;
  ta.xc = 0;
  ta.vp = 2;
  ta.s32 = 1.0f;
  ta.s64 = 1.0;
  ta.alpha32 = (float)h.alpha;
  ta.alpha64 = h.alpha;
  if (L.prec == GP_PREC_FP32) return khat_tiles_fp32(c, h, ta, nact, it);
  if (L.prec == GP_PREC_FP64) return khat_tiles_fp64(c, h, ta, nact, it);
  return hipErrorInvalidValue;
}

hipError_t launch_khat_reduce(const Ctx& c, const double* V, int ldv, double* W, int ldw, int ncols, const Hyper& h,
                              double* dot_part, const int* nact, const int* colmap, int ldpart) {
  if (ldpart <= 0) ldpart = ncols;
  const Layout& L = *c.lay;
  const dim3 nb((unsigned)((L.n + 63) / 64), (unsigned)((ncols + kRedCols - 1) / kRedCols));
  const bool f16 = L.prec == GP_PREC_FP16X3;
  const uint32_t* cm = f16 ? c.at<uint32_t>(L.vscale) : nullptr;
  const double fac_s = f16 ? h.s / 32768.0 : 1.0;
  if (L.prec == GP_PREC_FP64)
    hipLaunchKernelGGL(k_khat_reduce<double>, nb, dim3(kRedThreads), 0, c.st, c.at<double>(L.wpart), L.nsplit, L.n_pad,
                       L.tp, V, ldv, W, ldw, L.n, ncols, colmap, ldpart, h.s2, dot_part, nact, cm, fac_s);
  else
    hipLaunchKernelGGL(k_khat_reduce<float>, nb, dim3(kRedThreads), 0, c.st, c.at<float>(L.wpart), L.nsplit, L.n_pad,
                       L.tp, V, ldv, W, ldw, L.n, ncols, colmap, ldpart, h.s2, dot_part, nact, cm, fac_s);
  return hipGetLastError();
}

#endif  // part 0

}  // namespace gpmll
