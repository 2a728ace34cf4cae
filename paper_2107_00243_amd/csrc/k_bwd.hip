// Gradient of the log-likelihood estimate (Algorithm 2; Eq. 2; derivative
// decomposition of Section 3.3), reusing the forward solves:
//   a_i = K_hat^-1 b_i (CG solutions), c_i = P_hat^-1 b_i (first preconditioned
//   residuals), u = K_hat^-1 y.
//   grad = sum_pq M_pq dK_hat_pq - 1/2 tr(P_hat^-1 dP_hat) + 1/(2 ell) sum_i c_i^T dP_hat c_i
// with M = A' C'^T, A' = [u | a_1 .. a_ell], C' = [u/2 | -c_1/(2 ell) .. -c_ell/(2 ell)].
//
// (1) Kernel-derivative sweep: every n x n tile is rebuilt on the fly (never
//     stored).  Per tile: the distance MFMA, the M tile (MFMA with inner
//     dimension t), W = s g(r) . M and M . kappa in registers, then one more MFMA
//     per row against [1 | x~_q | x~_q^2] so that, per row p,
//       sum_q W_pq (x~_pj - x~_qj)^2 = x~_pj^2 rowsum(W)_p + (W X~^2)_pj - 2 x~_pj (W X~)_pj,
//     which gives the lengthscale terms with every accumulator row-local.
//     The outputscale term is sum_pq M_pq kappa_pq; the noise term is tr(M).
// (2) Preconditioner terms with frozen pivots (rank-k partial pivoted Cholesky =
//     Nystrom on its pivots S): with G = L C^-1 L_S^-1, H = L_S^-T (I - sigma^2 C^-1)
//     L_S^-1, U = L_S^-T L^T [c_1..c_ell], the preconditioner part of the gradient
//     for every kernel parameter is
//       sum_{p,q} Omega_pq dK_{p,S_q} + sum_{q,r} Psi_qr dK_{S_q,S_r},
//       Omega = -G + U-weighted solves / ell,  Psi = H/2 - U U^T / (2 ell),
//     and for sigma^2: -1/2 ((n - k)/sigma^2 + tr C^-1) + 1/(2 ell) sum_i |c_i|^2
//     (trace of P_hat^-1 dP_hat by the matrix inversion lemma, supplement S3.3).
#include "gpmll_impl.h"

#include <utility>
#include "small_dense.h"

namespace gpmll {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct BwMfma;
template <>
struct BwMfma<float> {
  typedef f32x4 acc_t;
  __device__ static acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct BwMfma<double> {
  typedef f64x4 acc_t;
  __device__ static acc_t mfma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

constexpr int kMaxBT = 5;  // [1 | x~ | x~^2] padded to 16-column tiles, d <= 32

// Row (within a 16-row block) of accumulator slot v in lane group g for the
// 16x16x4 MFMA outputs: FP32 rows 4g + v, FP64 rows g + 4v.
template <typename T>
__device__ constexpr int acc_row_b(int g, int v) {
  return sizeof(T) == 8 ? g + 4 * v : 4 * g + v;
}

// C' = [u/2 | -c_i / (2 ell) | 0]
__global__ void k_cprime(const double* __restrict__ Xs, const double* __restrict__ Z0, int64_t n, int64_t n_pad, int tp,
                         int ell, double* __restrict__ Cp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pad * tp) return;
  const int64_t i = e / tp;
  const int c = (int)(e % tp);
  double v = 0.0;
  if (i < n) {
    if (c == 0) v = 0.5 * Xs[e];
    else if (c <= ell) v = -Z0[e] / (2.0 * ell);
  }
  Cp[e] = v;
}

// rows of a row-major (n_pad x ld) FP64 array as 16 x 4 MFMA fragments:
// frag[(tile * nk + kc) * 64 + lane] = M[tile*16 + lane%16][kc*4 + lane/16]
template <typename T>
__global__ void k_stage_rows16x4(const double* __restrict__ M, int64_t n_pad, int ld, int ncols, int nk,
                                 T* __restrict__ frag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (n_pad / 16) * nk * 64) return;
  const int lane = (int)(e % 64);
  const int kc = (int)((e / 64) % nk);
  const int64_t tile = e / (64 * nk);
  const int col = kc * 4 + lane / 16;
  frag[e] = col < ncols ? (T)M[(tile * 16 + lane % 16) * ld + col] : (T)0;
}

// [1 | x~ | x~^2] as B fragments: frag[((j16 * nbt + tt) * 4 + v) * 64 + lane] = Xaug[j16*16 + 4(lane/16) + v][tt*16 + lane%16]
template <typename T>
__global__ void k_stage_xaug(const double* __restrict__ xs, int64_t n, int64_t n_pad, int d, int nbt,
                             T* __restrict__ frag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (n_pad / 16) * nbt * 256) return;
  const int lane = (int)(e % 64);
  const int v = (int)((e / 64) % 4);
  const int tt = (int)((e / 256) % nbt);
  const int64_t j16 = e / (256 * nbt);
  const int64_t q = j16 * 16 + acc_row_b<T>(lane / 16, v);
  const int col = tt * 16 + lane % 16;
  double val = 0.0;
  if (q < n) {
    if (col == 0) val = 1.0;
    else if (col <= d) val = xs[q * d + col - 1];
    else if (col <= 2 * d) {
      const double x = xs[q * d + col - 1 - d];
      val = x * x;
    }
  }
  frag[e] = (T)val;
}

struct BwdArgs {
  int64_t n_pad, n;
  int64_t cols_per_split;
  int nk4, nkt, nbt, ow;  // distance K/4, t/4, [1|x|x^2] tiles, output row width
  double s;
  double alpha;           // rational quadratic shape
};

template <typename T>
__device__ inline void kappa_g_t(int kind, T q, T s, T alpha, T* kap, T* sg) {
  if constexpr (sizeof(T) == 8) {
    double k, g;
    kappa_g64(kind, q > 0.0 ? q : 0.0, &k, &g, alpha);
    *kap = k;
    *sg = s * g;
  } else {
    const float log2e = 1.4426950408889634f;
    const float q0 = fmaxf(q, 0.0f);
    if (kind == GP_KERNEL_RATQUAD) {
      const float b = fmaf(q0, 0.5f / alpha, 1.0f);
      const float k = __builtin_amdgcn_exp2f(-alpha * __builtin_amdgcn_logf(b));
      *kap = k;
      *sg = s * k * __builtin_amdgcn_rcpf(b);
    } else if (kind == GP_KERNEL_RBF) {
      const float e = __builtin_amdgcn_exp2f(-0.5f * log2e * q0);
      *kap = e;
      *sg = s * e;
    } else if (kind == GP_KERNEL_MATERN32) {
      const float a = 1.7320508075688772f;
      const float r = __builtin_amdgcn_sqrtf(q0);
      const float e = __builtin_amdgcn_exp2f(-a * log2e * r);
      *kap = fmaf(a, r, 1.0f) * e;
      *sg = s * 3.0f * e;
    } else {
      const float a = 2.23606797749979f;
      const float r = __builtin_amdgcn_sqrtf(q0);
      const float e = __builtin_amdgcn_exp2f(-a * log2e * r);
      *kap = fmaf(5.0f / 3.0f, q0, fmaf(a, r, 1.0f)) * e;
      *sg = s * (5.0f / 3.0f) * fmaf(a, r, 1.0f) * e;
    }
  }
}

// One wave per 16 rows, four waves per workgroup; one column range per blockIdx.y.
// The distance here is always r^2 (x'_A = -sqrt2 x~, x'_B = sqrt2 x~, terms |x~|^2).
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_bwd_tiles(const T* __restrict__ xfa, const T* __restrict__ xfb,
                                                   const T* __restrict__ rowterm, const T* __restrict__ colterm,
                                                   const T* __restrict__ afrag, const T* __restrict__ cfrag,
                                                   const T* __restrict__ xaug, T* __restrict__ out, BwdArgs a) {
  typedef typename BwMfma<T>::acc_t acc_t;
  extern __shared__ char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int A_E = a.nk4 * 64, C_E = a.nkt * 64, X_E = a.nbt * 256, CT_E = 16;
  const int STAGE = A_E + C_E + X_E + CT_E;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t c_begin = (int64_t)blockIdx.y * a.cols_per_split;
  const int64_t c_end = min(a.n_pad, c_begin + a.cols_per_split);
  if (c_begin >= c_end) return;
  const T r = rowterm[row0 + li];
  const acc_t rt = acc_t{r, r, r, r};
  acc_t acc1[kMaxBT];
  acc_t acc2 = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int tt = 0; tt < kMaxBT; ++tt) acc1[tt] = acc_t{0, 0, 0, 0};
  const T* arow = afrag + (row0 / 16) * a.nkt * 64;
  const T* xbrow = xfb + (row0 / 16) * a.nk4 * 64;
  const T one = (li == 0) ? (T)1 : (T)0;

  for (int64_t c = c_begin; c < c_end; c += 16) {
    __syncthreads();
    for (int e = tid; e < STAGE; e += 256) {
      T v;
      if (e < A_E) v = xfa[(c / 16) * A_E + e];
      else if (e < A_E + C_E) v = cfrag[(c / 16) * C_E + (e - A_E)];
      else if (e < A_E + C_E + X_E) v = xaug[(c / 16) * X_E + (e - A_E - C_E)];
      else v = colterm[c + (e - A_E - C_E - X_E)];
      lds[e] = v;
    }
    __syncthreads();
    const T* A = lds;
    const T* Cf = lds + A_E;
    const T* Xf = Cf + C_E;
    const T* ct = Xf + X_E;
    acc_t dd = rt;
    for (int kc = 0; kc < a.nk4; ++kc) dd = BwMfma<T>::mfma(A[kc * 64 + lane], xbrow[kc * 64 + lane], dd);
    acc_t mm = acc_t{0, 0, 0, 0};
    for (int kc = 0; kc < a.nkt; ++kc) mm = BwMfma<T>::mfma(Cf[kc * 64 + lane], arow[kc * 64 + lane], mm);
    const int64_t p = row0 + li;
    T wv[4], mk[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t q = c + acc_row_b<T>(g, v);
      T kap, sg;
      kappa_g_t<T>(KIND, dd[v] + ct[acc_row_b<T>(g, v)], (T)a.s, (T)a.alpha, &kap, &sg);
      if (p == q) {
        kap = (T)1;
        sg = (T)0;  // the scaled difference is exactly zero on the diagonal
      }
      wv[v] = sg * mm[v];
      mk[v] = kap * mm[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int tt = 0; tt < kMaxBT; ++tt)
        if (tt < a.nbt) acc1[tt] = BwMfma<T>::mfma(wv[v], Xf[(tt * 4 + v) * 64 + lane], acc1[tt]);
      acc2 = BwMfma<T>::mfma(mk[v], one, acc2);
    }
  }
  T* o = out + (int64_t)blockIdx.y * a.n_pad * a.ow;
#pragma unroll
  for (int tt = 0; tt < kMaxBT; ++tt)
    if (tt < a.nbt)
#pragma unroll
      for (int v = 0; v < 4; ++v) o[(row0 + acc_row_b<T>(g, v)) * a.ow + tt * 16 + li] = acc1[tt][v];
  if (li == 0)
#pragma unroll
    for (int v = 0; v < 4; ++v) o[(row0 + acc_row_b<T>(g, v)) * a.ow + a.nbt * 16] = acc2[v];
}

// per-row combination and per-block partials: part[b][j] (j < d) lengthscale terms, part[b][d] outputscale
template <typename T>
__global__ void k_bwd_rows(const T* __restrict__ rows, int nsplit, int64_t n, int64_t n_pad, int ow, int nbt, int d,
                           const double* __restrict__ xs, Hyper h, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc[GP_MAX_D + 1];
  for (int j = 0; j <= d; ++j) acc[j] = 0.0;
  if (p < n) {
    double rs = 0.0, mk = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      const T* r = rows + ((int64_t)s * n_pad + p) * ow;
      rs += (double)r[0];
      mk += (double)r[nbt * 16];
    }
    for (int j = 0; j < d; ++j) {
      double wx = 0.0, wx2 = 0.0;
      for (int s = 0; s < nsplit; ++s) {
        const T* r = rows + ((int64_t)s * n_pad + p) * ow;
        wx += (double)r[1 + j];
        wx2 += (double)r[1 + d + j];
      }
      const double x = xs[p * d + j];
      acc[j] = (x * x * rs + wx2 - 2.0 * x * wx) * h.inv_ls[j];
    }
    acc[d] = mk;
  }
  for (int j = 0; j <= d; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (GP_MAX_D + 1) + j] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BF16x3 derivative sweep.  Same tile walk as the BF16x3 K_hat V kernel and the
// same staged distance operands (q = log2 k for RBF, q = r^2 for Matern).  The M
// tile M^T[q][p] = C'_q . A'_p uses the split (hi, hi, lo) x (hi, lo, hi) along the
// contraction; W = s g M and M kappa come out in the distance layout (lane = row
// p, 4 + 4 columns q), so W feeds W [x~ | x~^2] on MFMA as the A operand (same
// column permutation as the K_hat V kernel) while rowsum(W) and sum_q M kappa
// are per-lane sums finished across the four lane groups at the end.
// ---------------------------------------------------------------------------

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t bw_pack_bf16(float a, float b) {
  f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ inline void bw_split_pair(float a, float b, uint32_t* hi, uint32_t* lo) {
  uint32_t h = bw_pack_bf16(a, b);
  float ha = __builtin_bit_cast(float, h << 16);
  float hb = __builtin_bit_cast(float, h & 0xffff0000u);
  *hi = h;
  *lo = bw_pack_bf16(a - ha, b - hb);
}

// rows of an FP64 (n_pad x ld) array as 3-piece BF16 MFMA fragments along K:
// A side [hi | hi | lo], B side [hi | lo | hi], each piece tq wide, K padded to 32 * nkm
__global__ void k_stage_rows_bf16x3(const double* __restrict__ M, int64_t n_pad, int ld, int ncols, int tq, int nkm,
                                    int bside, u32x4* __restrict__ frag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (tile, kc, lane)
  if (e >= (n_pad / 16) * nkm * 64) return;
  const int lane = (int)(e % 64);
  const int kc = (int)((e / 64) % nkm);
  const int64_t tile = e / (64 * nkm);
  const int64_t row = tile * 16 + lane % 16;
  uint32_t w[4];
  for (int q = 0; q < 4; ++q) {
    uint16_t hv[2];
    for (int h2 = 0; h2 < 2; ++h2) {
      const int k = kc * 32 + (lane / 16) * 8 + q * 2 + h2;
      const int seg = k / tq, col = k % tq;
      uint16_t out = 0;
      if (seg < 3 && col < ncols) {
        const double x = M[row * ld + col];
        uint32_t hh, ll;
        bw_split_pair((float)x, 0.0f, &hh, &ll);
        // lo from the FP64 residual
        const double rem = x - (double)__builtin_bit_cast(float, (hh & 0xffffu) << 16);
        const uint16_t hi16 = (uint16_t)(hh & 0xffffu);
        const uint16_t lo16 = (uint16_t)(bw_pack_bf16((float)rem, 0.0f) & 0xffffu);
        const bool use_hi = bside ? (seg != 1) : (seg != 2);
        out = use_hi ? hi16 : lo16;
      }
      hv[h2] = out;
    }
    w[q] = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
  }
  frag[e] = u32x4{w[0], w[1], w[2], w[3]};
}

// [x~ | x~^2] (2d columns, padded to 16 * nxt) as hi/lo B fragments with the
// K_hat V kernel's column permutation: fragment (jb, tt, piece) lane l holds rows
// jb*32 + perm(l/16, s), perm(g, s) = 4g + s (s < 4) or 16 + 4g + s - 4
__global__ void k_stage_xaug_bf16(const double* __restrict__ xs, int64_t n, int64_t n_pad, int d, int nxt,
                                  u32x4* __restrict__ frag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (jb, tt, lane)
  if (e >= (n_pad / 32) * nxt * 64) return;
  const int lane = (int)(e % 64);
  const int tt = (int)((e / 64) % nxt);
  const int64_t jb = e / (64 * nxt);
  const int g = lane / 16, col = tt * 16 + lane % 16;
  uint32_t h[4], l[4];
  for (int w = 0; w < 4; ++w) {
    double v2[2];
    for (int h2 = 0; h2 < 2; ++h2) {
      const int s = 2 * w + h2;
      const int64_t q = jb * 32 + (s < 4 ? 4 * g + s : 16 + 4 * g + (s - 4));
      double val = 0.0;
      if (q < n) {
        if (col < d) val = xs[q * d + col];
        else if (col < 2 * d) {
          const double x = xs[q * d + col - d];
          val = x * x;
        }
      }
      v2[h2] = val;
    }
    const uint32_t hh = bw_pack_bf16((float)v2[0], (float)v2[1]);
    const double ra = v2[0] - (double)__builtin_bit_cast(float, hh << 16);
    const double rb = v2[1] - (double)__builtin_bit_cast(float, hh & 0xffff0000u);
    h[w] = hh;
    l[w] = bw_pack_bf16((float)ra, (float)rb);
  }
  frag[((jb * nxt + tt) * 2 + 0) * 64 + lane] = u32x4{h[0], h[1], h[2], h[3]};
  frag[((jb * nxt + tt) * 2 + 1) * 64 + lane] = u32x4{l[0], l[1], l[2], l[3]};
}

struct BwdBfArgs {
  int64_t n_pad;
  int64_t cols_per_split;
  int ow, nbt;
  float s, inv_s;
  float rbf_sg, rbf_kap;  // RBF: s g = rbf_sg * exp2(q), kappa = rbf_kap * exp2(q)
  float alpha;            // rational quadratic shape
};

template <int KIND>
__device__ inline void bw_map(float q, float s, float rbf_sg, float rbf_kap, float alpha, float* kap, float* sg) {
  if (KIND == GP_KERNEL_RATQUAD) {
    // split-precision staging: q = r^2 / (2 alpha); kappa = b^-alpha, g = b^(-alpha-1), b = 1 + q
    const float b = 1.0f + fabsf(q);
    const float k = __builtin_amdgcn_exp2f(-alpha * __builtin_amdgcn_logf(b));
    *kap = k;
    *sg = s * k * __builtin_amdgcn_rcpf(b);
  } else if (KIND == GP_KERNEL_RBF) {
    const float k = __builtin_amdgcn_exp2f(q);  // q: log2 of the staged kernel value
    *sg = k * rbf_sg;
    *kap = k * rbf_kap;
  } else {
    // split-precision staging: q = rho^2 with rho = a log2(e) r, a r = ln2 rho
    const float ln2 = 0.6931471805599453f;
    const float rho = __builtin_amdgcn_sqrtf(fabsf(q));
    const float e = __builtin_amdgcn_exp2f(-rho);
    const float ar = ln2 * rho;
    if (KIND == GP_KERNEL_MATERN32) {
      *kap = (1.0f + ar) * e;
      *sg = s * 3.0f * e;
    } else {
      *kap = fmaf(ar * ar, 1.0f / 3.0f, 1.0f + ar) * e;
      *sg = s * (5.0f / 3.0f) * (1.0f + ar) * e;
    }
  }
}

// One step's operands of the split-precision derivative sweep, global -> LDS
// without registers (each wave instruction moves one contiguous 1 KB chunk):
// [A fragments 2 NKC | C' fragments 2 NKM | [x~ | x~^2] fragments 2 NXT | column
// terms (units 0-7 of the last chunk)].  The chunk walk is wave-uniform.
template <int NKC, int NKM, int NXT>
__device__ __forceinline__ void bwd_issue_stage(u32x4* dst, const u32x4* __restrict__ xfa,
                                                const u32x4* __restrict__ cfr, const u32x4* __restrict__ xau,
                                                const float* __restrict__ colterm, int64_t c, int wave, int lane) {
  constexpr int NA = 2 * NKC, NC = 2 * NKM, NX = 2 * NXT;
  constexpr int NCH = NA + NC + NX + 1;
  for (int ch = __builtin_amdgcn_readfirstlane(wave); ch < NCH; ch += 4) {
    const u32x4* src;
    if (ch < NA) src = xfa + (c / 16) * NKC * 64 + ch * 64 + lane;
    else if (ch < NA + NC) src = cfr + (c / 16) * NKM * 64 + (ch - NA) * 64 + lane;
    else if (ch < NA + NC + NX) src = xau + (c / 32) * NXT * 128 + (ch - NA - NC) * 64 + lane;
    else src = reinterpret_cast<const u32x4*>(colterm + c) + (lane < 8 ? lane : 7);
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(dst + ch * 64), 16, 0, 0);
  }
}

constexpr int kLdsBytesPerCu = 163840;

template <int KIND, int NKC, int NKM, int NXT, int RG>
__global__ __launch_bounds__(256, 2) void k_bwd_bf16(const u32x4* __restrict__ xfa, const u32x4* __restrict__ xfb,
                                                     const float* __restrict__ rowterm,
                                                     const float* __restrict__ colterm,
                                                     const u32x4* __restrict__ afr, const u32x4* __restrict__ cfr,
                                                     const u32x4* __restrict__ xau, float* __restrict__ out,
                                                     BwdBfArgs a) {
  constexpr int A_U = 2 * NKC * 64, C_U = 2 * NKM * 64, X_U = NXT * 2 * 64;
  // two-stage ring filled by global -> LDS loads (the column terms take a whole
  // 64-unit chunk there) while two stages keep two workgroups per CU; otherwise
  // one stage filled through registers
  constexpr int STAGE_RING = A_U + C_U + X_U + 64;
  constexpr bool RING = 2 * STAGE_RING * 16 <= kLdsBytesPerCu / 2;
  constexpr int T_U = RING ? 64 : 8;
  constexpr int STAGE = A_U + C_U + X_U + T_U;
  constexpr int PER = (STAGE + 255) / 256;
  __shared__ u32x4 lds[RING ? 2 : 1][STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * RG) + wave * (16 * RG);
  const int64_t c_begin = (int64_t)blockIdx.y * a.cols_per_split;
  const int64_t c_end = min(a.n_pad, c_begin + a.cols_per_split);
  if (c_begin >= c_end) return;
  u32x4 xbv[RG][NKC], abv[RG][NKM];
  f32x4 rt[RG];
  f32x4 acc[RG][NXT];
  float rs[RG], mk[RG];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) xbv[rg][kc] = xfb[((row0 / 16 + rg) * NKC + kc) * 64 + lane];
#pragma unroll
    for (int kc = 0; kc < NKM; ++kc) abv[rg][kc] = afr[((row0 / 16 + rg) * NKM + kc) * 64 + lane];
    const float r = rowterm[row0 + rg * 16 + li];
    rt[rg] = f32x4{r, r, r, r};
#pragma unroll
    for (int tt = 0; tt < NXT; ++tt) acc[rg][tt] = f32x4{0.f, 0.f, 0.f, 0.f};
    rs[rg] = 0.f;
    mk[rg] = 0.f;
  }
  const int nsteps = (int)((c_end - c_begin) / 32);
  if constexpr (RING) {
    // step s sits in lds[s & 1]; iteration j loads step j + 1 into the buffer step
    // j - 1 left, then works on step j
    bwd_issue_stage<NKC, NKM, NXT>(lds[0], xfa, cfr, xau, colterm, c_begin, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int j = 0; j < nsteps; ++j) {
      const int64_t c = c_begin + (int64_t)j * 32;
      if (j + 1 < nsteps)
        bwd_issue_stage<NKC, NKM, NXT>(lds[(j + 1) & 1], xfa, cfr, xau, colterm, c + 32, wave, lane);
      const u32x4* base = lds[j & 1];
      const u32x4* A = base;
      const u32x4* Cf = A + A_U;
      const u32x4* Xf = Cf + C_U;
      const float* ct = reinterpret_cast<const float*>(Xf + X_U);
      const bool diag = (c + 32 > row0) && (c < row0 + 16 * RG);
      u32x4 wh[RG], wl[RG];
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
        for (int js = 0; js < 2; ++js) {
          f32x4 dd = rt[rg];
#pragma unroll
          for (int kc = 0; kc < NKC; ++kc)
            dd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[(js * NKC + kc) * 64 + lane]),
                                                         __builtin_bit_cast(bf16x8, xbv[rg][kc]), dd, 0, 0, 0);
          f32x4 mm = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < NKM; ++kc)
            mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, Cf[(js * NKM + kc) * 64 + lane]),
                                                         __builtin_bit_cast(bf16x8, abv[rg][kc]), mm, 0, 0, 0);
          const f32x4 ctv = *reinterpret_cast<const f32x4*>(ct + js * 16 + 4 * g);
          float wv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float kap, sg;
            bw_map<KIND>(dd[v] + ctv[v], a.s, a.rbf_sg, a.rbf_kap, a.alpha, &kap, &sg);
            if (diag && row0 + rg * 16 + li == c + js * 16 + 4 * g + v) {
              kap = 1.0f;
              sg = 0.0f;
            }
            wv[v] = sg * mm[v];
            rs[rg] += wv[v];
            mk[rg] += kap * mm[v];
          }
          uint32_t h0, l0, h1, l1;
          bw_split_pair(wv[0], wv[1], &h0, &l0);
          bw_split_pair(wv[2], wv[3], &h1, &l1);
          wh[rg][2 * js] = h0;
          wh[rg][2 * js + 1] = h1;
          wl[rg][2 * js] = l0;
          wl[rg][2 * js + 1] = l1;
        }
      }
#pragma unroll
      for (int tt = 0; tt < NXT; ++tt) {
        const bf16x8 xh = __builtin_bit_cast(bf16x8, Xf[(tt * 2 + 0) * 64 + lane]);
        const bf16x8 xl = __builtin_bit_cast(bf16x8, Xf[(tt * 2 + 1) * 64 + lane]);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
          const bf16x8 h = __builtin_bit_cast(bf16x8, wh[rg]);
          const bf16x8 l = __builtin_bit_cast(bf16x8, wl[rg]);
          acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, xh, acc[rg][tt], 0, 0, 0);
          acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, xl, acc[rg][tt], 0, 0, 0);
          acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, xh, acc[rg][tt], 0, 0, 0);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  } else {
    u32x4* lds1 = lds[0];
    for (int64_t c = c_begin; c < c_end; c += 32) {
      u32x4 pre[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        int e = tid + q * 256;
        e = e < STAGE ? e : STAGE - 1;
        const u32x4* src;
        if (e < A_U) src = xfa + (c / 16) * NKC * 64 + e;
        else if (e < A_U + C_U) src = cfr + (c / 16) * NKM * 64 + (e - A_U);
        else if (e < A_U + C_U + X_U) src = xau + (c / 32) * NXT * 128 + (e - A_U - C_U);
        else src = reinterpret_cast<const u32x4*>(colterm + c) + (e - A_U - C_U - X_U);
        pre[q] = *src;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * 256;
        if (e < STAGE) lds1[e] = pre[q];
      }
      __syncthreads();
      const u32x4* A = lds1;
      const u32x4* Cf = A + A_U;
      const u32x4* Xf = Cf + C_U;
      const float* ct = reinterpret_cast<const float*>(Xf + X_U);
      const bool diag = (c + 32 > row0) && (c < row0 + 16 * RG);
      u32x4 wh[RG], wl[RG];
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
        for (int js = 0; js < 2; ++js) {
          f32x4 dd = rt[rg];
#pragma unroll
          for (int kc = 0; kc < NKC; ++kc)
            dd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[(js * NKC + kc) * 64 + lane]),
                                                         __builtin_bit_cast(bf16x8, xbv[rg][kc]), dd, 0, 0, 0);
          f32x4 mm = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < NKM; ++kc)
            mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, Cf[(js * NKM + kc) * 64 + lane]),
                                                         __builtin_bit_cast(bf16x8, abv[rg][kc]), mm, 0, 0, 0);
          const f32x4 ctv = *reinterpret_cast<const f32x4*>(ct + js * 16 + 4 * g);
          float wv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float kap, sg;
            bw_map<KIND>(dd[v] + ctv[v], a.s, a.rbf_sg, a.rbf_kap, a.alpha, &kap, &sg);
            if (diag && row0 + rg * 16 + li == c + js * 16 + 4 * g + v) {
              kap = 1.0f;
              sg = 0.0f;
            }
            wv[v] = sg * mm[v];
            rs[rg] += wv[v];
            mk[rg] += kap * mm[v];
          }
          uint32_t h0, l0, h1, l1;
          bw_split_pair(wv[0], wv[1], &h0, &l0);
          bw_split_pair(wv[2], wv[3], &h1, &l1);
          wh[rg][2 * js] = h0;
          wh[rg][2 * js + 1] = h1;
          wl[rg][2 * js] = l0;
          wl[rg][2 * js + 1] = l1;
        }
      }
#pragma unroll
      for (int tt = 0; tt < NXT; ++tt) {
        const bf16x8 xh = __builtin_bit_cast(bf16x8, Xf[(tt * 2 + 0) * 64 + lane]);
        const bf16x8 xl = __builtin_bit_cast(bf16x8, Xf[(tt * 2 + 1) * 64 + lane]);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
          const bf16x8 h = __builtin_bit_cast(bf16x8, wh[rg]);
          const bf16x8 l = __builtin_bit_cast(bf16x8, wl[rg]);
          acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, xh, acc[rg][tt], 0, 0, 0);
          acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, xl, acc[rg][tt], 0, 0, 0);
          acc[rg][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, xh, acc[rg][tt], 0, 0, 0);
        }
      }
    }
  }
  float* o = out + (int64_t)blockIdx.y * a.n_pad * a.ow;
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
    // [x~ | x~^2] products land in columns 1 .. 2d of the row record
#pragma unroll
    for (int tt = 0; tt < NXT; ++tt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = tt * 16 + li;
        if (col + 1 < a.nbt * 16) o[(row0 + rg * 16 + 4 * g + v) * a.ow + 1 + col] = acc[rg][tt][v];
      }
    // per-lane partial sums over q: finish across the four lane groups (same row p = li)
    float r1 = rs[rg], m1 = mk[rg];
    r1 += __shfl_xor(r1, 16);
    r1 += __shfl_xor(r1, 32);
    m1 += __shfl_xor(m1, 16);
    m1 += __shfl_xor(m1, 32);
    if (g == 0) {
      o[(row0 + rg * 16 + li) * a.ow + 0] = r1;
      o[(row0 + rg * 16 + li) * a.ow + a.nbt * 16] = m1;
    }
  }
}

// ---------------------------------------------------------------------------
// Preconditioner derivative terms
// ---------------------------------------------------------------------------

__global__ void k_pg_small(const double* __restrict__ L, const int32_t* __restrict__ piv, const int* __restrict__ kpp,
                           int64_t n, int k, const double* __restrict__ Cinv, const double* __restrict__ ltrc, int tp,
                           int ell, double s2, double* __restrict__ LSinv, double* __restrict__ Gk,
                           double* __restrict__ Psi, double* __restrict__ U, double* __restrict__ tmp) {
  pg_small_body(L, piv, kpp, n, k, Cinv, ltrc, tp, ell, s2, LSinv, Gk, Psi, U, tmp);
}

// Generic FP64 tile product C(i, j) = alpha * sum_m A(i, m) B(m, j) + beta * C(i, j)
// with element strides (64 x 64 tiles, 4 x 4 per thread).  M, N, K are runtime sizes.
__global__ __launch_bounds__(256) void k_gemm64(int64_t M, int N, int K, const double* __restrict__ A, int64_t sAi,
                                                int64_t sAm, const double* __restrict__ B, int64_t sBm, int64_t sBj,
                                                double* __restrict__ C, int64_t sCi, int64_t sCj, double alpha,
                                                double beta, const int* __restrict__ ndyn,
                                                const int* __restrict__ kdyn) {
  __shared__ double As[16][65], Bs[16][65];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  const int Kr = kdyn ? min(K, *kdyn) : K;
  const int Nr = ndyn ? min(N, *ndyn) : N;
  if (j0 >= Nr) return;
  double acc[4][4] = {};
  for (int mb = 0; mb < Kr; mb += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int mm = e / 64, rr = e % 64;
      const int64_t i = i0 + rr;
      As[mm][rr] = (i < M && mb + mm < Kr) ? A[i * sAi + (int64_t)(mb + mm) * sAm] : 0.0;
      const int j = j0 + rr;
      Bs[mm][rr] = (mb + mm < Kr && j < Nr) ? B[(int64_t)(mb + mm) * sBm + (int64_t)j * sBj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) {
      double av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = As[mm][ty * 4 + q];
        bv[q] = Bs[mm][tx * 4 + q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t i = i0 + ty * 4 + x;
    if (i >= M) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int j = j0 + tx * 4 + y;
      if (j >= Nr) continue;
      double* cp = C + i * sCi + (int64_t)j * sCj;
      *cp = alpha * acc[x][y] + (beta != 0.0 ? beta * *cp : 0.0);
    }
  }
}

// sum over (row point x_p, pivot point x_{S_q}) of w * dK: rows p < n use Omega[:, q],
// rows n + q' use Psi[q'][:]; part[b][j] lengthscale terms (already / ls_j), part[b][d] outputscale
__global__ void k_pg_contract(const double* __restrict__ xs, const int32_t* __restrict__ piv,
                              const int* __restrict__ kpp, int64_t n, int k, const double* __restrict__ Omega,
                              const double* __restrict__ Psi, Hyper h, int mode, double* __restrict__ part) {
  __shared__ double red[256];
  const int kp = *kpp;
  const int d = h.d;
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc[GP_MAX_D + 1];
  for (int j = 0; j <= d; ++j) acc[j] = 0.0;
  if (row < n + kp) {
    const int64_t pi = row < n ? row : (int64_t)piv[row - n];
    double xp[GP_MAX_D];
    for (int j = 0; j < d; ++j) xp[j] = xs[pi * d + j];
    for (int q = 0; q < kp; ++q) {
      const double w = row < n ? Omega[(int64_t)q * n + row] : Psi[(row - n) * k + q];
      const int64_t sq = piv[q];
      double r2 = 0.0;
      double df2[GP_MAX_D];
      for (int j = 0; j < d; ++j) {
        const double df = xp[j] - xs[sq * d + j];
        df2[j] = df * df;
        r2 += df2[j];
      }
      double kap, g;
      kappa_g64(h.kind, r2, &kap, &g, h.alpha);
      const double wg = w * h.s * g;
      if (mode == 0)
        for (int j = 0; j < d; ++j) acc[j] += wg * df2[j];
      acc[d] += w * kap;
    }
    for (int j = 0; j < d; ++j) acc[j] *= h.inv_ls[j];
  }
  for (int j = 0; j <= d; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (GP_MAX_D + 1) + j] = red[0];
    __syncthreads();
  }
}

// Random Fourier feature preconditioner: sum over rows p and features of
// Omega * dZ with the frequencies W fixed.  For lengthscale q,
//   d cos(Phi_pj) = Z_{p,m+j} w_jq x~_pq / ls_q,  d sin(Phi_pj) = -Z_{p,j} w_jq x~_pq / ls_q
// (dPhi_pj / dls_q = -w_jq x~_pq / ls_q, amplitude folded into Z), so the term is
// (x~_pq / ls_q) sum_j w_jq (Omega_pj Z_{p,m+j} - Omega_{p,m+j} Z_pj); the outputscale
// term is sum_j Omega_pj Z_pj / (2 s).  part[b][q] (q < d) and part[b][d] as k_pg_contract.
__global__ void k_rff_contract(const double* __restrict__ xs, int64_t n, int m, const double* __restrict__ W,
                               const double* __restrict__ Omega, const double* __restrict__ Z, Hyper h, int mode,
                               double* __restrict__ part) {
  __shared__ double red[256];
  const int d = h.d;
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc[GP_MAX_D + 1];
  for (int j = 0; j <= d; ++j) acc[j] = 0.0;
  if (row < n) {
    double os = 0.0;
    for (int j = 0; j < m; ++j) {
      const double oc = Omega[(int64_t)j * n + row], osn = Omega[(int64_t)(m + j) * n + row];
      const double zc = Z[(int64_t)j * n + row], zs = Z[(int64_t)(m + j) * n + row];
      os += oc * zc + osn * zs;
      if (mode == 0) {
        const double hj = oc * zs - osn * zc;
        for (int q = 0; q < d; ++q) acc[q] = fma(hj, W[j * d + q], acc[q]);
      }
    }
    for (int q = 0; q < d; ++q) acc[q] *= xs[row * d + q] * h.inv_ls[q];
    acc[d] = os / (2.0 * h.s);
  }
  for (int j = 0; j <= d; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (GP_MAX_D + 1) + j] = red[0];
    __syncthreads();
  }
}

// gradient assembly (natural parameters [ls | s | sigma^2]); one workgroup,
// fixed-order tree reductions
__device__ double block_sum256(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void k_grad_final(const double* __restrict__ bwd_part, int nb_bwd, const double* __restrict__ pg_part,
                             int nb_pg, const double* __restrict__ trm_part, const double* __restrict__ cc_part,
                             int nb_dot, int tp, int ell, int64_t n, int k, int ard, Hyper h,
                             const double* __restrict__ Cinv, int have_precond, double* __restrict__ grad) {
  __shared__ double bil[GP_MAX_D + 1], pg[GP_MAX_D + 1];
  const int d = h.d;
  for (int j = 0; j <= d; ++j) {
    double s = 0.0, q = 0.0;
    for (int b = threadIdx.x; b < nb_bwd; b += 256) s += bwd_part[(int64_t)b * (GP_MAX_D + 1) + j];
    for (int b = threadIdx.x; b < nb_pg; b += 256) q += pg_part[(int64_t)b * (GP_MAX_D + 1) + j];
    s = block_sum256(s);
    q = block_sum256(q);
    if (threadIdx.x == 0) {
      bil[j] = s;
      pg[j] = have_precond ? q : 0.0;
    }
  }
  double trm = 0.0, cc = 0.0, tci = 0.0;
  for (int e = threadIdx.x; e < nb_dot * tp; e += 256) {
    const int c = e % tp;
    trm += trm_part[e];
    if (c >= 1 && c <= ell) cc += cc_part[e];
  }
  for (int j = threadIdx.x; j < k; j += 256) tci += Cinv[(int64_t)j * k + j];
  trm = block_sum256(trm);
  cc = block_sum256(cc);
  tci = block_sum256(tci);
  if (threadIdx.x != 0) return;
  const double trPinv = (double)(n - k) / h.s2 + tci;
  const int p = ard ? d : 1;
  if (ard) {
    for (int j = 0; j < d; ++j) grad[j] = bil[j] + pg[j];
  } else {
    double s = 0.0;
    for (int j = 0; j < d; ++j) s += bil[j] + pg[j];
    grad[0] = s;
  }
  grad[p] = bil[d] + pg[d];
  grad[p + 1] = trm - 0.5 * trPinv + cc / (2.0 * ell);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_woodbury(const Ctx& c, const Hyper& h, const double* Rsrc, double* Zdst, const int* nact,
                           double* rz_part);
hipError_t launch_coldot(const Ctx& c, const double* A, const double* B, double* part);
hipError_t launch_ltr(const Ctx& c, const double* Rsrc, double* dst, const int* nact);

static unsigned nbk(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

template <typename T>
static hipError_t run_bwd_tiles(const Ctx& c, const Hyper& h, BwdArgs ba, const T* xfa, const T* xfb, const T* rt,
                                const T* ct, T* afr, T* cfr, T* xau, T* rows) {
  const Layout& L = *c.lay;
  const size_t smem = (size_t)(ba.nk4 * 64 + ba.nkt * 64 + ba.nbt * 256 + 16) * sizeof(T);
  dim3 grid((unsigned)(L.n_pad / 64), (unsigned)L.nsplit);
  switch (h.kind) {
    case GP_KERNEL_RBF:
      hipLaunchKernelGGL((k_bwd_tiles<T, GP_KERNEL_RBF>), grid, dim3(256), smem, c.st, xfa, xfb, rt, ct, afr, cfr, xau,
                         rows, ba);
      break;
    case GP_KERNEL_MATERN32:
      hipLaunchKernelGGL((k_bwd_tiles<T, GP_KERNEL_MATERN32>), grid, dim3(256), smem, c.st, xfa, xfb, rt, ct, afr, cfr,
                         xau, rows, ba);
      break;
    case GP_KERNEL_RATQUAD:
      hipLaunchKernelGGL((k_bwd_tiles<T, GP_KERNEL_RATQUAD>), grid, dim3(256), smem, c.st, xfa, xfb, rt, ct, afr, cfr,
                         xau, rows, ba);
      break;
    default:
      hipLaunchKernelGGL((k_bwd_tiles<T, GP_KERNEL_MATERN52>), grid, dim3(256), smem, c.st, xfa, xfb, rt, ct, afr, cfr,
                         xau, rows, ba);
  }
  return hipGetLastError();
}

namespace {
template <int KIND, int NKC, int NKM, int NXT>
hipError_t run_bwd_bf16(const Ctx& c, const BwdBfArgs& ba) {
  const Layout& L = *c.lay;
  constexpr int RG = 2;
  dim3 grid((unsigned)(L.n_pad / (64 * RG)), (unsigned)L.nsplit);
  hipLaunchKernelGGL((k_bwd_bf16<KIND, NKC, NKM, NXT, RG>), grid, dim3(256), 0, c.st, c.at<u32x4>(L.xfa),
                     c.at<u32x4>(L.xfb), c.at<float>(L.rowterm), c.at<float>(L.colterm), c.at<u32x4>(L.bafrag),
                     c.at<u32x4>(L.bcfrag), c.at<u32x4>(L.bxaug), c.at<float>(L.wpart), ba);
  return hipGetLastError();
}
template <int KIND, int NKC, int NXT>
hipError_t sel_bwd_nkm(const Ctx& c, const BwdBfArgs& ba, int nkm) {
  switch (nkm) {
#define CASE(N) case N: return run_bwd_bf16<KIND, NKC, N, NXT>(c, ba);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12)
    CASE(14) CASE(16) CASE(18) CASE(20) CASE(22) CASE(24)
#undef CASE
  }
  return hipErrorInvalidValue;
}
template <int KIND>
hipError_t sel_bwd(const Ctx& c, const BwdBfArgs& ba, int nkc, int nkm, int nxt) {
  if (nxt == 1) {
    switch (nkc) {
      case 1: return sel_bwd_nkm<KIND, 1, 1>(c, ba, nkm);
      case 2: return sel_bwd_nkm<KIND, 2, 1>(c, ba, nkm);
    }
  } else if (nxt == 2) {
    switch (nkc) {
      case 2: return sel_bwd_nkm<KIND, 2, 2>(c, ba, nkm);
    }
  } else if (nxt == 3) {
    switch (nkc) {
      case 3: return sel_bwd_nkm<KIND, 3, 3>(c, ba, nkm);
    }
  } else if (nxt == 4) {
    switch (nkc) {
      case 3: return sel_bwd_nkm<KIND, 3, 4>(c, ba, nkm);
      case 4: return sel_bwd_nkm<KIND, 4, 4>(c, ba, nkm);
    }
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_bwd_bf16(const Ctx& c, const Hyper& h) {
  const Layout& L = *c.lay;
  const int tq = (L.t + 7) / 8 * 8;
  const int nkm = bwd_nkm(L.t);
  const int nxt = (2 * L.d + 15) / 16;
  const int nkc = L.kd / 32;
  const int64_t nfr = (L.n_pad / 16) * nkm * 64;
  hipLaunchKernelGGL(k_stage_rows_bf16x3, dim3((unsigned)((nfr + 255) / 256)), dim3(256), 0, c.st,
                     c.at<double>(L.Xs), L.n_pad, L.tp, L.t, tq, nkm, 1, c.at<u32x4>(L.bafrag));
  hipLaunchKernelGGL(k_stage_rows_bf16x3, dim3((unsigned)((nfr + 255) / 256)), dim3(256), 0, c.st,
                     c.at<double>(L.cprime), L.n_pad, L.tp, L.t, tq, nkm, 0, c.at<u32x4>(L.bcfrag));
  const int64_t nxf = (L.n_pad / 32) * nxt * 64;
  hipLaunchKernelGGL(k_stage_xaug_bf16, dim3((unsigned)((nxf + 255) / 256)), dim3(256), 0, c.st, c.at<double>(L.xs),
                     L.n, L.n_pad, L.d, nxt, c.at<u32x4>(L.bxaug));
  BwdBfArgs ba;
  ba.n_pad = L.n_pad;
  ba.cols_per_split = L.cols_per_split;
  ba.ow = L.bow;
  ba.nbt = (2 * L.d + 1 + 15) / 16;
  ba.s = (float)h.s;
  ba.inv_s = (float)(1.0 / h.s);
  ba.alpha = (float)h.alpha;
  if (L.prec == GP_PREC_FP16X3) {  // staged RBF values are 2^15 kappa
    ba.rbf_sg = (float)(h.s / 32768.0);
    ba.rbf_kap = 1.0f / 32768.0f;
  } else {  // staged RBF values are s kappa
    ba.rbf_sg = 1.0f;
    ba.rbf_kap = (float)(1.0 / h.s);
  }
  switch (h.kind) {
    case GP_KERNEL_RBF: return sel_bwd<GP_KERNEL_RBF>(c, ba, nkc, nkm, nxt);
    case GP_KERNEL_MATERN32: return sel_bwd<GP_KERNEL_MATERN32>(c, ba, nkc, nkm, nxt);
    case GP_KERNEL_RATQUAD: return sel_bwd<GP_KERNEL_RATQUAD>(c, ba, nkc, nkm, nxt);
    default: return sel_bwd<GP_KERNEL_MATERN52>(c, ba, nkc, nkm, nxt);
  }
}

// ---------------------------------------------------------------------------
// Probes through the symmetric square root of P_hat = sigma^2 I + L L^T:
//   P_hat^1/2 w = sigma w + L M L^T w,  M = (C^1/2 + sigma I)^-1,  C = sigma^2 I + L^T L
// (for L^T L = V diag(lam) V^T, M = V diag(1 / (sigma + sqrt(sigma^2 + lam))) V^T).
// C^1/2 comes from the coupled Newton-Schulz iteration on A = C / tr(C) (spectrum in
// (0, 1]): T = (3I - Z Y) / 2, Y <- Y T, Z <- T Z, with Y -> A^1/2 and Z -> A^-1/2
// quadratically once close (Higham, "Functions of Matrices", Sec. 6.7); a fixed
// count of steps covers condition numbers of C up to about 1e16.
// ---------------------------------------------------------------------------

constexpr int kSqrtSteps = 100;

// R = [y | sigma w_1 .. sigma w_ell | 0] with w the Rademacher stream 0 (the eps of the
// first probe form), Xs = 0; padding rows zero
__global__ void k_probes_base(const double* __restrict__ y, int64_t n, int64_t n_pad, int ell, int tp, double sigma,
                              uint64_t seed, double* __restrict__ R, double* __restrict__ Xs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  double* row = R + i * tp;
  double* xrow = Xs + i * tp;
  for (int c = 0; c < tp; ++c) {
    xrow[c] = 0.0;
    row[c] = 0.0;
  }
  if (i >= n) return;
  row[0] = y[i];
  for (int c = 0; c < ell; ++c) row[1 + c] = sigma * rademacher(seed, 0, (uint64_t)c, (uint64_t)i);
}

// eta signs of the probes: H[l][c] for preconditioner column l and probe c (stream 1)
__global__ void k_probe_eta(uint64_t seed, int k, int ell, double* __restrict__ H) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * ell) return;
  const int l = e / ell, c = e % ell;
  H[e] = rademacher(seed, 1, (uint64_t)c, (uint64_t)l);
}

// R = [y | sigma eps + L eta] (n_pad x tp row-major; the product L H as one tile GEMM)
hipError_t launch_probes(const Ctx& c, const double* y, const Hyper& h, uint64_t seed) {
  const Layout& L = *c.lay;
  hipLaunchKernelGGL(k_probes_base, dim3((unsigned)((L.n_pad + 255) / 256)), dim3(256), 0, c.st, y, L.n, L.n_pad,
                     L.ell, L.tp, sqrt(h.s2), seed, c.at<double>(L.R), c.at<double>(L.Xs));
  if (L.k == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_probe_eta, dim3((L.k * L.ell + 255) / 256), dim3(256), 0, c.st, seed, L.k, L.ell,
                     c.at<double>(L.H));
  hipLaunchKernelGGL(k_gemm64, dim3(nbk(L.n, 64), (L.ell + 63) / 64), dim3(256), 0, c.st, L.n, L.ell, L.k,
                     c.at<double>(L.L), (int64_t)1, (int64_t)L.n, c.at<double>(L.H), (int64_t)L.ell, (int64_t)1,
                     c.at<double>(L.R) + 1, (int64_t)L.tp, (int64_t)1, 1.0, 1.0, (const int*)nullptr,
                     (const int*)nullptr);
  return hipGetLastError();
}

// inverse of an SPD k x k matrix by the small Cholesky routine (logdet and status
// outputs go to scratch / the deferred-status slot)
__global__ void k_sqrt_inverse(int64_t n, int k, double s2, const double* __restrict__ Bm, double* __restrict__ Rc,
                               double* __restrict__ Rinv, double* __restrict__ Binv, double* __restrict__ scratch,
                               int* __restrict__ status) {
  small_chol_body(n, k, s2, Bm, Rc, Rinv, Binv, scratch, status);
}

// A = C / tr(C), Y = A, Z = I; scal[0] = tr(C) (one workgroup)
__global__ void k_sqrt_init(const double* __restrict__ C, int k, double* __restrict__ Y, double* __restrict__ Z,
                            double* __restrict__ scal) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) s += C[(int64_t)j * k + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double tr = red[0];
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    Y[e] = C[e] / tr;
    Z[e] = (e / k == e % k) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) scal[0] = tr;
}

// T = (3 I - P) / 2
__global__ void k_sqrt_t(const double* __restrict__ P, int k, double* __restrict__ T) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  T[e] = ((e / k == e % k) ? 1.5 : 0.0) - 0.5 * P[e];
}

// B = sqrt(tr C) Y + sigma I
__global__ void k_sqrt_shift(const double* __restrict__ Y, const double* __restrict__ scal, int k, double sigma,
                             double* __restrict__ Bm) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  Bm[e] = sqrt(scal[0]) * Y[e] + ((e / k == e % k) ? sigma : 0.0);
}

hipError_t launch_probes_sqrt(const Ctx& c, const double* y, const Hyper& h, uint64_t seed) {
  const Layout& L = *c.lay;
  const double sigma = sqrt(h.s2);
  // R = [y | sigma w] with w the Rademacher stream of the first probe form
  hipLaunchKernelGGL(k_probes_base, dim3((unsigned)((L.n_pad + 255) / 256)), dim3(256), 0, c.st, y, L.n, L.n_pad,
                     L.ell, L.tp, sigma, seed, c.at<double>(L.R), c.at<double>(L.Xs));
  if (L.k == 0) return hipGetLastError();
  const int k = L.k;
  const int64_t kk = (int64_t)k * k;
  double* w = c.at<double>(L.sqrt_work);
  double *Y = w, *Z = w + kk, *P = w + 2 * kk, *T = w + 3 * kk, *Y2 = w + 4 * kk, *Z2 = w + 5 * kk;
  double* scal = c.at<double>(L.pg_part);  // free until the derivative sweep
  hipLaunchKernelGGL(k_sqrt_init, dim3(1), dim3(256), 0, c.st, c.at<double>(L.C), k, Y, Z, scal);
  const dim3 gk(nbk(k, 64), (k + 63) / 64), bk(256);
  const unsigned ne = nbk(kk, 256);
  for (int it = 0; it < kSqrtSteps; ++it) {
    hipLaunchKernelGGL(k_gemm64, gk, bk, 0, c.st, (int64_t)k, k, k, Z, (int64_t)k, (int64_t)1, Y, (int64_t)k,
                       (int64_t)1, P, (int64_t)k, (int64_t)1, 1.0, 0.0, (const int*)nullptr, (const int*)nullptr);
    hipLaunchKernelGGL(k_sqrt_t, dim3(ne), dim3(256), 0, c.st, P, k, T);
    hipLaunchKernelGGL(k_gemm64, gk, bk, 0, c.st, (int64_t)k, k, k, Y, (int64_t)k, (int64_t)1, T, (int64_t)k,
                       (int64_t)1, Y2, (int64_t)k, (int64_t)1, 1.0, 0.0, (const int*)nullptr, (const int*)nullptr);
    hipLaunchKernelGGL(k_gemm64, gk, bk, 0, c.st, (int64_t)k, k, k, T, (int64_t)k, (int64_t)1, Z, (int64_t)k,
                       (int64_t)1, Z2, (int64_t)k, (int64_t)1, 1.0, 0.0, (const int*)nullptr, (const int*)nullptr);
    std::swap(Y, Y2);
    std::swap(Z, Z2);
  }
  // M = (C^1/2 + sigma I)^-1 by the small Cholesky routine (its log-det output is a scratch slot)
  hipLaunchKernelGGL(k_sqrt_shift, dim3(ne), dim3(256), 0, c.st, Y, scal, k, sigma, P);
  double* M = T;
  hipLaunchKernelGGL(k_sqrt_inverse, dim3(1), dim3(1024), 0, c.st, L.n, k, h.s2, P, Z2, Y2, M, scal + 1,
                     c.at<int>(L.flags) + 1);
  // U = L^T (sigma w) into ltr_raw ([k][tp]); V = M U / sigma; R[:, 1..ell] += L V
  hipError_t e = launch_ltr(c, c.at<double>(L.R), c.at<double>(L.ltr_raw), nullptr);
  if (e != hipSuccess) return e;
  double* V = c.at<double>(L.ltr);
  hipLaunchKernelGGL(k_gemm64, dim3(nbk(k, 64), (L.tp + 63) / 64), bk, 0, c.st, (int64_t)k, L.tp, k, M, (int64_t)k,
                     (int64_t)1, c.at<double>(L.ltr_raw), (int64_t)L.tp, (int64_t)1, V, (int64_t)L.tp, (int64_t)1,
                     1.0 / sigma, 0.0, (const int*)nullptr, (const int*)nullptr);
  hipLaunchKernelGGL(k_gemm64, dim3(nbk(L.n, 64), (L.ell + 63) / 64), bk, 0, c.st, L.n, L.ell, k, c.at<double>(L.L),
                     (int64_t)1, (int64_t)L.n, V + 1, (int64_t)L.tp, (int64_t)1, c.at<double>(L.R) + 1, (int64_t)L.tp,
                     (int64_t)1, 1.0, 1.0, (const int*)nullptr, (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_backward(const Ctx& c, const Hyper& h, int ard, int precond_grad, int precond_kind, double* grad) {
  const Layout& L = *c.lay;
  const int tp = L.tp;
  // (1) C' and the staged operands of the derivative sweep
  hipLaunchKernelGGL(k_cprime, dim3(nbk(L.n_pad * tp, 256)), dim3(256), 0, c.st, c.at<double>(L.Xs), c.at<double>(L.Z0),
                     L.n, L.n_pad, tp, L.ell, c.at<double>(L.cprime));
  BwdArgs ba;
  ba.n_pad = L.n_pad;
  ba.n = L.n;
  ba.cols_per_split = L.cols_per_split;
  ba.nk4 = L.bkd / 4;
  ba.nkt = tp / 4;
  ba.nbt = (2 * L.d + 1 + 15) / 16;
  ba.ow = L.bow;
  ba.s = h.s;
  ba.alpha = h.alpha;
  const int64_t nfr_t = (L.n_pad / 16) * ba.nkt * 64;
  const int64_t nfr_x = (L.n_pad / 16) * ba.nbt * 256;
  const bool f64 = L.bprec == GP_PREC_FP64;
  hipError_t e;
  if (L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3) {
    e = launch_bwd_bf16(c, h);
  } else if (f64) {
    hipLaunchKernelGGL(k_stage_rows16x4<double>, dim3(nbk(nfr_t, 256)), dim3(256), 0, c.st, c.at<double>(L.Xs),
                       L.n_pad, tp, tp, ba.nkt, c.at<double>(L.bafrag));
    hipLaunchKernelGGL(k_stage_rows16x4<double>, dim3(nbk(nfr_t, 256)), dim3(256), 0, c.st, c.at<double>(L.cprime),
                       L.n_pad, tp, tp, ba.nkt, c.at<double>(L.bcfrag));
    hipLaunchKernelGGL(k_stage_xaug<double>, dim3(nbk(nfr_x, 256)), dim3(256), 0, c.st, c.at<double>(L.xs), L.n,
                       L.n_pad, L.d, ba.nbt, c.at<double>(L.bxaug));
    e = run_bwd_tiles<double>(c, h, ba, c.at<double>(L.bxa), c.at<double>(L.bxb), c.at<double>(L.brt),
                              c.at<double>(L.bct), c.at<double>(L.bafrag), c.at<double>(L.bcfrag),
                              c.at<double>(L.bxaug), c.at<double>(L.wpart));
  } else {
    hipLaunchKernelGGL(k_stage_rows16x4<float>, dim3(nbk(nfr_t, 256)), dim3(256), 0, c.st, c.at<double>(L.Xs), L.n_pad,
                       tp, tp, ba.nkt, c.at<float>(L.bafrag));
    hipLaunchKernelGGL(k_stage_rows16x4<float>, dim3(nbk(nfr_t, 256)), dim3(256), 0, c.st, c.at<double>(L.cprime),
                       L.n_pad, tp, tp, ba.nkt, c.at<float>(L.bcfrag));
    hipLaunchKernelGGL(k_stage_xaug<float>, dim3(nbk(nfr_x, 256)), dim3(256), 0, c.st, c.at<double>(L.xs), L.n, L.n_pad,
                       L.d, ba.nbt, c.at<float>(L.bxaug));
    e = run_bwd_tiles<float>(c, h, ba, c.at<float>(L.bxa), c.at<float>(L.bxb), c.at<float>(L.brt), c.at<float>(L.bct),
                             c.at<float>(L.bafrag), c.at<float>(L.bcfrag), c.at<float>(L.bxaug), c.at<float>(L.wpart));
  }
  if (e != hipSuccess) return e;
  const unsigned nbr = nbk(L.n, 256);
  double* bwd_part = c.at<double>(L.bwd_part);
  if (f64)
    hipLaunchKernelGGL(k_bwd_rows<double>, dim3(nbr), dim3(256), 0, c.st, c.at<double>(L.wpart), L.nsplit, L.n, L.n_pad,
                       L.bow, ba.nbt, L.d, c.at<double>(L.xs), h, bwd_part);
  else
    hipLaunchKernelGGL(k_bwd_rows<float>, dim3(nbr), dim3(256), 0, c.st, c.at<float>(L.wpart), L.nsplit, L.n, L.n_pad,
                       L.bow, ba.nbt, L.d, c.at<double>(L.xs), h, bwd_part);

  // (2) tr(M) and sum_i |c_i|^2
  double* dots = c.at<double>(L.dot_part);
  double* trm_part = dots;
  double* cc_part = dots + (int64_t)L.nred * tp;
  e = launch_coldot(c, c.at<double>(L.Xs), c.at<double>(L.cprime), trm_part);
  if (e != hipSuccess) return e;
  e = launch_coldot(c, c.at<double>(L.Z0), c.at<double>(L.Z0), cc_part);
  if (e != hipSuccess) return e;

  // (3) preconditioner terms
  double* pg_part = c.at<double>(L.pg_part);
  unsigned nb_pg = 1;
  if (L.k > 0 && precond_kind == kRff) {
    // Z^T [c_i] into ltr_raw (columns 1..ell); Omega = -Z C^-1 + (1/ell) [c_i] (Z^T [c_i])^T
    e = launch_ltr(c, c.at<double>(L.Z0), c.at<double>(L.ltr_raw), nullptr);
    if (e != hipSuccess) return e;
    double* Om = c.at<double>(L.omega);
    dim3 gg(nbk(L.n, 64), (L.k + 63) / 64);
    hipLaunchKernelGGL(k_gemm64, gg, dim3(256), 0, c.st, L.n, L.k, L.k, c.at<double>(L.L), (int64_t)1, (int64_t)L.n,
                       c.at<double>(L.Cinv), (int64_t)L.k, (int64_t)1, Om, (int64_t)1, (int64_t)L.n, -1.0, 0.0,
                       (const int*)nullptr, (const int*)nullptr);
    hipLaunchKernelGGL(k_gemm64, gg, dim3(256), 0, c.st, L.n, L.k, L.ell, c.at<double>(L.Z0) + 1, (int64_t)tp,
                       (int64_t)1, c.at<double>(L.ltr_raw) + 1, (int64_t)1, (int64_t)tp, Om, (int64_t)1, (int64_t)L.n,
                       1.0 / L.ell, 1.0, (const int*)nullptr, (const int*)nullptr);
    nb_pg = nbk(L.n, 256);
    hipLaunchKernelGGL(k_rff_contract, dim3(nb_pg), dim3(256), 0, c.st, c.at<double>(L.xs), L.n, L.k / 2,
                       c.at<double>(L.freq), Om, c.at<double>(L.L), h, precond_grad, pg_part);
  } else if (L.k > 0) {
    // L^T [c_i] into ltr_raw (columns 1..ell)
    e = launch_ltr(c, c.at<double>(L.Z0), c.at<double>(L.ltr_raw), nullptr);
    if (e != hipSuccess) return e;
    double* sm = c.at<double>(L.pg_small);
    const int64_t kk = (int64_t)L.k * L.k;
    double* LSinv = sm;
    double* Gk = sm + kk;
    double* Psi = sm + 2 * kk;
    double* tmp = sm + 3 * kk;
    double* U = sm + 4 * kk;
    hipLaunchKernelGGL(k_pg_small, dim3(1), dim3(1024), 0, c.st, c.at<double>(L.L), c.at<int32_t>(L.piv),
                       c.at<int>(L.scal_small) + 1, L.n, L.k, c.at<double>(L.Cinv), c.at<double>(L.ltr_raw), tp, L.ell,
                       h.s2, LSinv, Gk, Psi, U, tmp);
    // Omega = -L Gk + (1/ell) Z0[:, 1:] U^T  (column-major n x k)
    double* Om = c.at<double>(L.omega);
    const int* kpp = c.at<int>(L.scal_small) + 1;
    dim3 gg(nbk(L.n, 64), (L.k + 63) / 64);
    hipLaunchKernelGGL(k_gemm64, gg, dim3(256), 0, c.st, L.n, L.k, L.k, c.at<double>(L.L), (int64_t)1, (int64_t)L.n, Gk,
                       (int64_t)L.k, (int64_t)1, Om, (int64_t)1, (int64_t)L.n, -1.0, 0.0, kpp, kpp);
    hipLaunchKernelGGL(k_gemm64, gg, dim3(256), 0, c.st, L.n, L.k, L.ell, c.at<double>(L.Z0) + 1, (int64_t)tp,
                       (int64_t)1, U, (int64_t)1, (int64_t)tp, Om, (int64_t)1, (int64_t)L.n, 1.0 / L.ell, 1.0,
                       kpp, (const int*)nullptr);
    nb_pg = nbk(L.n + L.k, 256);
    hipLaunchKernelGGL(k_pg_contract, dim3(nb_pg), dim3(256), 0, c.st, c.at<double>(L.xs), c.at<int32_t>(L.piv), kpp,
                       L.n, L.k, Om, Psi, h, precond_grad, pg_part);
  }
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(256), 0, c.st, bwd_part, (int)nbr, pg_part, (int)nb_pg, trm_part,
                     cc_part, L.nred, tp, L.ell, L.n, L.k, ard, h, c.at<double>(L.Cinv), L.k > 0 ? 1 : 0, grad);
  return hipGetLastError();
}

}  // namespace gpmll
