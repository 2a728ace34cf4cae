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
};

template <typename T>
__device__ inline void kappa_g_t(int kind, T q, T s, T* kap, T* sg) {
  if constexpr (sizeof(T) == 8) {
    double k, g;
    kappa_g64(kind, q > 0.0 ? q : 0.0, &k, &g);
    *kap = k;
    *sg = s * g;
  } else {
    const float log2e = 1.4426950408889634f;
    const float q0 = fmaxf(q, 0.0f);
    if (kind == GP_KERNEL_RBF) {
      const float e = __builtin_amdgcn_exp2f(-0.5f * log2e * q0);
      *kap = e;
      *sg = s * e;
    } else if (kind == GP_KERNEL_MATERN32) {
      const float a = 1.7320508075688772f;
      const float r = __builtin_sqrtf(q0);
      const float e = __builtin_amdgcn_exp2f(-a * log2e * r);
      *kap = fmaf(a, r, 1.0f) * e;
      *sg = s * 3.0f * e;
    } else {
      const float a = 2.23606797749979f;
      const float r = __builtin_sqrtf(q0);
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
      kappa_g_t<T>(KIND, dd[v] + ct[acc_row_b<T>(g, v)], (T)a.s, &kap, &sg);
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
// Preconditioner derivative terms
// ---------------------------------------------------------------------------

// small k x k algebra in one workgroup: LS = L[piv, :kp], LSinv, Gk = C^-1 LSinv,
// H = LSinv^T (I - sigma^2 C^-1) LSinv, U = LSinv^T (L^T C_mat), Psi = H/2 - U U^T/(2 ell)
__global__ void k_pg_small(const double* __restrict__ L, const int32_t* __restrict__ piv, const int* __restrict__ kpp,
                           int64_t n, int k, const double* __restrict__ Cinv, const double* __restrict__ ltrc, int tp,
                           int ell, double s2, double* __restrict__ LSinv, double* __restrict__ Gk,
                           double* __restrict__ Psi, double* __restrict__ U, double* __restrict__ tmp) {
  const int kp = *kpp;
  // LS (row a = pivot a, column b) into tmp, lower triangular
  for (int e = threadIdx.x; e < kp * kp; e += blockDim.x) {
    const int a0 = e / kp, b0 = e % kp;
    tmp[a0 * k + b0] = (b0 <= a0) ? L[(int64_t)b0 * n + piv[a0]] : 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kp; c += blockDim.x) {
    for (int i = 0; i < kp; ++i) {
      double acc = (i == c) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) acc -= tmp[i * k + l] * LSinv[l * k + c];
      LSinv[i * k + c] = (i < c) ? 0.0 : acc / tmp[i * k + i];
    }
  }
  __syncthreads();
  // Gk[r][q] = sum_m Cinv[r][m] LSinv[m][q]
  for (int e = threadIdx.x; e < kp * kp; e += blockDim.x) {
    const int r = e / kp, q = e % kp;
    double s = 0.0;
    for (int m = q; m < kp; ++m) s += Cinv[r * k + m] * LSinv[m * k + q];
    Gk[r * k + q] = s;
  }
  // tmp[m][q] = sum_r (I - s2 Cinv)[m][r] LSinv[r][q]
  __syncthreads();
  for (int e = threadIdx.x; e < kp * kp; e += blockDim.x) {
    const int m = e / kp, q = e % kp;
    double s = 0.0;
    for (int r = q; r < kp; ++r) s += ((m == r ? 1.0 : 0.0) - s2 * Cinv[m * k + r]) * LSinv[r * k + q];
    tmp[m * k + q] = s;
  }
  // U[q][i] = sum_m LSinv[m][q] ltrc[m][1 + i]
  for (int e = threadIdx.x; e < kp * ell; e += blockDim.x) {
    const int q = e / ell, i = e % ell;
    double s = 0.0;
    for (int m = q; m < kp; ++m) s += LSinv[m * k + q] * ltrc[m * tp + 1 + i];
    U[q * tp + i] = s;
  }
  __syncthreads();
  // Psi[q][r] = 1/2 sum_m LSinv[m][q] tmp[m][r] - 1/(2 ell) sum_i U[q][i] U[r][i]
  for (int e = threadIdx.x; e < kp * kp; e += blockDim.x) {
    const int q = e / kp, r = e % kp;
    double h = 0.0;
    for (int m = q; m < kp; ++m) h += LSinv[m * k + q] * tmp[m * k + r];
    double uu = 0.0;
    for (int i = 0; i < ell; ++i) uu += U[q * tp + i] * U[r * tp + i];
    Psi[q * k + r] = 0.5 * h - uu / (2.0 * ell);
  }
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
      kappa_g64(h.kind, r2, &kap, &g);
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

// gradient assembly (natural parameters [ls | s | sigma^2])
__global__ void k_grad_final(const double* __restrict__ bwd_part, int nb_bwd, const double* __restrict__ pg_part,
                             int nb_pg, const double* __restrict__ trm_part, const double* __restrict__ cc_part,
                             int nb_dot, int tp, int ell, int64_t n, int k, int ard, Hyper h,
                             const double* __restrict__ Cinv, int have_precond, double* __restrict__ grad) {
  if (threadIdx.x != 0) return;
  const int d = h.d;
  double bil[GP_MAX_D + 1], pg[GP_MAX_D + 1];
  for (int j = 0; j <= d; ++j) {
    double s = 0.0, q = 0.0;
    for (int b = 0; b < nb_bwd; ++b) s += bwd_part[(int64_t)b * (GP_MAX_D + 1) + j];
    for (int b = 0; b < nb_pg; ++b) q += pg_part[(int64_t)b * (GP_MAX_D + 1) + j];
    bil[j] = s;
    pg[j] = have_precond ? q : 0.0;
  }
  double trm = 0.0, cc = 0.0;
  for (int b = 0; b < nb_dot; ++b)
    for (int c = 0; c < tp; ++c) {
      trm += trm_part[(int64_t)b * tp + c];
      if (c >= 1 && c <= ell) cc += cc_part[(int64_t)b * tp + c];
    }
  double trCinv = 0.0;
  for (int j = 0; j < k; ++j) trCinv += Cinv[j * k + j];
  const double trPinv = (double)(n - k) / h.s2 + trCinv;
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
    default:
      hipLaunchKernelGGL((k_bwd_tiles<T, GP_KERNEL_MATERN52>), grid, dim3(256), smem, c.st, xfa, xfb, rt, ct, afr, cfr,
                         xau, rows, ba);
  }
  return hipGetLastError();
}

hipError_t launch_backward(const Ctx& c, const Hyper& h, int ard, int precond_grad, double* grad) {
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
  const int64_t nfr_t = (L.n_pad / 16) * ba.nkt * 64;
  const int64_t nfr_x = (L.n_pad / 16) * ba.nbt * 256;
  const bool f64 = L.bprec == GP_PREC_FP64;
  hipError_t e;
  if (f64) {
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
  if (L.k > 0) {
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
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(64), 0, c.st, bwd_part, (int)nbr, pg_part, (int)nb_pg, trm_part,
                     cc_part, L.nred, tp, L.ell, L.n, L.k, ard, h, c.at<double>(L.Cinv), L.k > 0 ? 1 : 0, grad);
  return hipGetLastError();
}

}  // namespace gpmll
