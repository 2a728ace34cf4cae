// Lanczos quadrature for the log-determinant (Algorithm 1; Section 2.2, SLQ) with
// the tridiagonal recovered from the CG coefficients (supplement S1.2; Saad 2003,
// Sec. 6.7.3):
//   T_11 = 1/alpha_0,  T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
//   T_{j,j+1} = sqrt(beta_{j-1}) / alpha_{j-1}.
// Its eigenvalues theta_j and the first components tau_1j of its eigenvectors give
//   gamma_i = rho0_i * sum_j tau_1j^2 log(theta_j),  rho0_i = b_i^T P_hat^-1 b_i,
// and log p ~ -1/2 (y^T u + log det P_hat + mean_i gamma_i + n log 2 pi).
//
// Eigen-solver: implicit symmetric QR steps with the Wilkinson shift (Golub & Van
// Loan, "Matrix Computations", Sec. 8.3), Givens rotations chasing the bulge, and
// deflation of negligible off-diagonals; only the first row of the accumulated
// rotation product is kept (Golub & Welsch 1969).  One thread per probe.
#include "gpmll_impl.h"
#include "small_dense.h"

namespace gpmll {

// one workgroup of 256 threads per probe column c = 1 + blockIdx.x, tridiagonal in
// LDS (dynamic shared memory: 3 max_iters + 256 doubles).  Up to kSlqQrMax Lanczos
// steps one lane diagonalises T (QR, first row of the eigenvectors); longer T take
// e1^T log(T) e1 from the quadrature of tridiag_log_e1 over the whole workgroup,
// with lam_lo a lower bound of the preconditioned spectrum, and fall back to the
// QR if T is not numerically positive definite.
__global__ __launch_bounds__(256) void k_slq(const double* __restrict__ alog, const double* __restrict__ blog,
                                             const int* __restrict__ iters, const double* __restrict__ rho0, int ell,
                                             int max_iters, double lam_lo, double* __restrict__ gamma,
                                             int* __restrict__ clamp) {
  extern __shared__ double sm_tri[];
  __shared__ int bad;
  const int i = blockIdx.x;
  if (i >= ell) return;
  const int c = 1 + i;
  const int m = iters[c];
  if (m == 0) {
    if (threadIdx.x == 0) gamma[i] = 0.0;
    return;
  }
  double* a = sm_tri;
  double* b = a + max_iters;
  double* z = b + max_iters;
  double* red = z + max_iters;
  const double* al = alog + (int64_t)c * max_iters;
  const double* be = blog + (int64_t)c * max_iters;
  // T_11 = 1/alpha_0, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1}^2 = beta_j / alpha_j^2
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    a[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < m) b[j] = be[j] / (al[j] * al[j]);
  }
  __syncthreads();
  if (m > kSlqQrMax) {
    double v;
    if (tridiag_log_e1(a, b, m, lam_lo, red, &bad, &v)) {
      if (threadIdx.x == 0) gamma[i] = rho0[c] * v;
      return;
    }
  }
  if (threadIdx.x != 0) return;
  for (int j = 0; j + 1 < m; ++j) b[j] = sqrt(b[j]);
  tridiag_eig_first_row(a, b, z, m);
  double s = 0.0;
  int cl = 0;
  for (int j = 0; j < m; ++j) {
    double th = a[j];
    if (th < 1e-300) {
      th = 1e-300;
      ++cl;
    }
    s += z[j] * z[j] * log(th);
  }
  gamma[i] = rho0[c] * s;
  if (cl) atomicAdd(clamp, cl);
}

// the same with the tridiagonal in global memory (iteration caps above 2645)
__global__ void k_slq_global(const double* __restrict__ alog, const double* __restrict__ blog,
                             const int* __restrict__ iters, const double* __restrict__ rho0, int ell, int max_iters,
                             double* __restrict__ work, double* __restrict__ gamma, int* __restrict__ clamp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ell) return;
  const int c = 1 + i;
  const int m = iters[c];
  double* a = work + (int64_t)i * 3 * max_iters;
  double* b = a + max_iters;
  double* z = b + max_iters;
  const double* al = alog + (int64_t)c * max_iters;
  const double* be = blog + (int64_t)c * max_iters;
  if (m == 0) {
    gamma[i] = 0.0;
    return;
  }
  a[0] = 1.0 / al[0];
  for (int j = 1; j < m; ++j) {
    a[j] = 1.0 / al[j] + be[j - 1] / al[j - 1];
    b[j - 1] = sqrt(be[j - 1]) / al[j - 1];
  }
  tridiag_eig_first_row(a, b, z, m);
  double s = 0.0;
  int cl = 0;
  for (int j = 0; j < m; ++j) {
    double th = a[j];
    if (th < 1e-300) {
      th = 1e-300;
      ++cl;
    }
    s += z[j] * z[j] * log(th);
  }
  gamma[i] = rho0[c] * s;
  if (cl) atomicAdd(clamp, cl);
}

// partial y^T u over row blocks (u = column 0 of the solutions)
__global__ void k_dot_y(const double* __restrict__ y, const double* __restrict__ Xs, int64_t n, int tp,
                        double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  red[threadIdx.x] = (i < n) ? y[i] * Xs[i * tp] : 0.0;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// log p and the diagnostics: flags[0] bits, flags[1] status, flags[2] clamps
__global__ void k_logp(const double* __restrict__ part, int nblk, const double* __restrict__ gamma, int ell, int64_t n,
                       const double* __restrict__ logdetP, const int* __restrict__ nactive,
                       const int* __restrict__ stop, int* __restrict__ flags, double* __restrict__ datafit,
                       double* __restrict__ logdet_est, double* __restrict__ logp) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double yu = red[0];
    double g = 0.0;
    for (int i = 0; i < ell; ++i) g += gamma[i];
    const double ld = *logdetP + (ell > 0 ? g / ell : 0.0);
    *datafit = yu;
    *logdet_est = ld;
    *logp = -0.5 * (yu + ld + (double)n * 1.8378770664093453);
    int f = 0;
    if (*nactive > 0) f |= GP_FLAG_NOT_CONVERGED;
    if (*stop) f |= GP_FLAG_RANK_DEFICIENT;
    if (flags[2] > 0) f |= GP_FLAG_RITZ_CLAMPED;
    flags[0] = f;
  }
}

hipError_t launch_slq_logp(const Ctx& c, const Hyper& h, const double* y, double* logp) {
  const Layout& L = *c.lay;
  double* sl = c.at<double>(L.gamma);  // gamma[ell] | datafit | logdet_est
  const size_t smem = ((size_t)3 * L.max_iters + 256) * sizeof(double);
  // lower bound of the spectrum of P^-1/2 K_hat P^-1/2: sigma^2 / (sigma^2 + tr L L^T), tr L L^T <= n s
  const double lam_lo = h.s2 / (h.s2 + (double)L.n * h.s);
  if (smem <= 64 * 1024)
    hipLaunchKernelGGL(k_slq, dim3(L.ell), dim3(256), smem, c.st, c.at<double>(L.alog), c.at<double>(L.blog),
                       c.at<int>(L.iters), c.at<double>(L.rho0), L.ell, L.max_iters, lam_lo, sl,
                       c.at<int>(L.flags) + 2);
  else
    hipLaunchKernelGGL(k_slq_global, dim3((L.ell + 63) / 64), dim3(64), 0, c.st, c.at<double>(L.alog),
                       c.at<double>(L.blog), c.at<int>(L.iters), c.at<double>(L.rho0), L.ell, L.max_iters,
                       c.at<double>(L.slq_work), sl, c.at<int>(L.flags) + 2);
  const unsigned nb = (unsigned)((L.n + 255) / 256);
  double* part = c.at<double>(L.dot_part);
  hipLaunchKernelGGL(k_dot_y, dim3(nb), dim3(256), 0, c.st, y, c.at<double>(L.Xs), L.n, L.tp, part);
  hipLaunchKernelGGL(k_logp, dim3(1), dim3(256), 0, c.st, part, (int)nb, sl, L.ell, L.n, c.at<double>(L.logdetP),
                     c.at<int>(L.nactive), c.at<int>(L.scal_small), c.at<int>(L.flags), sl + L.ell, sl + L.ell + 1,
                     logp);
  return hipGetLastError();
}

}  // namespace gpmll
