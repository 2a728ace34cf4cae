// Small dense routines shared by the single-problem and the batched paths:
// the k x k Cholesky of C = sigma^2 I + L^T L with its inverse and log det P_hat,
// the k x k algebra of the preconditioner derivative, the first-row eigen-solve
// of a Lanczos tridiagonal, and the SplitMix64 counter stream of the probes.
// Every routine here runs inside one workgroup (or one lane) on one problem.
#pragma once

#include "gpmll_impl.h"

namespace gpmll {

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// sign +1 when the top bit of output (stream << 56 | col << 32 | idx) is clear
__device__ inline double rademacher(uint64_t seed, uint64_t stream, uint64_t col, uint64_t idx) {
  uint64_t v = splitmix64(seed, (stream << 56) | (col << 32) | idx);
  return (v >> 63) ? -1.0 : 1.0;
}


// Right-looking Cholesky of the k x k matrix C (row-major) by one workgroup,
// then the lower-triangular inverse, C^-1 = Rinv^T Rinv and the log-determinant.
inline __device__ void small_chol_body(int64_t n, int k, double s2, const double* __restrict__ C, double* __restrict__ Rc,
                                double* __restrict__ Rinv, double* __restrict__ Cinv, double* __restrict__ logdetP,
                                int* __restrict__ status) {
  __shared__ int bad;
  __shared__ double red[1024];
  if (threadIdx.x == 0) bad = 0;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) Rc[e] = C[e];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) {
      double v = Rc[j * k + j];
      if (!(v > 0.0)) {
        bad = 1;
        v = 1.0;
      }
      Rc[j * k + j] = sqrt(v);
    }
    __syncthreads();
    const double piv = Rc[j * k + j];
    for (int i = j + 1 + threadIdx.x; i < k; i += blockDim.x) Rc[i * k + j] /= piv;
    __syncthreads();
    const int m = k - j - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) Rc[i * k + l] -= Rc[i * k + j] * Rc[l * k + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    int i = e / k, l = e % k;
    if (l > i) Rc[e] = 0.0;
  }
  __syncthreads();
  // Rinv column c: solve Rc x = e_c by forward substitution (one thread per column)
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    for (int i = 0; i < k; ++i) {
      double acc = (i == c) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) acc -= Rc[i * k + l] * Rinv[l * k + c];
      Rinv[i * k + c] = (i < c) ? 0.0 : acc / Rc[i * k + i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    int a = e / k, b = e % k;
    int lo = a > b ? a : b;
    double s = 0.0;
    for (int l = lo; l < k; ++l) s += Rinv[l * k + a] * Rinv[l * k + b];
    Cinv[e] = s;
  }
  double acc = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) acc += log(Rc[j * k + j]);
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < (int)blockDim.x; ++q) s += red[q];
    *logdetP = (double)(n - k) * log(s2) + 2.0 * s;
    if (bad) *status = GP_ENOTSPD;
  }
}

// small k x k algebra in one workgroup: LS = L[piv, :kp], LSinv, Gk = C^-1 LSinv,
// H = LSinv^T (I - sigma^2 C^-1) LSinv, U = LSinv^T (L^T C_mat), Psi = H/2 - U U^T/(2 ell)
inline __device__ void pg_small_body(const double* __restrict__ L, const int32_t* __restrict__ piv, const int* __restrict__ kpp,
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

// Eigenvalues of the symmetric tridiagonal (a diagonal, b off-diagonal, order m)
// and the first components z of its eigenvectors; a and b are overwritten (a
// ends up holding the eigenvalues).  Implicit symmetric QR steps with the
// Wilkinson shift (Golub & Van Loan, "Matrix Computations", Sec. 8.3), Givens
// rotations chasing the bulge, deflation of negligible off-diagonals; only the
// first row of the accumulated rotations is kept (Golub & Welsch 1969).
inline __device__ void tridiag_eig_first_row(double* a, double* b, double* z, int m) {
  const double eps = 2.220446049250313e-16;
  for (int i = 0; i < m; ++i) z[i] = (i == 0) ? 1.0 : 0.0;
  int hi = m - 1;
  int sweeps = 0;
  while (hi > 0 && sweeps < 60 * m) {
    if (fabs(b[hi - 1]) <= eps * (fabs(a[hi - 1]) + fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(b[lo - 1]) > eps * (fabs(a[lo - 1]) + fabs(a[lo]))) --lo;
    if (lo > 0) b[lo - 1] = 0.0;
    // Wilkinson shift: eigenvalue of the trailing 2 x 2 closer to a[hi]
    const double dl = 0.5 * (a[hi - 1] - a[hi]);
    const double bb = b[hi - 1];
    const double den = dl + copysign(sqrt(dl * dl + bb * bb), dl == 0.0 ? 1.0 : dl);
    const double mu = a[hi] - bb * bb / den;
    // one implicit QR sweep over [lo, hi]; the entries of row / column k travel in
    // registers from one rotation to the next (ak, bk, zk are a[k], b[k], z[k])
    double x = a[lo] - mu, y = b[lo];
    double ak = a[lo], bk = b[lo], zk = z[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = sqrt(x * x + y * y);
      const double inv = r > 0.0 ? 1.0 / r : 0.0;
      const double cs = r > 0.0 ? x * inv : 1.0;
      const double sn = y * inv;
      if (k > lo) b[k - 1] = r;
      const double ak1 = a[k + 1], zk1 = z[k + 1];
      const double c2 = cs * cs, s2 = sn * sn, csn = cs * sn;
      a[k] = c2 * ak + 2.0 * csn * bk + s2 * ak1;
      const double nak1 = s2 * ak - 2.0 * csn * bk + c2 * ak1;
      const double nbk = csn * (ak1 - ak) + (c2 - s2) * bk;
      double bulge = 0.0, bk1 = 0.0;
      if (k + 1 < hi) {
        const double bn = b[k + 1];
        bulge = sn * bn;
        bk1 = cs * bn;
      }
      z[k] = cs * zk + sn * zk1;
      zk = -sn * zk + cs * zk1;
      ak = nak1;
      bk = bk1;
      x = nbk;
      y = bulge;
    }
    a[hi] = ak;
    z[hi] = zk;
    b[hi - 1] = x;
    ++sweeps;
  }
}

// e1^T log(T) e1 of a symmetric positive definite tridiagonal T (diagonal a,
// squared off-diagonal bb, order m, both readable by the whole workgroup), by the
// trapezoidal rule on
//   log x = int_R ( e^u / (1 + e^u) - e^u / (x + e^u) ) du,
// whose integrand is analytic in |Im u| < pi: with step h = 1/2 the rule's error
// is about exp(-2 pi^2 / h) ~ 1e-17, and u runs from log(min(lam_lo, 1)) - 40 to
// log(max(Gershgorin bound, 1)) + 40 (tails below 4e-18).  At each node
// e1^T (T + t I)^-1 e1 = 1 / f_0 with the continued fraction
//   f_{m-1} = a_{m-1} + t,  f_k = a_k + t - bb_k / f_{k+1},
// and the integrand t (f_0 - 1 - t) / ((1 + t) f_0) uses f_0 - 1 - t formed without
// t, free of cancellation.  Returns false on every thread if some f_k <= 0 (T not
// numerically positive definite).  red: blockDim.x doubles of shared memory.
inline __device__ bool tridiag_log_e1(const double* a, const double* bb, int m, double lam_lo, double* red,
                                      int* bad, double* result) {
  // Gershgorin upper bound of the spectrum
  double g = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    double r = a[k];
    if (k > 0) r += sqrt(bb[k - 1]);
    if (k + 1 < m) r += sqrt(bb[k]);
    g = fmax(g, r);
  }
  red[threadIdx.x] = g;
  if (threadIdx.x == 0) *bad = 0;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  const double hi = red[0];
  __syncthreads();
  const double h = 0.5;
  const double u0 = log(fmin(lam_lo, 1.0)) - 40.0;
  const double u1 = log(fmax(hi, 1.0)) + 40.0;
  const int nodes = (int)ceil((u1 - u0) / h) + 1;
  double acc = 0.0;
  int mybad = 0;
  for (int q = threadIdx.x; q < nodes; q += blockDim.x) {
    const double t = exp(u0 + h * q);
    double f = a[m - 1] + t;
    mybad |= !(f > 0.0);
    for (int k = m - 2; k >= 1; --k) {
      f = a[k] + t - bb[k] / f;
      mybad |= !(f > 0.0);
    }
    // f0 - 1 - t and f0
    const double fm = (m >= 2) ? (a[0] - 1.0 - bb[0] / f) : (a[0] - 1.0);
    const double f0 = fm + 1.0 + t;
    mybad |= !(f0 > 0.0);
    acc += t * fm / ((1.0 + t) * f0);
  }
  if (mybad) atomicOr(bad, 1);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double total = red[0];
  const bool ok = *bad == 0;
  __syncthreads();
  *result = h * total;
  return ok;
}

}  // namespace gpmll
