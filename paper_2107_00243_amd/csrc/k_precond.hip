// Input staging, the partial pivoted Cholesky preconditioner and the probes.
//
// Preconditioner: P_hat = sigma^2 I + L L^T with L from a greedy partial pivoted
// Cholesky factorisation of K (Section 2.2, "Preconditioning", diagonal-plus-low-rank
// preconditioners; supplement S5.3).  Solves use the matrix inversion lemma with
// C = sigma^2 I_k + L^T L; log det P_hat = (n - k) log sigma^2 + log det C.
// Probes: b_i = sigma * eps_i + L * eta_i with Rademacher eps_i, eta_i drawn from a
// SplitMix64 counter stream (Steele, Lea & Flood 2014), so that E[b b^T] = P_hat.
#include "gpmll_impl.h"
#include "small_dense.h"

#include <algorithm>

namespace gpmll {

// ---------------------------------------------------------------------------
// Column means and the scaled inputs x~ = (x - mean) / ls
// ---------------------------------------------------------------------------

__global__ void k_colsum_part(const double* __restrict__ X, int64_t n, int d, int64_t rows_per_block,
                              double* __restrict__ part) {
  __shared__ double red[8][GP_MAX_D];
  const int j = threadIdx.x % GP_MAX_D;
  const int g = threadIdx.x / GP_MAX_D;  // 8 row groups
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  double acc = 0.0;
  if (j < d)
    for (int64_t r = r0 + g; r < r1; r += 8) acc += X[r * d + j];
  red[g][j] = acc;
  __syncthreads();
  if (g == 0 && j < d) {
    double s = 0.0;
    for (int q = 0; q < 8; ++q) s += red[q][j];
    part[(int64_t)blockIdx.x * GP_MAX_D + j] = s;
  }
}

__global__ void k_colmean_final(const double* __restrict__ part, int nblk, int64_t n, int d,
                                double* __restrict__ mean) {
  const int j = threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * GP_MAX_D + j];
  mean[j] = s / (double)n;
}

__global__ void k_scale(const double* __restrict__ X, const double* __restrict__ mean, int64_t n,
                        int64_t n_pad, Hyper h, double* __restrict__ xs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  for (int j = 0; j < h.d; ++j)
    xs[i * h.d + j] = (i < n) ? (X[i * h.d + j] - mean[j]) * h.inv_ls[j] : 0.0;
}

// ---------------------------------------------------------------------------
// Partial pivoted Cholesky: one launch per step.  Each launch
//   1. reduces the previous step's per-block (value, index) maxima of the residual
//      diagonal to the pivot (larger value wins, ties to the lower index),
//   2. writes column j of L:  L[r, j] = (K[r, piv] - sum_{l<j} L[r, l] L[piv, l]) / sqrt(d_piv),
//      with L[piv, j] = sqrt(d_piv) and zeros on earlier pivot rows,
//   3. updates the residual diagonal and emits this block's maximum for step j+1.
// A step whose largest residual is <= 1e-12 * s stops the factorisation: it and
// all later steps leave their columns zero and record pivot -1.
// With prescribed pivots (the randomized Nystrom preconditioner of Table 1 on
// given landmark rows) step 1 takes the next landmark instead; the factor is then
// K_{:S} K_SS^-1 K_{S:} on those rows, and the same breakdown rule applies to the
// landmark's residual diagonal.
// ---------------------------------------------------------------------------

struct ArgMax {
  double v;
  int64_t i;
};

__device__ inline ArgMax amax_better(ArgMax a, ArgMax b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ ArgMax block_argmax(ArgMax x) {
  __shared__ double sv[kRedBlock];
  __shared__ int64_t si[kRedBlock];
  sv[threadIdx.x] = x.v;
  si[threadIdx.x] = x.i;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      ArgMax a{sv[threadIdx.x], si[threadIdx.x]};
      ArgMax b{sv[threadIdx.x + off], si[threadIdx.x + off]};
      a = amax_better(a, b);
      sv[threadIdx.x] = a.v;
      si[threadIdx.x] = a.i;
    }
    __syncthreads();
  }
  ArgMax r{sv[0], si[0]};
  __syncthreads();
  return r;
}

__global__ void k_pivchol_init(int64_t n, int k, double s, double* __restrict__ L,
                               double* __restrict__ diag, int8_t* __restrict__ ispiv,
                               int32_t* __restrict__ piv, ArgMax* __restrict__ amax, int* __restrict__ stop) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    diag[i] = s;
    ispiv[i] = 0;
    for (int j = 0; j < k; ++j) L[(int64_t)j * n + i] = 0.0;
  }
  if (i < k) piv[i] = -1;
  // every entry ties at s: the block maximum is its first row
  if (threadIdx.x == 0) {
    const int64_t first = (int64_t)blockIdx.x * blockDim.x;
    amax[blockIdx.x] = ArgMax{first < n ? s : -1.0, first < n ? first : (int64_t)n};
  }
  if (i == 0) {
    stop[0] = 0;  // stop flag
    stop[1] = k;  // achieved rank
  }
}

__global__ void k_pivchol_step(int j, int64_t n, int k, int nblk, Hyper h, const double* __restrict__ xs,
                               double* __restrict__ L, double* __restrict__ diag, int8_t* __restrict__ ispiv,
                               int32_t* __restrict__ piv, const ArgMax* __restrict__ amax_in,
                               ArgMax* __restrict__ amax_out, int* __restrict__ stop,
                               const int32_t* __restrict__ forced) {
  __shared__ double Lp[GP_MAX_RANK];
  __shared__ double xp[GP_MAX_D];
  __shared__ ArgMax pivot;
  __shared__ int halted;
  if (threadIdx.x == 0) halted = *stop;
  __syncthreads();
  if (halted) return;
  // 1. pivot of this step: the largest residual diagonal, or the prescribed row
  // (its residual diagonal is left in place below, so every block reads the same value)
  if (forced) {
    if (threadIdx.x == 0) {
      const int64_t f = forced[j];
      pivot = ArgMax{diag[f], f};
    }
  } else {
    ArgMax loc{-1.0, (int64_t)n};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) loc = amax_better(loc, amax_in[b]);
    ArgMax best = block_argmax(loc);
    if (threadIdx.x == 0) pivot = best;
  }
  __syncthreads();
  const double dpiv = pivot.v;
  const int64_t ip = pivot.i;
  if (!(dpiv > 1e-12 * h.s)) {
    // breakdown: stop here (all blocks see the same pivot and agree)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      stop[0] = 1;
      stop[1] = j;
    }
    return;
  }
  for (int l = threadIdx.x; l < j; l += blockDim.x) Lp[l] = L[(int64_t)l * n + ip];
  for (int q = threadIdx.x; q < h.d; q += blockDim.x) xp[q] = xs[ip * h.d + q];
  __syncthreads();
  const double sq = sqrt(dpiv);
  const double inv = 1.0 / sq;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  ArgMax mine{-1.0, (int64_t)n};
  if (i < n) {
    double lij;
    if (i == ip) {
      lij = sq;
    } else if (ispiv[i]) {
      lij = 0.0;
    } else {
      double r2 = 0.0;
      for (int q = 0; q < h.d; ++q) {
        double df = xs[i * h.d + q] - xp[q];
        r2 += df * df;
      }
      double kv = h.s * kappa64(h.kind, r2, h.alpha);
      double dot = 0.0;
      for (int l = 0; l < j; ++l) dot += L[(int64_t)l * n + i] * Lp[l];
      lij = (kv - dot) * inv;
    }
    L[(int64_t)j * n + i] = lij;
    double dn;
    if (i == ip || ispiv[i]) {
      dn = 0.0;
    } else {
      dn = diag[i] - lij * lij;
      mine = ArgMax{dn, i};
    }
    if (!(forced && i == ip)) diag[i] = dn;
  }
  if (!forced) {
    ArgMax bm = block_argmax(mine);
    if (threadIdx.x == 0) amax_out[blockIdx.x] = bm;
  }
  if (i == ip) ispiv[i] = 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) piv[j] = (int32_t)ip;
}

// ---------------------------------------------------------------------------
// C = sigma^2 I + L^T L (partials over row chunks, then a fixed-order sum),
// its Cholesky factor Rc, the inverse Rinv = Rc^-1, C^-1 and log det P_hat.
// ---------------------------------------------------------------------------

__global__ void k_gram_part(const double* __restrict__ L, int64_t n, int k, int64_t chunk,
                            double* __restrict__ part) {
  // block (tile a, tile b, chunk): 16 x 16 tile of L^T L over one row chunk
  __shared__ double la[16][65], lb[16][65];
  const int ta = blockIdx.x, tb = blockIdx.y;
  if (tb > ta) return;
  const int a0 = ta * 16, b0 = tb * 16;
  const int64_t r0 = (int64_t)blockIdx.z * chunk, r1 = min(n, r0 + chunk);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc = 0.0;
  for (int64_t base = r0; base < r1; base += 64) {
    for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
      int c = e / 64, rr = e % 64;
      int64_t r = base + rr;
      la[c][rr] = (a0 + c < k && r < r1) ? L[(int64_t)(a0 + c) * n + r] : 0.0;
      lb[c][rr] = (b0 + c < k && r < r1) ? L[(int64_t)(b0 + c) * n + r] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < 64; ++rr) acc += la[ty][rr] * lb[tx][rr];
    __syncthreads();
  }
  const int a = a0 + ty, b = b0 + tx;
  if (a < k && b < k) part[((int64_t)blockIdx.z * k + a) * k + b] = acc;
}

__global__ void k_gram_final(const double* __restrict__ part, int nchunk, int k, double s2,
                             double* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int a = e / k, b = e % k;
  const int hi = a > b ? a : b, lo = a > b ? b : a;
  double s = 0.0;
  for (int q = 0; q < nchunk; ++q) s += part[((int64_t)q * k + hi) * k + lo];
  C[e] = s + (a == b ? s2 : 0.0);
}

__global__ void k_small_chol(int64_t n, int k, double s2, const double* __restrict__ C,
                             double* __restrict__ Rc, double* __restrict__ Rinv, double* __restrict__ Cinv,
                             double* __restrict__ logdetP, int* __restrict__ status) {
  small_chol_body(n, k, s2, C, Rc, Rinv, Cinv, logdetP, status);
}

__global__ void k_logdet_noprecond(int64_t n, double s2, double* logdetP) {
  *logdetP = (double)n * log(s2);
}

// ---------------------------------------------------------------------------
// Random Fourier feature preconditioner (Table 1, "RFF"): Z = sqrt(s/m)
// [cos(Phi) | sin(Phi)] with Phi = x~ W^T, x~ the centred scaled inputs and W the
// m x d spectral samples at unit lengthscale.  Quadrature Fourier features (Table
// 1, "QFF") use the same form with quadrature nodes as W and per-frequency
// amplitudes sqrt(s w_j) (amps; null: sqrt(s/m) for all).  One thread per row; Z is written
// column-major n x 2m in the slot of the pivoted Cholesky factor, the pivots read
// -1 and the achieved rank is 2m.
// ---------------------------------------------------------------------------

__global__ void k_rff_features(const double* __restrict__ xs, int64_t n, int d, int m,
                               const double* __restrict__ W, const double* __restrict__ amps, double amp0,
                               double* __restrict__ Z, int32_t* __restrict__ piv, int* __restrict__ small) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * m) piv[i] = -1;
  if (i == 0) {
    small[0] = 0;
    small[1] = 2 * m;
  }
  if (i >= n) return;
  double x[GP_MAX_D];
  for (int q = 0; q < d; ++q) x[q] = xs[i * d + q];
  for (int j = 0; j < m; ++j) {
    double ph = 0.0;
    for (int q = 0; q < d; ++q) ph = fma(W[j * d + q], x[q], ph);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double amp = amps ? amps[j] : amp0;
    Z[(int64_t)j * n + i] = amp * cs;
    Z[(int64_t)(m + j) * n + i] = amp * sn;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_prep(const Ctx& c, const double* X, const Hyper& h) {
  const Layout& L = *c.lay;
  const int64_t rows_per_block = (L.n + L.nred - 1) / L.nred;
  hipLaunchKernelGGL(k_colsum_part, dim3(L.nred), dim3(256), 0, c.st, X, L.n, L.d, rows_per_block,
                     c.at<double>(L.mean_part));
  hipLaunchKernelGGL(k_colmean_final, dim3(1), dim3(GP_MAX_D), 0, c.st, c.at<double>(L.mean_part), L.nred,
                     L.n, L.d, c.at<double>(L.mean));
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((L.n_pad + 255) / 256)), dim3(256), 0, c.st, X,
                     c.at<double>(L.mean), L.n, L.n_pad, h, c.at<double>(L.xs));
  return hipGetLastError();
}

hipError_t launch_pivchol(const Ctx& c, const Hyper& h, const int32_t* forced) {
  const Layout& L = *c.lay;
  const int nblk = (int)((L.n + kRedBlock - 1) / kRedBlock);
  ArgMax* am = c.at<ArgMax>(L.amax);
  int* stop = c.at<int>(L.scal_small);
  hipLaunchKernelGGL(k_pivchol_init, dim3(nblk), dim3(kRedBlock), 0, c.st, L.n, L.k, h.s, c.at<double>(L.L),
                     c.at<double>(L.diag), c.at<int8_t>(L.ispiv), c.at<int32_t>(L.piv), am, stop);
  for (int j = 0; j < L.k; ++j) {
    ArgMax* in = am + (j % 2) * nblk;
    ArgMax* out = am + ((j + 1) % 2) * nblk;
    hipLaunchKernelGGL(k_pivchol_step, dim3(nblk), dim3(kRedBlock), 0, c.st, j, L.n, L.k, nblk, h,
                       c.at<double>(L.xs), c.at<double>(L.L), c.at<double>(L.diag), c.at<int8_t>(L.ispiv),
                       c.at<int32_t>(L.piv), in, out, stop, forced);
  }
  return hipGetLastError();
}

hipError_t launch_rff(const Ctx& c, const Hyper& h, bool weighted) {
  const Layout& L = *c.lay;
  const int m = L.k / 2;
  const int64_t cnt = std::max<int64_t>(L.n, L.k);
  hipLaunchKernelGGL(k_rff_features, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c.st, c.at<double>(L.xs),
                     L.n, L.d, m, c.at<double>(L.freq), weighted ? c.at<double>(L.famp) : nullptr, sqrt(h.s / m),
                     c.at<double>(L.L), c.at<int32_t>(L.piv), c.at<int>(L.scal_small));
  return hipGetLastError();
}

// L (k x n, row l contiguous) in the operand order of the L^T R MFMAs: entry e of
// rup(n, 64) x kpad, zero outside l < k, i < n; group (i/4, l/16), lane (kq, m) holds
// l = 16 (group % (kpad/16)) + m, i = 4 (group / (kpad/16)) + kq
__global__ void k_stage_l_frag(const double* __restrict__ L, int64_t n, int k, int kpad, int64_t total,
                               double* __restrict__ lf_ltr) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int lane = (int)(e & 63), m = lane & 15, kq = lane >> 4;
  const int64_t g = e >> 6;
  const int nlb = kpad / 16;
  const int l = (int)(g % nlb) * 16 + m;
  const int64_t i = (g / nlb) * 4 + kq;
  lf_ltr[e] = (l < k && i < n) ? L[(int64_t)l * n + i] : 0.0;
}

hipError_t launch_precond_finish(const Ctx& c, const Hyper& h) {
  const Layout& L = *c.lay;
  if (L.k == 0) {
    hipLaunchKernelGGL(k_logdet_noprecond, dim3(1), dim3(1), 0, c.st, L.n, h.s2, c.at<double>(L.logdetP));
    return hipGetLastError();
  }
  {
    const int kpad = (L.k + 15) / 16 * 16;
    const int64_t total = (L.n + 63) / 64 * 64 * kpad;
    hipLaunchKernelGGL(k_stage_l_frag, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.st, c.at<double>(L.L),
                       L.n, L.k, kpad, total, c.at<double>(L.lf_ltr));
  }
  const int tiles = (L.k + 15) / 16;
  hipLaunchKernelGGL(k_gram_part, dim3(tiles, tiles, L.nchunk), dim3(256), 0, c.st, c.at<double>(L.L), L.n,
                     L.k, (int64_t)kChunkRows, c.at<double>(L.ltr_part));
  hipLaunchKernelGGL(k_gram_final, dim3((L.k * L.k + 255) / 256), dim3(256), 0, c.st,
                     c.at<double>(L.ltr_part), L.nchunk, L.k, h.s2, c.at<double>(L.C));
  hipLaunchKernelGGL(k_small_chol, dim3(1), dim3(1024), 0, c.st, L.n, L.k, h.s2, c.at<double>(L.C),
                     c.at<double>(L.Rc), c.at<double>(L.Rinv), c.at<double>(L.Cinv), c.at<double>(L.logdetP),
                     c.at<int>(L.flags) + 1);
  return hipGetLastError();
}


}  // namespace gpmll
