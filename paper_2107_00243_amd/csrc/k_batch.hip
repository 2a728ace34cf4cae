// Ragged batches: Algorithms 1 and 2 (Sec. 4.4) for many independent problems
// in one call.  The one-call-many-right-hand-sides form of CG (footnote to
// Sec. 4.4) extends here across problems: each phase below is one launch for
// every problem, with per-problem hyperparameters, preconditioners and CG
// scalars and per-(problem, column) convergence masks.  The K_hat V product
// reuses the FP32 / FP64 MFMA tile kernel through a table of work items that
// stay inside one problem's diagonal block; the small per-problem algebra
// (pivoted Cholesky, C and its Cholesky factor, Lanczos quadrature, the
// preconditioner-derivative algebra) runs one workgroup per problem; per-row
// work runs over the kBRows-row blocks of the concatenation.
//
// The arithmetic of every phase is that of the single-problem path: pivoted
// Cholesky with ties to the lower index and the 1e-12 s stop (supplement S5.3),
// probes b = sigma eps + L eta, preconditioned CG with x0 = 0, Lanczos
// coefficients from alpha and beta (supplement S1.2), and the gradient
// sum_pq M_pq dK_pq - 1/2 tr(P^-1 dP) + 1/(2 ell) sum_i c_i^T dP c_i with
// frozen pivots (Sec. 3.3).  Problem b draws its probes from seed + b.
#include "batch_impl.h"
#include "small_dense.h"

namespace gpmll {

namespace {

__device__ double bsum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// sum over the problem's row blocks of a [block][tp] partial (fixed order)
__device__ double problem_total(const double* __restrict__ part, const BDesc& D, int tp, int c) {
  double s = 0.0;
  for (int q = 0; q < D.nblk; ++q) s += part[(int64_t)(D.blk0 + q) * tp + c];
  return s;
}

// ---------------------------------------------------------------------------
// inputs: column means and x~ = (x - mean) / ls per problem (one workgroup each)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void kb_prep(const double* __restrict__ X, const BDesc* __restrict__ desc, int d,
                                               double* __restrict__ xs) {
  __shared__ double red[256];
  __shared__ double mean[GP_MAX_D];
  const BDesc& D = desc[blockIdx.x];
  for (int j = 0; j < d; ++j) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < D.n; i += 256) s += X[(D.xoff + i) * d + j];
    s = bsum(s, red);
    if (threadIdx.x == 0) mean[j] = s / (double)D.n;
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < D.n_pad; i += 256)
    for (int j = 0; j < d; ++j)
      xs[(D.off + i) * d + j] = i < D.n ? (X[(D.xoff + i) * d + j] - mean[j]) * D.inv_ls[j] : 0.0;
}

// ---------------------------------------------------------------------------
// partial pivoted Cholesky, one workgroup of 1024 threads per problem, all steps
// ---------------------------------------------------------------------------
struct BArg {
  double v;
  int64_t i;
};

__device__ inline BArg barg_better(BArg a, BArg b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ BArg barg_block(BArg x, double* sv, int64_t* si) {
  sv[threadIdx.x] = x.v;
  si[threadIdx.x] = x.i;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      BArg a = barg_better(BArg{sv[threadIdx.x], si[threadIdx.x]}, BArg{sv[threadIdx.x + off], si[threadIdx.x + off]});
      sv[threadIdx.x] = a.v;
      si[threadIdx.x] = a.i;
    }
    __syncthreads();
  }
  BArg r{sv[0], si[0]};
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(1024) void kb_pivchol(const BDesc* __restrict__ desc, int d, int kind, int K,
                                                   const double* __restrict__ xs, double* __restrict__ Lall,
                                                   double* __restrict__ diag, int8_t* __restrict__ ispiv,
                                                   int32_t* __restrict__ piv, int32_t* __restrict__ kach,
                                                   int32_t* __restrict__ stop) {
  __shared__ double sv[1024];
  __shared__ int64_t si[1024];
  __shared__ double Lp[kBMaxRank];
  __shared__ double xp[GP_MAX_D];
  const int b = blockIdx.x;
  const BDesc& D = desc[b];
  const int64_t n = D.n, np = D.n_pad;
  const int k = D.k;
  double* Lb = Lall + D.loff;
  const double* xb = xs + D.off * d;
  double* dg = diag + D.off;
  int8_t* sp = ispiv + D.off;
  for (int64_t i = threadIdx.x; i < np; i += 1024) {
    dg[i] = D.s;
    sp[i] = 0;
    for (int j = 0; j < K; ++j) Lb[(int64_t)j * np + i] = 0.0;
  }
  for (int j = threadIdx.x; j < K; j += 1024) piv[b * K + j] = -1;
  if (threadIdx.x == 0) {
    kach[b] = k;
    stop[b] = 0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    BArg loc{-1.0, n};
    for (int64_t i = threadIdx.x; i < n; i += 1024)
      if (!sp[i]) loc = barg_better(loc, BArg{dg[i], i});
    const BArg best = barg_block(loc, sv, si);
    if (!(best.v > 1e-12 * D.s)) {
      if (threadIdx.x == 0) {
        stop[b] = 1;
        kach[b] = j;
      }
      return;
    }
    const int64_t ip = best.i;
    for (int l = threadIdx.x; l < j; l += 1024) Lp[l] = Lb[(int64_t)l * np + ip];
    for (int q = threadIdx.x; q < d; q += 1024) xp[q] = xb[ip * d + q];
    __syncthreads();
    const double sq = sqrt(best.v);
    const double inv = 1.0 / sq;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
      double lij;
      if (i == ip) {
        lij = sq;
      } else if (sp[i]) {
        lij = 0.0;
      } else {
        double r2 = 0.0;
        for (int q = 0; q < d; ++q) {
          const double df = xb[i * d + q] - xp[q];
          r2 += df * df;
        }
        const double kv = D.s * kappa64(kind, r2, 1.0);  // batches take no rational quadratic kernel
        double dot = 0.0;
        for (int l = 0; l < j; ++l) dot += Lb[(int64_t)l * np + i] * Lp[l];
        lij = (kv - dot) * inv;
      }
      Lb[(int64_t)j * np + i] = lij;
      dg[i] = (i == ip || sp[i]) ? 0.0 : dg[i] - lij * lij;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      sp[ip] = 1;
      piv[b * K + j] = (int32_t)ip;
    }
    __syncthreads();
  }
}

// C = sigma^2 I + L^T L, its Cholesky factor, inverse, C^-1 and log det P_hat
__global__ __launch_bounds__(1024) void kb_gram_chol(const BDesc* __restrict__ desc, int K,
                                                     const double* __restrict__ Lall, double* __restrict__ C,
                                                     double* __restrict__ Rc, double* __restrict__ Rinv,
                                                     double* __restrict__ Cinv, double* __restrict__ logdetP,
                                                     int* __restrict__ flags) {
  const int b = blockIdx.x;
  const BDesc& D = desc[b];
  const int k = D.k;
  if (k == 0) {
    if (threadIdx.x == 0) logdetP[b] = (double)D.n * log(D.s2);
    return;
  }
  const double* Lb = Lall + D.loff;
  const int64_t kk = (int64_t)K * K;
  double* Cb = C + b * kk;
  for (int e = threadIdx.x; e < k * k; e += 1024) {
    const int a = e / k, c = e % k;
    if (c > a) continue;
    double s = 0.0;
    for (int64_t i = 0; i < D.n; ++i) s += Lb[(int64_t)a * D.n_pad + i] * Lb[(int64_t)c * D.n_pad + i];
    Cb[a * k + c] = s + (a == c ? D.s2 : 0.0);
    Cb[c * k + a] = s + (a == c ? D.s2 : 0.0);
  }
  __syncthreads();
  small_chol_body(D.n, k, D.s2, Cb, Rc + b * kk, Rinv + b * kk, Cinv + b * kk, logdetP + b, flags + b * 4 + 1);
}

// ---------------------------------------------------------------------------
// probes: R = [y | sigma eps + L eta], X = 0; eta per problem first
// ---------------------------------------------------------------------------
__global__ void kb_eta(const BDesc* __restrict__ desc, int K, int ell, double* __restrict__ H) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const BDesc& D = desc[b];
  if (e >= D.k * ell) return;
  const int l = e / ell, c = e % ell;
  H[(int64_t)b * K * ell + e] = rademacher(D.seed, 1, (uint64_t)c, (uint64_t)l);
}

__global__ __launch_bounds__(256) void kb_probes(const BDesc* __restrict__ desc, const int32_t* __restrict__ blkprob,
                                                 const double* __restrict__ y, const double* __restrict__ Lall,
                                                 const double* __restrict__ H, int K, int ell, int tp,
                                                 double* __restrict__ R, double* __restrict__ Xs) {
  const int b = blkprob[blockIdx.x];
  const BDesc& D = desc[b];
  const int64_t i = (int64_t)(blockIdx.x - D.blk0) * kBRows + threadIdx.x;
  const int64_t row = D.off + i;
  double* r = R + row * tp;
  double* x = Xs + row * tp;
  for (int c = 0; c < tp; ++c) x[c] = 0.0;
  if (i >= D.n) {
    for (int c = 0; c < tp; ++c) r[c] = 0.0;
    return;
  }
  const double* Lb = Lall + D.loff;
  const double* Hb = H + (int64_t)b * K * ell;
  r[0] = y[D.xoff + i];
  for (int c = 0; c < ell; ++c) {
    double acc = D.sigma * rademacher(D.seed, 0, (uint64_t)c, (uint64_t)i);
    for (int l = 0; l < D.k; ++l) acc += Lb[(int64_t)l * D.n_pad + i] * Hb[l * ell + c];
    r[1 + c] = acc;
  }
  for (int c = 1 + ell; c < tp; ++c) r[c] = 0.0;
}

// ---------------------------------------------------------------------------
// Woodbury apply Z = (R - L C^-1 L^T R) / sigma^2 per problem
// ---------------------------------------------------------------------------

typedef double f64x4 __attribute__((ext_vector_type(4)));

// part[blk][l][c] = sum over the block's rows of L[i][l] R[i][c] on the FP64
// matrix cores (v_mfma_f64_16x16x4f64; A lane = (l, 4 rows), B lane = (4 rows,
// column)); wave w of workgroup (blk, y) owns the 16 l of block 4 y + w
template <int NT>
__global__ __launch_bounds__(256) void kb_ltr_mfma(const BDesc* __restrict__ desc, const int32_t* __restrict__ blkprob,
                                                   const double* __restrict__ Lall, const double* __restrict__ R,
                                                   int KP, int tp, double* __restrict__ part,
                                                   const int* __restrict__ nactive, const int* __restrict__ pact) {
  if (nactive != nullptr && *nactive == 0) return;
  const int b = blkprob[blockIdx.x];
  if (pact != nullptr && pact[b] == 0) return;
  const BDesc& D = desc[b];
  const int k = D.k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mb = blockIdx.y * 4 + wave;
  if (mb * 16 >= k) return;
  const int64_t i0 = (int64_t)(blockIdx.x - D.blk0) * kBRows;
  const int64_t i1 = i0 + min((int64_t)kBRows, D.n - i0);
  const int m = lane & 15, kq = lane >> 4;
  const int l = mb * 16 + m;
  const double* Lc = Lall + D.loff + (int64_t)min(l, k - 1) * D.n_pad;
  const double* Rb = R + D.off * tp;
  f64x4 acc[NT];
#pragma unroll
  for (int nb = 0; nb < NT; ++nb) acc[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int U = 4;
  for (int64_t i = i0; i < i1; i += 4 * U) {
    double av[U], bv[U][NT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ir = i + 4 * u + kq;
      const bool in = ir < i1;
      av[u] = (in && l < k) ? Lc[ir] : 0.0;
      const double* Rr = Rb + (in ? ir : i0) * tp + m;
#pragma unroll
      for (int nb = 0; nb < NT; ++nb) bv[u][nb] = in ? Rr[nb * 16] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int nb = 0; nb < NT; ++nb) acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u][nb], acc[nb], 0, 0, 0);
  }
  double* out = part + ((int64_t)blockIdx.x * KP + mb * 16) * tp;
#pragma unroll
  for (int nb = 0; nb < NT; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(int64_t)(kq + 4 * v) * tp + nb * 16 + m] = acc[nb][v];
}

// Z = (R - L Y) / sigma^2 on the block's rows (four 16-row tiles per wave, FP64
// MFMA over the rank), padding rows zero; partial r.z per column
template <int NT>
__global__ __launch_bounds__(256) void kb_zapply_mfma(const BDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ blkprob,
                                                      const double* __restrict__ Lall, const double* __restrict__ Y,
                                                      const double* __restrict__ R, int K, int tp,
                                                      double* __restrict__ Z, double* __restrict__ part,
                                                      const int* __restrict__ nactive, const int* __restrict__ pact) {
  if (nactive != nullptr && *nactive == 0) return;
  __shared__ double red[16][16 * NT];
  const int b = blkprob[blockIdx.x];
  if (pact != nullptr && pact[b] == 0) return;
  const BDesc& D = desc[b];
  const int k = D.k;
  const double inv_s2 = 1.0 / D.s2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const double* Lb = Lall + D.loff;
  const double* Yb = Y + (int64_t)b * K * tp;
  const int64_t ib = (int64_t)(blockIdx.x - D.blk0) * kBRows + wave * 64;
  double rzs[NT];
#pragma unroll
  for (int nb = 0; nb < NT; ++nb) rzs[nb] = 0.0;
  for (int rt = 0; rt < 4; ++rt) {
    const int64_t r0 = ib + rt * 16;
    const int64_t ra = r0 + m;
    f64x4 acc[NT];
#pragma unroll
    for (int nb = 0; nb < NT; ++nb) acc[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
    constexpr int U = 4;
    for (int l0 = 0; l0 < k; l0 += 4 * U) {
      double av[U], bv[U][NT];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int l = l0 + 4 * u + kq;
        const bool in = l < k;
        av[u] = (in && ra < D.n) ? Lb[(int64_t)l * D.n_pad + ra] : 0.0;
        const double* Yr = Yb + (int64_t)(in ? l : 0) * tp + m;
#pragma unroll
        for (int nb = 0; nb < NT; ++nb) bv[u][nb] = in ? Yr[nb * 16] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int nb = 0; nb < NT; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u][nb], acc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < NT; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + kq + 4 * v;
        const int64_t e = (D.off + r) * tp + nb * 16 + m;
        if (r < D.n) {
          const double rv = R[e];
          const double z = (rv - acc[nb][v]) * inv_s2;
          Z[e] = z;
          rzs[nb] += rv * z;
        } else {
          Z[e] = 0.0;
        }
      }
  }
#pragma unroll
  for (int nb = 0; nb < NT; ++nb) red[wave * 4 + kq][nb * 16 + m] = rzs[nb];
  __syncthreads();
  for (int c = threadIdx.x; c < 16 * NT; c += 256) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += red[q][c];
    part[(int64_t)blockIdx.x * tp + c] = s;
  }
}

// Y = C^-1 (sum of the problem's partials of L^T R)
__global__ __launch_bounds__(256) void kb_wood_y(const BDesc* __restrict__ desc, const double* __restrict__ part,
                                                 const double* __restrict__ Cinv, int K, int KP, int tp,
                                                 double* __restrict__ Tb, double* __restrict__ Y,
                                                 const int* __restrict__ nactive) {
  if (nactive != nullptr && *nactive == 0) return;
  const int b = blockIdx.x;
  const BDesc& D = desc[b];
  const int k = D.k;
  if (k == 0) return;
  double* T = Tb + (int64_t)b * K * tp;
  for (int e = threadIdx.x; e < k * tp; e += 256) {
    const int l = e / tp, c = e % tp;
    double s = 0.0;
    for (int q = 0; q < D.nblk; ++q) s += part[((int64_t)(D.blk0 + q) * KP + l) * tp + c];
    T[l * tp + c] = s;
  }
  __syncthreads();
  const double* Ci = Cinv + (int64_t)b * K * K;
  double* Yb = Y + (int64_t)b * K * tp;
  for (int e = threadIdx.x; e < k * tp; e += 256) {
    const int l = e / tp, c = e % tp;
    double s = 0.0;
    for (int m = 0; m < k; ++m) s += Ci[l * k + m] * T[m * tp + c];
    Yb[l * tp + c] = s;
  }
}

// ---------------------------------------------------------------------------
// CG phases
// ---------------------------------------------------------------------------

// partial column dots A.B over the block's rows
__global__ __launch_bounds__(256) void kb_coldot(const double* __restrict__ A, const double* __restrict__ Bm, int tp,
                                                 double* __restrict__ part) {
  __shared__ double red[256];
  const int G = 256 / tp;
  const int c = threadIdx.x % tp, rg = threadIdx.x / tp;
  const int64_t r0 = (int64_t)blockIdx.x * kBRows;
  double s = 0.0;
  if (rg < G)
    for (int q = rg; q < kBRows; q += G) s += A[(r0 + q) * tp + c] * Bm[(r0 + q) * tp + c];
  red[threadIdx.x] = rg < G ? s : 0.0;
  __syncthreads();
  if ((int)threadIdx.x < tp) {
    double t = 0.0;
    for (int q = 0; q < G; ++q) t += red[q * tp + threadIdx.x];
    part[(int64_t)blockIdx.x * tp + threadIdx.x] = t;
  }
}

__global__ void kb_cg_start(const BDesc* __restrict__ desc, const double* __restrict__ part_bb,
                            const double* __restrict__ part_rz, int tp, int t, double* __restrict__ bnorm,
                            double* __restrict__ rho, double* __restrict__ rho0, int* __restrict__ active,
                            int* __restrict__ iters, int* __restrict__ nactive, int* __restrict__ pact) {
  const int b = blockIdx.x, c = threadIdx.x;
  int act = 0;
  if (c < tp) {
    const BDesc& D = desc[b];
    const double bb = problem_total(part_bb, D, tp, c);
    const double rz = problem_total(part_rz, D, tp, c);
    const int e = b * tp + c;
    bnorm[e] = sqrt(bb);
    rho[e] = rz;
    rho0[e] = rz;
    act = (c < t && bb > 0.0) ? 1 : 0;
    active[e] = act;
    iters[e] = 0;
    if (act) atomicAdd(nactive, 1);
  }
  const int cnt = __syncthreads_count(act);
  if (threadIdx.x == 0) pact[b] = cnt;
}

__global__ void kb_copy(const double* __restrict__ a, double* __restrict__ b, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) b[e] = a[e];
}

__global__ void kb_zero_i32(int* __restrict__ p, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0;
}

// W = s (sum of the problem's split partials) + sigma^2 P; partial p.w.  Thread = four
// consecutive columns (one vector load per split and row) x 1024 / tp row lanes; four
// rows per pass, all their split loads in flight together; rows past the problem's n
// get W = 0.  The row lanes' dot sums are added in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void kb_reduce(const BDesc* __restrict__ desc, const int32_t* __restrict__ blkprob,
                                                 const T* __restrict__ wpart, int64_t N, int tp,
                                                 const double* __restrict__ P, double* __restrict__ W,
                                                 double* __restrict__ part, const int* __restrict__ nactive,
                                                 const int* __restrict__ pact) {
  if (*nactive == 0) return;
  typedef T T4 __attribute__((ext_vector_type(4)));
  typedef double D4 __attribute__((ext_vector_type(4)));
  __shared__ double red[1024];
  const int b = blkprob[blockIdx.x];
  if (pact[b] == 0) return;
  const BDesc& D = desc[b];
  const int nq = tp / 4, G = 256 / nq;
  const int cq = threadIdx.x % nq, rg = threadIdx.x / nq;
  const int64_t i0 = (int64_t)(blockIdx.x - D.blk0) * kBRows;
  double dot[4] = {0.0, 0.0, 0.0, 0.0};
  if (rg < G) {
    for (int q0 = rg; q0 < kBRows; q0 += 4 * G) {
      int64_t row[4];
      bool inb[4];
      double w[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = q0 + j * G;
        inb[j] = q < kBRows;
        // the block's rows all exist in the partials, so a clamped row needs no condition
        row[j] = D.off + i0 + (inb[j] ? q : kBRows - 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) w[j][v] = 0.0;
      }
      for (int s = 0; s < D.nsplit; ++s) {
        T4 pv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pv[j] = *reinterpret_cast<const T4*>(wpart + ((int64_t)s * N + row[j]) * tp + 4 * cq);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) w[j][v] += (double)pv[j][v];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!inb[j]) continue;
        const int64_t e = row[j] * tp + 4 * cq;
        if (i0 + q0 + j * G >= D.n) {
          *reinterpret_cast<D4*>(W + e) = D4{0.0, 0.0, 0.0, 0.0};
          continue;
        }
        const D4 pv = *reinterpret_cast<const D4*>(P + e);
        D4 wv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          wv[v] = D.s * w[j][v] + D.s2 * pv[v];
          dot[v] += pv[v] * wv[v];
        }
        *reinterpret_cast<D4*>(W + e) = wv;
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (rg < G) red[rg * tp + 4 * cq + v] = dot[v];
  __syncthreads();
  if ((int)threadIdx.x < tp) {
    double s = 0.0;
    for (int q = 0; q < G; ++q) s += red[q * tp + threadIdx.x];
    part[(int64_t)blockIdx.x * tp + threadIdx.x] = s;
  }
}

__global__ void kb_alpha(const BDesc* __restrict__ desc, const double* __restrict__ part, int tp, int it,
                         int max_iters, const double* __restrict__ rho, const int* __restrict__ active,
                         double* __restrict__ alpha, double* __restrict__ alog, int* __restrict__ flags,
                         const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int b = blockIdx.x, c = threadIdx.x;
  if (c >= tp) return;
  const int e = b * tp + c;
  double a = 0.0;
  if (active[e]) {
    const double pw = problem_total(part, desc[b], tp, c);
    if (!(pw > 0.0)) {
      flags[b * 4 + 1] = GP_ENOTSPD;
    } else {
      a = rho[e] / pw;
      alog[(int64_t)e * max_iters + it] = a;
    }
  }
  alpha[e] = a;
}

// x += alpha p, r -= alpha w on active columns; partial |r|^2
__global__ __launch_bounds__(256) void kb_update(const int32_t* __restrict__ blkprob, double* __restrict__ Xs,
                                                 double* __restrict__ R, const double* __restrict__ P,
                                                 const double* __restrict__ W, const double* __restrict__ alpha,
                                                 const int* __restrict__ active, int tp, double* __restrict__ part,
                                                 const int* __restrict__ nactive, const int* __restrict__ pact) {
  if (*nactive == 0) return;
  __shared__ double red[256];
  const int b = blkprob[blockIdx.x];
  if (pact[b] == 0) return;
  const int G = 256 / tp;
  const int c = threadIdx.x % tp, rg = threadIdx.x / tp;
  const int64_t r0 = (int64_t)blockIdx.x * kBRows;
  double s = 0.0;
  if (rg < G && active[b * tp + c]) {
    const double a = alpha[b * tp + c];
    for (int q = rg; q < kBRows; q += G) {
      const int64_t e = (r0 + q) * tp + c;
      Xs[e] += a * P[e];
      const double rv = R[e] - a * W[e];
      R[e] = rv;
      s += rv * rv;
    }
  }
  red[threadIdx.x] = rg < G ? s : 0.0;
  __syncthreads();
  if ((int)threadIdx.x < tp) {
    double t = 0.0;
    for (int q = 0; q < G; ++q) t += red[q * tp + threadIdx.x];
    part[(int64_t)blockIdx.x * tp + threadIdx.x] = t;
  }
}

// convergence test after the update; pact[b] = columns of problem b still active
__global__ void kb_check(const BDesc* __restrict__ desc, const double* __restrict__ part, int tp, int it, double tol,
                         const double* __restrict__ bnorm, int* __restrict__ active, int* __restrict__ iters,
                         double* __restrict__ rnorm, int* __restrict__ nactive_next, const int* __restrict__ nactive,
                         int* __restrict__ pact) {
  if (*nactive == 0) return;
  const int b = blockIdx.x, c = threadIdx.x;
  int still = 0;
  if (c < tp) {
    const int e = b * tp + c;
    if (active[e]) {
      const double rr = problem_total(part, desc[b], tp, c);
      iters[e] = it + 1;
      rnorm[e] = sqrt(rr);
      if (sqrt(rr) <= tol * bnorm[e]) {
        active[e] = 0;
      } else {
        still = 1;
        atomicAdd(nactive_next, 1);
      }
    }
  }
  const int cnt = __syncthreads_count(still);
  if (threadIdx.x == 0) pact[b] = cnt;
}

__global__ void kb_beta(const BDesc* __restrict__ desc, const double* __restrict__ part, int tp, int it,
                        int max_iters, double* __restrict__ rho, const int* __restrict__ active,
                        double* __restrict__ beta, double* __restrict__ blog, const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int b = blockIdx.x, c = threadIdx.x;
  if (c >= tp) return;
  const int e = b * tp + c;
  double bt = 0.0;
  if (active[e]) {
    const double rz = problem_total(part, desc[b], tp, c);
    bt = rz / rho[e];
    rho[e] = rz;
    blog[(int64_t)e * max_iters + it] = bt;
  }
  beta[e] = bt;
}

__global__ void kb_p(const int32_t* __restrict__ blkprob, double* __restrict__ P, const double* __restrict__ Z,
                     const double* __restrict__ beta, const int* __restrict__ active, int tp, int64_t count,
                     const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int64_t row = e / tp;
  const int c = (int)(e % tp);
  const int b = blkprob[row / kBRows];
  if (active[b * tp + c]) P[e] = Z[e] + beta[b * tp + c] * P[e];
}

__global__ void kb_swap(int* __restrict__ nactive, int* __restrict__ nactive_next) {
  *nactive = *nactive_next;
  *nactive_next = 0;
}

// ---------------------------------------------------------------------------
// Lanczos quadrature and log p per problem
// ---------------------------------------------------------------------------
// one workgroup per (problem, probe), as k_slq (QR up to kSlqQrMax steps, else the
// quadrature of tridiag_log_e1 with the problem's spectral lower bound)
__global__ __launch_bounds__(256) void kb_slq(const BDesc* __restrict__ desc, const double* __restrict__ alog,
                                              const double* __restrict__ blog, const int* __restrict__ iters,
                                              const double* __restrict__ rho0, int ell, int tp, int max_iters,
                                              double* __restrict__ gamma, int* __restrict__ flags) {
  extern __shared__ double sm_tri[];
  __shared__ int bad;
  const int b = blockIdx.x / ell, i = blockIdx.x % ell;
  const int e = b * tp + 1 + i;
  const int m = iters[e];
  if (m == 0) {
    if (threadIdx.x == 0) gamma[b * ell + i] = 0.0;
    return;
  }
  const BDesc& D = desc[b];
  double* a = sm_tri;
  double* bb = a + max_iters;
  double* z = bb + max_iters;
  double* red = z + max_iters;
  const double* al = alog + (int64_t)e * max_iters;
  const double* be = blog + (int64_t)e * max_iters;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    a[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < m) bb[j] = be[j] / (al[j] * al[j]);
  }
  __syncthreads();
  if (m > kSlqQrMax) {
    double v;
    const double lam_lo = D.s2 / (D.s2 + (double)D.n * D.s);
    if (tridiag_log_e1(a, bb, m, lam_lo, red, &bad, &v)) {
      if (threadIdx.x == 0) gamma[b * ell + i] = rho0[e] * v;
      return;
    }
  }
  if (threadIdx.x != 0) return;
  for (int j = 0; j + 1 < m; ++j) bb[j] = sqrt(bb[j]);
  tridiag_eig_first_row(a, bb, z, m);
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
  gamma[b * ell + i] = rho0[e] * s;
  if (cl) atomicAdd(flags + b * 4 + 2, cl);
}

__global__ __launch_bounds__(256) void kb_logp(const BDesc* __restrict__ desc, const double* __restrict__ y,
                                               const double* __restrict__ Xs, int tp, int t, int ell,
                                               const double* __restrict__ gamma, const double* __restrict__ logdetP,
                                               const int* __restrict__ active, const int32_t* __restrict__ stop,
                                               int* __restrict__ flags, double* __restrict__ aux,
                                               double* __restrict__ logp) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  const BDesc& D = desc[b];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < D.n; i += 256) s += y[D.xoff + i] * Xs[(D.off + i) * tp];
  const double yu = bsum(s, red);
  if (threadIdx.x != 0) return;
  double g = 0.0;
  for (int i = 0; i < ell; ++i) g += gamma[b * ell + i];
  const double ld = logdetP[b] + (ell > 0 ? g / ell : 0.0);
  aux[2 * b] = yu;
  aux[2 * b + 1] = ld;
  logp[b] = -0.5 * (yu + ld + (double)D.n * 1.8378770664093453);
  int f = 0;
  for (int c = 0; c < t; ++c)
    if (active[b * tp + c]) f |= GP_FLAG_NOT_CONVERGED;
  if (stop[b]) f |= GP_FLAG_RANK_DEFICIENT;
  if (flags[b * 4 + 2] > 0) f |= GP_FLAG_RITZ_CLAMPED;
  flags[b * 4] = f;
}

// ---------------------------------------------------------------------------
// gradient
// ---------------------------------------------------------------------------

// C' = [u/2 | -c_i / (2 ell) | 0]
__global__ void kb_cprime(const double* __restrict__ Xs, const double* __restrict__ Z0, int64_t count, int tp, int ell,
                          double* __restrict__ Cp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int c = (int)(e % tp);
  double v = 0.0;
  if (c == 0) v = 0.5 * Xs[e];
  else if (c <= ell) v = -Z0[e] / (2.0 * ell);
  Cp[e] = v;
}

// Kernel-derivative sweep in FP64 (VALU): every pair (p, q) of one problem's
// diagonal block, rebuilt on the fly.  Thread = row p; columns q staged in LDS
// 32 at a time.  Per pair: r^2, kappa, g, M_pq = A'_p . C'_q, then
//   ls_j: s g M (x~_pj - x~_qj)^2,   s: M kappa.
// Item = int4 {first row, column begin, column end, problem}.
template <int KIND, int NT, int DM>
__global__ __launch_bounds__(256) void kb_bwd(const BDesc* __restrict__ desc, const int4* __restrict__ items,
                                              const double* __restrict__ xs, int d, const double* __restrict__ Xs,
                                              const double* __restrict__ Cp, double* __restrict__ part) {
  constexpr int TP = 16 * NT;
  constexpr int QC = 32;
  __shared__ double xq[QC][DM];
  __shared__ double cq[QC][TP];
  __shared__ double red[256];
  const int4 it = items[blockIdx.x];
  const BDesc& D = desc[it.w];
  const int64_t p = (int64_t)it.x + threadIdx.x;
  const bool valid = p - D.off < D.n;
  double ap[TP], xp[DM], acc[DM];
  double accs = 0.0;
#pragma unroll
  for (int c = 0; c < TP; ++c) ap[c] = valid ? Xs[p * TP + c] : 0.0;
#pragma unroll
  for (int j = 0; j < DM; ++j) {
    xp[j] = (valid && j < d) ? xs[p * d + j] : 0.0;
    acc[j] = 0.0;
  }
  const int64_t cend = min((int64_t)it.z, D.off + D.n);
  for (int64_t c0 = it.y; c0 < cend; c0 += QC) {
    const int nq = (int)min((int64_t)QC, cend - c0);
    for (int e = threadIdx.x; e < QC * DM; e += 256) {
      const int q = e / DM, j = e % DM;
      xq[q][j] = (q < nq && j < d) ? xs[(c0 + q) * d + j] : 0.0;
    }
    for (int e = threadIdx.x; e < QC * TP; e += 256) {
      const int q = e / TP, c = e % TP;
      cq[q][c] = q < nq ? Cp[(c0 + q) * TP + c] : 0.0;
    }
    __syncthreads();
    if (valid) {
      for (int q = 0; q < nq; ++q) {
        double df2[DM];
        double r2 = 0.0;
#pragma unroll
        for (int j = 0; j < DM; ++j) {
          const double df = xp[j] - xq[q][j];
          df2[j] = df * df;
          r2 += df2[j];
        }
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < TP; ++c) m += ap[c] * cq[q][c];
        double kap, g;
        kappa_g64(KIND, r2, &kap, &g, 1.0);
        const double wg = D.s * g * m;
#pragma unroll
        for (int j = 0; j < DM; ++j) acc[j] += wg * df2[j];
        accs += m * kap;
      }
    }
    __syncthreads();
  }
  for (int j = 0; j < d; ++j) {
    const double v = bsum(acc[j] * D.inv_ls[j], red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (GP_MAX_D + 1) + j] = v;
  }
  const double v = bsum(accs, red);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (GP_MAX_D + 1) + d] = v;
}

// Preconditioner-derivative algebra per problem: L^T [c_i], then the k x k
// quantities (LS^-1, G = C^-1 LS^-1, Psi, U) and the pivot-pair term
// sum_{q,r} Psi_qr dK(x_{S_q}, x_{S_r}).
__global__ __launch_bounds__(1024) void kb_pg_small(const BDesc* __restrict__ desc, int K, int tp, int ell, int d,
                                                    int kind, int mode, const double* __restrict__ Lall,
                                                    const double* __restrict__ Z0, const int32_t* __restrict__ piv,
                                                    const int32_t* __restrict__ kach, const double* __restrict__ Cinv,
                                                    const double* __restrict__ xs, double* __restrict__ Tb,
                                                    double* __restrict__ pgs, double* __restrict__ pg_psi) {
  __shared__ double red[1024];
  const int b = blockIdx.x;
  const BDesc& D = desc[b];
  const int k = D.k;
  if (k == 0) {
    if (threadIdx.x <= d) pg_psi[b * (GP_MAX_D + 1) + threadIdx.x] = 0.0;
    return;
  }
  const double* Lb = Lall + D.loff;
  double* T = Tb + (int64_t)b * K * tp;
  for (int e = threadIdx.x; e < k * tp; e += 1024) {
    const int l = e / tp, c = e % tp;
    double s = 0.0;
    for (int64_t i = 0; i < D.n; ++i) s += Lb[(int64_t)l * D.n_pad + i] * Z0[(D.off + i) * tp + c];
    T[l * tp + c] = s;
  }
  __syncthreads();
  const int64_t kk = (int64_t)K * K;
  double* base = pgs + (int64_t)b * (4 * kk + (int64_t)K * tp);
  double* LSinv = base;
  double* Gk = base + kk;
  double* Psi = base + 2 * kk;
  double* tmp = base + 3 * kk;
  double* U = base + 4 * kk;
  pg_small_body(Lb, piv + b * K, kach + b, D.n_pad, k, Cinv + b * kk, T, tp, ell, D.s2, LSinv, Gk, Psi, U, tmp);
  __syncthreads();
  const int kp = kach[b];
  const double* xb = xs + D.off * d;
  double acc[GP_MAX_D + 1];
  for (int j = 0; j <= d; ++j) acc[j] = 0.0;
  for (int e = threadIdx.x; e < kp * kp; e += 1024) {
    const int q = e / kp, r = e % kp;
    const double w = Psi[q * k + r];
    const int64_t a = piv[b * K + q], c = piv[b * K + r];
    double r2 = 0.0, df2[GP_MAX_D];
    for (int j = 0; j < d; ++j) {
      const double df = xb[a * d + j] - xb[c * d + j];
      df2[j] = df * df;
      r2 += df2[j];
    }
    double kap, g;
    kappa_g64(kind, r2, &kap, &g, 1.0);
    if (mode == 0)
      for (int j = 0; j < d; ++j) acc[j] += w * D.s * g * df2[j];
    acc[d] += w * kap;
  }
  for (int j = 0; j <= d; ++j) {
    const double v = bsum(j < d ? acc[j] * D.inv_ls[j] : acc[j], red);
    if (threadIdx.x == 0) pg_psi[b * (GP_MAX_D + 1) + j] = v;
  }
}

// rows of one problem against its pivots: sum_q Omega_iq dK(x_i, x_{S_q}) with
// Omega = -L G + (1/ell) [c_1..c_ell] U^T
__global__ __launch_bounds__(256) void kb_pg_rows(const BDesc* __restrict__ desc, const int32_t* __restrict__ blkprob,
                                                  int K, int tp, int ell, int d, int kind, int mode,
                                                  const double* __restrict__ Lall, const double* __restrict__ Z0,
                                                  const int32_t* __restrict__ piv, const int32_t* __restrict__ kach,
                                                  const double* __restrict__ xs, const double* __restrict__ pgs,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const int b = blkprob[blockIdx.x];
  const BDesc& D = desc[b];
  const int k = D.k;
  const int64_t i = (int64_t)(blockIdx.x - D.blk0) * kBRows + threadIdx.x;
  double acc[GP_MAX_D + 1];
  for (int j = 0; j <= d; ++j) acc[j] = 0.0;
  if (k > 0 && i < D.n) {
    const int kp = kach[b];
    const int64_t kk = (int64_t)K * K;
    const double* base = pgs + (int64_t)b * (4 * kk + (int64_t)K * tp);
    const double* Gk = base + kk;
    const double* U = base + 4 * kk;
    const double* Lb = Lall + D.loff;
    const double* xb = xs + D.off * d;
    const double* zr = Z0 + (D.off + i) * tp;
    for (int q = 0; q < kp; ++q) {
      double om = 0.0;
      for (int r = 0; r < kp; ++r) om -= Lb[(int64_t)r * D.n_pad + i] * Gk[r * k + q];
      double cu = 0.0;
      for (int c = 0; c < ell; ++c) cu += zr[1 + c] * U[q * tp + c];
      om += cu / ell;
      const int64_t sq = piv[b * K + q];
      double r2 = 0.0, df2[GP_MAX_D];
      for (int j = 0; j < d; ++j) {
        const double df = xb[i * d + j] - xb[sq * d + j];
        df2[j] = df * df;
        r2 += df2[j];
      }
      double kap, g;
      kappa_g64(kind, r2, &kap, &g, 1.0);
      if (mode == 0)
        for (int j = 0; j < d; ++j) acc[j] += om * D.s * g * df2[j];
      acc[d] += om * kap;
    }
  }
  for (int j = 0; j <= d; ++j) {
    const double v = bsum(j < d ? acc[j] * D.inv_ls[j] : acc[j], red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (GP_MAX_D + 1) + j] = v;
  }
}

// gradient assembly per problem: [ls | s | sigma^2]
__global__ __launch_bounds__(256) void kb_grad_final(const BDesc* __restrict__ desc, int d, int ard, int tp, int ell,
                                                     int K, const double* __restrict__ bwd_part,
                                                     const double* __restrict__ pg_part,
                                                     const double* __restrict__ pg_psi,
                                                     const double* __restrict__ Xs, const double* __restrict__ Cp,
                                                     const double* __restrict__ Z0, const double* __restrict__ Cinv,
                                                     double* __restrict__ grad) {
  __shared__ double red[256];
  __shared__ double bil[GP_MAX_D + 1], pg[GP_MAX_D + 1];
  const int b = blockIdx.x;
  const BDesc& D = desc[b];
  for (int j = 0; j <= d; ++j) {
    double s = 0.0, q = 0.0;
    for (int it = threadIdx.x; it < D.nbitem; it += 256) s += bwd_part[(int64_t)(D.bitem0 + it) * (GP_MAX_D + 1) + j];
    for (int q0 = threadIdx.x; q0 < D.nblk; q0 += 256) q += pg_part[(int64_t)(D.blk0 + q0) * (GP_MAX_D + 1) + j];
    s = bsum(s, red);
    q = bsum(q, red);
    if (threadIdx.x == 0) {
      bil[j] = s;
      pg[j] = D.k > 0 ? q + pg_psi[b * (GP_MAX_D + 1) + j] : 0.0;
    }
  }
  double trm = 0.0, cc = 0.0, tci = 0.0;
  for (int64_t e = threadIdx.x; e < D.n * tp; e += 256) {
    const int64_t row = D.off + e / tp;
    const int c = (int)(e % tp);
    trm += Xs[row * tp + c] * Cp[row * tp + c];
    if (c >= 1 && c <= ell) cc += Z0[row * tp + c] * Z0[row * tp + c];
  }
  for (int j = threadIdx.x; j < D.k; j += 256) tci += Cinv[(int64_t)b * K * K + (int64_t)j * D.k + j];
  trm = bsum(trm, red);
  cc = bsum(cc, red);
  tci = bsum(tci, red);
  if (threadIdx.x != 0) return;
  const double trPinv = (double)(D.n - D.k) / D.s2 + tci;
  const int p = ard ? d : 1;
  double* g = grad + (int64_t)b * (p + 2);
  if (ard) {
    for (int j = 0; j < d; ++j) g[j] = bil[j] + pg[j];
  } else {
    double s = 0.0;
    for (int j = 0; j < d; ++j) s += bil[j] + pg[j];
    g[0] = s;
  }
  g[p] = bil[d] + pg[d];
  g[p + 1] = trm - 0.5 * trPinv + cc / (2.0 * ell);
}

template <typename T>
T* at(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

unsigned nbl(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

template <int KIND, int NT>
hipError_t run_bwd_dm(const BLayout& L, char* ws, hipStream_t st) {
  const int dm = L.dm;
#define BWD_ARGS                                                                                               \
  at<BDesc>(ws, L.desc), at<int4>(ws, L.bitems), at<double>(ws, L.xs), L.d, at<double>(ws, L.Xs),              \
      at<double>(ws, L.cprime), at<double>(ws, L.bwd_part)
  if (dm == 4) hipLaunchKernelGGL((kb_bwd<KIND, NT, 4>), dim3(L.nbitems), dim3(256), 0, st, BWD_ARGS);
  else if (dm == 8) hipLaunchKernelGGL((kb_bwd<KIND, NT, 8>), dim3(L.nbitems), dim3(256), 0, st, BWD_ARGS);
  else if (dm == 16) hipLaunchKernelGGL((kb_bwd<KIND, NT, 16>), dim3(L.nbitems), dim3(256), 0, st, BWD_ARGS);
  else hipLaunchKernelGGL((kb_bwd<KIND, NT, 32>), dim3(L.nbitems), dim3(256), 0, st, BWD_ARGS);
#undef BWD_ARGS
  return hipGetLastError();
}

template <int KIND>
hipError_t run_bwd_nt(const BLayout& L, char* ws, hipStream_t st) {
  switch (L.tp / 16) {
    case 1: return run_bwd_dm<KIND, 1>(L, ws, st);
    case 2: return run_bwd_dm<KIND, 2>(L, ws, st);
    case 3: return run_bwd_dm<KIND, 3>(L, ws, st);
    case 4: return run_bwd_dm<KIND, 4>(L, ws, st);
    case 5: return run_bwd_dm<KIND, 5>(L, ws, st);
  }
  return hipErrorInvalidValue;
}

// Woodbury apply of Rsrc into Zdst with r.z partials in part
// pact: per-problem active-column counts (rows of finished problems are skipped), or NULL
hipError_t bl_woodbury(const BLayout& L, char* ws, hipStream_t st, const double* Rsrc, double* Zdst, double* part,
                       const int* nact, const int* pact) {
  const int KP = (L.K + 15) / 16 * 16;
  if (L.K > 0) {
    const dim3 g(L.nblk, (KP / 16 + 3) / 4);
#define BLTR(NT)                                                                                                  \
  hipLaunchKernelGGL((kb_ltr_mfma<NT>), g, dim3(256), 0, st, at<BDesc>(ws, L.desc), at<int32_t>(ws, L.blkprob),   \
                     at<double>(ws, L.L), Rsrc, KP, L.tp, at<double>(ws, L.ltr_part), nact, pact)
    switch (L.tp / 16) {
      case 1: BLTR(1); break;
      case 2: BLTR(2); break;
      case 3: BLTR(3); break;
      case 4: BLTR(4); break;
      case 5: BLTR(5); break;
      default: return hipErrorInvalidValue;
    }
#undef BLTR
    hipLaunchKernelGGL(kb_wood_y, dim3(L.B), dim3(256), 0, st, at<BDesc>(ws, L.desc), at<double>(ws, L.ltr_part),
                       at<double>(ws, L.Cinv), L.K, KP, L.tp, at<double>(ws, L.Tb), at<double>(ws, L.Y), nact);
  }
#define BZAP(NT)                                                                                                   \
  hipLaunchKernelGGL((kb_zapply_mfma<NT>), dim3(L.nblk), dim3(256), 0, st, at<BDesc>(ws, L.desc),                  \
                     at<int32_t>(ws, L.blkprob), at<double>(ws, L.L), at<double>(ws, L.Y), Rsrc, L.K, L.tp, Zdst, part, \
                     nact, pact)
  switch (L.tp / 16) {
    case 1: BZAP(1); break;
    case 2: BZAP(2); break;
    case 3: BZAP(3); break;
    case 4: BZAP(4); break;
    case 5: BZAP(5); break;
    default: return hipErrorInvalidValue;
  }
#undef BZAP
  return hipGetLastError();
}

}  // namespace

hipError_t bl_zero_flags(const BLayout& L, char* ws, hipStream_t st) {
  hipLaunchKernelGGL(kb_zero_i32, dim3(nbl(4 * L.B, 256)), dim3(256), 0, st, at<int>(ws, L.flags), (int64_t)4 * L.B);
  hipLaunchKernelGGL(kb_zero_i32, dim3(1), dim3(256), 0, st, at<int>(ws, L.nactive), (int64_t)2);
  return hipGetLastError();
}

hipError_t bl_prep(const BLayout& L, char* ws, hipStream_t st, const double* X) {
  hipLaunchKernelGGL(kb_prep, dim3(L.B), dim3(256), 0, st, X, at<BDesc>(ws, L.desc), L.d, at<double>(ws, L.xs));
  return hipGetLastError();
}

hipError_t bl_precond(const BLayout& L, char* ws, hipStream_t st) {
  if (L.K > 0)
    hipLaunchKernelGGL(kb_pivchol, dim3(L.B), dim3(1024), 0, st, at<BDesc>(ws, L.desc), L.d, L.kind, L.K,
                       at<double>(ws, L.xs), at<double>(ws, L.L), at<double>(ws, L.diag), at<int8_t>(ws, L.ispiv),
                       at<int32_t>(ws, L.piv), at<int32_t>(ws, L.kach), at<int32_t>(ws, L.stop));
  else
    hipLaunchKernelGGL(kb_zero_i32, dim3(nbl(2 * L.B, 256)), dim3(256), 0, st, at<int>(ws, L.kach), (int64_t)2 * L.B);
  hipLaunchKernelGGL(kb_gram_chol, dim3(L.B), dim3(1024), 0, st, at<BDesc>(ws, L.desc), L.K, at<double>(ws, L.L),
                     at<double>(ws, L.C), at<double>(ws, L.Rc), at<double>(ws, L.Rinv), at<double>(ws, L.Cinv),
                     at<double>(ws, L.logdetP), at<int>(ws, L.flags));
  return hipGetLastError();
}

hipError_t bl_probes(const BLayout& L, char* ws, hipStream_t st, const double* y) {
  if (L.K > 0)
    hipLaunchKernelGGL(kb_eta, dim3(nbl((int64_t)L.K * L.ell, 256), L.B), dim3(256), 0, st, at<BDesc>(ws, L.desc), L.K,
                       L.ell, at<double>(ws, L.H));
  hipLaunchKernelGGL(kb_probes, dim3(L.nblk), dim3(kBRows), 0, st, at<BDesc>(ws, L.desc), at<int32_t>(ws, L.blkprob), y,
                     at<double>(ws, L.L), at<double>(ws, L.H), L.K, L.ell, L.tp, at<double>(ws, L.R),
                     at<double>(ws, L.Xs));
  return hipGetLastError();
}

hipError_t bl_cg_init(const BLayout& L, char* ws, hipStream_t st) {
  double* part = at<double>(ws, L.part);
  double* part2 = at<double>(ws, L.part2);
  hipLaunchKernelGGL(kb_coldot, dim3(L.nblk), dim3(256), 0, st, at<double>(ws, L.R), at<double>(ws, L.R), L.tp, part);
  hipError_t e = bl_woodbury(L, ws, st, at<double>(ws, L.R), at<double>(ws, L.Z0), part2, nullptr, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_cg_start, dim3(L.B), dim3(256), 0, st, at<BDesc>(ws, L.desc), part, part2, L.tp, L.t,
                     at<double>(ws, L.bnorm), at<double>(ws, L.rho), at<double>(ws, L.rho0), at<int>(ws, L.active),
                     at<int>(ws, L.iters), at<int>(ws, L.nactive), at<int>(ws, L.pact));
  const int64_t cnt = L.N * L.tp;
  hipLaunchKernelGGL(kb_copy, dim3(nbl(cnt, 256)), dim3(256), 0, st, at<double>(ws, L.Z0), at<double>(ws, L.Pd), cnt);
  return hipGetLastError();
}

hipError_t bl_reduce(const BLayout& L, char* ws, hipStream_t st) {
  const int* nact = at<int>(ws, L.nactive);
  if (L.prec == GP_PREC_FP64)
    hipLaunchKernelGGL(kb_reduce<double>, dim3(L.nblk), dim3(256), 0, st, at<BDesc>(ws, L.desc),
                       at<int32_t>(ws, L.blkprob), at<double>(ws, L.view.wpart), L.N, L.tp, at<double>(ws, L.Pd),
                       at<double>(ws, L.W), at<double>(ws, L.part), nact, at<int>(ws, L.pact));
  else
    hipLaunchKernelGGL(kb_reduce<float>, dim3(L.nblk), dim3(256), 0, st, at<BDesc>(ws, L.desc),
                       at<int32_t>(ws, L.blkprob), at<float>(ws, L.view.wpart), L.N, L.tp, at<double>(ws, L.Pd),
                       at<double>(ws, L.W), at<double>(ws, L.part), nact, at<int>(ws, L.pact));
  return hipGetLastError();
}

hipError_t bl_cg_after_product(const BLayout& L, char* ws, hipStream_t st, int it, double tol) {
  int* nact = at<int>(ws, L.nactive);
  int* nact_next = nact + 1;
  const BDesc* desc = at<BDesc>(ws, L.desc);
  double* part = at<double>(ws, L.part);
  double* part2 = at<double>(ws, L.part2);
  hipLaunchKernelGGL(kb_alpha, dim3(L.B), dim3(256), 0, st, desc, part, L.tp, it, L.max_iters, at<double>(ws, L.rho),
                     at<int>(ws, L.active), at<double>(ws, L.alpha), at<double>(ws, L.alog), at<int>(ws, L.flags),
                     nact);
  hipLaunchKernelGGL(kb_update, dim3(L.nblk), dim3(256), 0, st, at<int32_t>(ws, L.blkprob), at<double>(ws, L.Xs),
                     at<double>(ws, L.R), at<double>(ws, L.Pd), at<double>(ws, L.W), at<double>(ws, L.alpha),
                     at<int>(ws, L.active), L.tp, part, nact, at<int>(ws, L.pact));
  hipLaunchKernelGGL(kb_check, dim3(L.B), dim3(256), 0, st, desc, part, L.tp, it, tol, at<double>(ws, L.bnorm),
                     at<int>(ws, L.active), at<int>(ws, L.iters), at<double>(ws, L.rnorm), nact_next, nact,
                     at<int>(ws, L.pact));
  hipError_t e = bl_woodbury(L, ws, st, at<double>(ws, L.R), at<double>(ws, L.W), part2, nact, at<int>(ws, L.pact));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_beta, dim3(L.B), dim3(256), 0, st, desc, part2, L.tp, it, L.max_iters, at<double>(ws, L.rho),
                     at<int>(ws, L.active), at<double>(ws, L.beta), at<double>(ws, L.blog), nact);
  hipLaunchKernelGGL(kb_p, dim3(nbl(L.N * L.tp, 256)), dim3(256), 0, st, at<int32_t>(ws, L.blkprob),
                     at<double>(ws, L.Pd), at<double>(ws, L.W), at<double>(ws, L.beta), at<int>(ws, L.active), L.tp,
                     L.N * L.tp, nact);
  hipLaunchKernelGGL(kb_swap, dim3(1), dim3(1), 0, st, nact, nact_next);
  return hipGetLastError();
}

hipError_t bl_slq_logp(const BLayout& L, char* ws, hipStream_t st, const double* y, double* logp) {
  const size_t smem = ((size_t)3 * L.max_iters + 256) * sizeof(double);
  if (smem > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kb_slq, dim3(L.B * L.ell), dim3(256), smem, st, at<BDesc>(ws, L.desc), at<double>(ws, L.alog),
                     at<double>(ws, L.blog), at<int>(ws, L.iters), at<double>(ws, L.rho0), L.ell, L.tp, L.max_iters,
                     at<double>(ws, L.gamma), at<int>(ws, L.flags));
  hipLaunchKernelGGL(kb_logp, dim3(L.B), dim3(256), 0, st, at<BDesc>(ws, L.desc), y, at<double>(ws, L.Xs), L.tp, L.t,
                     L.ell, at<double>(ws, L.gamma), at<double>(ws, L.logdetP), at<int>(ws, L.active),
                     at<int32_t>(ws, L.stop), at<int>(ws, L.flags), at<double>(ws, L.logp_aux), logp);
  return hipGetLastError();
}

hipError_t bl_backward(const BLayout& L, char* ws, hipStream_t st, int precond_grad, double* grad) {
  const int64_t cnt = L.N * L.tp;
  hipLaunchKernelGGL(kb_cprime, dim3(nbl(cnt, 256)), dim3(256), 0, st, at<double>(ws, L.Xs), at<double>(ws, L.Z0), cnt,
                     L.tp, L.ell, at<double>(ws, L.cprime));
  hipError_t e;
  switch (L.kind) {
    case GP_KERNEL_RBF: e = run_bwd_nt<GP_KERNEL_RBF>(L, ws, st); break;
    case GP_KERNEL_MATERN32: e = run_bwd_nt<GP_KERNEL_MATERN32>(L, ws, st); break;
    default: e = run_bwd_nt<GP_KERNEL_MATERN52>(L, ws, st); break;
  }
  if (e != hipSuccess) return e;
  if (L.K > 0) {
    hipLaunchKernelGGL(kb_pg_small, dim3(L.B), dim3(1024), 0, st, at<BDesc>(ws, L.desc), L.K, L.tp, L.ell, L.d, L.kind,
                       precond_grad, at<double>(ws, L.L), at<double>(ws, L.Z0), at<int32_t>(ws, L.piv),
                       at<int32_t>(ws, L.kach), at<double>(ws, L.Cinv), at<double>(ws, L.xs), at<double>(ws, L.Tb),
                       at<double>(ws, L.pgs), at<double>(ws, L.pg_psi));
    hipLaunchKernelGGL(kb_pg_rows, dim3(L.nblk), dim3(256), 0, st, at<BDesc>(ws, L.desc), at<int32_t>(ws, L.blkprob),
                       L.K, L.tp, L.ell, L.d, L.kind, precond_grad, at<double>(ws, L.L), at<double>(ws, L.Z0),
                       at<int32_t>(ws, L.piv), at<int32_t>(ws, L.kach), at<double>(ws, L.xs), at<double>(ws, L.pgs),
                       at<double>(ws, L.pg_part));
  }
  hipLaunchKernelGGL(kb_grad_final, dim3(L.B), dim3(256), 0, st, at<BDesc>(ws, L.desc), L.d, L.ard, L.tp, L.ell, L.K,
                     at<double>(ws, L.bwd_part), at<double>(ws, L.pg_part), at<double>(ws, L.pg_psi),
                     at<double>(ws, L.Xs), at<double>(ws, L.cprime), at<double>(ws, L.Z0), at<double>(ws, L.Cinv),
                     grad);
  return hipGetLastError();
}

}  // namespace gpmll
