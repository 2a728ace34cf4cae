// Batched preconditioned CG over the t = 1 + ell right hand sides [y | b_1..b_ell]
// (one CG call with many right hand sides: footnote to Section 4.4; preconditioned
// CG: Section 2.2 and supplement S1.1), all recurrences in FP64.
//
// Per iteration and per active column c:
//   w = K_hat p;  alpha = rho / p.w;  x += alpha p;  r -= alpha w;
//   stop the column once ||r|| <= tol ||b||;
//   z = P_hat^-1 r = (r - L C^-1 L^T r) / sigma^2   (matrix inversion lemma);
//   beta = r.z / rho;  rho = r.z;  p = z + beta p.
// alpha and beta are logged per column for the Lanczos tridiagonal.
//
// Reductions over n are two-stage with a fixed order: row-block partials, then one
// workgroup per column.  No floating-point atomics.
#include "gpmll_impl.h"

namespace gpmll {

// ---- row-block partial column dots: part[b][c] = sum_{rows of b} A[i][c] * B[i][c]
__global__ void k_coldot_part(const double* __restrict__ A, const double* __restrict__ B, int64_t n, int tp,
                              int64_t rows_per_block, double* __restrict__ part) {
  __shared__ double red[256];
  const int G = 256 / tp;
  const int c = threadIdx.x % tp, rg = threadIdx.x / tp;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  double s = 0.0;
  if (rg < G)
    for (int64_t r = r0 + rg; r < r1; r += G) s += A[r * tp + c] * B[r * tp + c];
  red[threadIdx.x] = (rg < G) ? s : 0.0;
  __syncthreads();
  if (threadIdx.x < tp) {
    double t = 0.0;
    for (int q = 0; q < G; ++q) t += red[q * tp + threadIdx.x];
    part[(int64_t)blockIdx.x * tp + threadIdx.x] = t;
  }
}

// sum of nblk partials of column blockIdx.x (one workgroup per column)
__device__ double column_total(const double* __restrict__ part, int nblk, int tp, int c) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(int64_t)b * tp + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// CG start: bnorm = ||b||, rho = rho0 = r.z, masks; Pd = Z0 copy happens in k_copy
__global__ void k_cg_start(const double* __restrict__ part_bb, int nblk_bb, const double* __restrict__ part_rz,
                           int nblk_rz, int tp,
                           int t, double* __restrict__ bnorm, double* __restrict__ rho, double* __restrict__ rho0,
                           int* __restrict__ active, int* __restrict__ iters, int* __restrict__ nactive) {
  const int c = blockIdx.x;
  const double bb = column_total(part_bb, nblk_bb, tp, c);
  const double rz = column_total(part_rz, nblk_rz, tp, c);
  if (threadIdx.x == 0) {
    bnorm[c] = sqrt(bb);
    rho[c] = rz;
    rho0[c] = rz;
    const int act = (c < t && bb > 0.0) ? 1 : 0;
    active[c] = act;
    iters[c] = 0;
    if (act) atomicAdd(nactive, 1);
  }
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) b[e] = a[e];
}

__global__ void k_zero_int(int* p) { *p = 0; }

// alpha = rho / p.w for active columns; logs alpha; p.w <= 0 is a hard error
__global__ void k_cg_alpha(const double* __restrict__ part_pw, int nblk, int tp, int it, int max_iters,
                           const double* __restrict__ rho, const int* __restrict__ active, double* __restrict__ alpha,
                           double* __restrict__ alog, int* __restrict__ status, const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int c = blockIdx.x;
  const double pw = column_total(part_pw, nblk, tp, c);
  if (threadIdx.x == 0) {
    double a = 0.0;
    if (active[c]) {
      if (!(pw > 0.0)) {
        *status = GP_ENOTSPD;
      } else {
        a = rho[c] / pw;
        alog[(int64_t)c * max_iters + it] = a;
      }
    }
    alpha[c] = a;
  }
}

typedef double f64x4v __attribute__((ext_vector_type(4)));

// x += alpha p; r -= alpha w (active columns); partial ||r||^2.  Thread = column x
// 256 / tp row lanes.  (Four-column vector loads, as k_cg_p and k_khat_reduce use,
// were measured slower here at n = 100k: 84.5 against 68.9 us.)
__global__ void k_cg_update(double* __restrict__ X, double* __restrict__ R, const double* __restrict__ P,
                            const double* __restrict__ W, const double* __restrict__ alpha,
                            const int* __restrict__ active, int64_t n, int tp, int64_t rows_per_block,
                            double* __restrict__ part, const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  __shared__ double red[256];
  const int G = 256 / tp;
  const int c = threadIdx.x % tp, rg = threadIdx.x / tp;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  double s = 0.0;
  if (rg < G && active[c]) {
    const double a = alpha[c];
#pragma unroll 4
    for (int64_t r = r0 + rg; r < r1; r += G) {
      const int64_t e = r * tp + c;
      X[e] += a * P[e];
      const double rv = R[e] - a * W[e];
      R[e] = rv;
      s += rv * rv;
    }
  }
  red[threadIdx.x] = (rg < G) ? s : 0.0;
  __syncthreads();
  if (threadIdx.x < tp) {
    double t = 0.0;
    for (int q = 0; q < G; ++q) t += red[q * tp + threadIdx.x];
    part[(int64_t)blockIdx.x * tp + threadIdx.x] = t;
  }
}

// convergence test after the update: iteration count, residual, mask
__global__ void k_cg_check(const double* __restrict__ part_rr, int nblk, int tp, int it, double tol,
                           const double* __restrict__ bnorm, int* __restrict__ active, int* __restrict__ iters,
                           double* __restrict__ rnorm, int* __restrict__ nactive_next,
                           const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int c = blockIdx.x;
  const double rr = column_total(part_rr, nblk, tp, c);
  if (threadIdx.x == 0 && active[c]) {
    iters[c] = it + 1;
    rnorm[c] = sqrt(rr);
    if (sqrt(rr) <= tol * bnorm[c]) active[c] = 0;
    else atomicAdd(nactive_next, 1);
  }
}

// beta = r.z / rho; rho = r.z (active columns)
__global__ void k_cg_beta(const double* __restrict__ part_rz, int nblk, int tp, int it, int max_iters,
                          double* __restrict__ rho, const int* __restrict__ active, double* __restrict__ beta,
                          double* __restrict__ blog, const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int c = blockIdx.x;
  const double rz = column_total(part_rz, nblk, tp, c);
  if (threadIdx.x == 0) {
    double b = 0.0;
    if (active[c]) {
      b = rz / rho[c];
      rho[c] = rz;
      blog[(int64_t)c * max_iters + it] = b;
    }
    beta[c] = b;
  }
}

// p = z + beta p on active columns; thread = four consecutive columns (one 32-byte
// load per array and row) x 1024 / tp row lanes (tp <= 256), rows_per_block rows per
// workgroup as in k_cg_update; a quad with no active column is skipped
__global__ __launch_bounds__(256) void k_cg_p(double* __restrict__ P, const double* __restrict__ Z,
                                              const double* __restrict__ beta, const int* __restrict__ active,
                                              int64_t n, int tp, int64_t rows_per_block,
                                              const int* __restrict__ nactive) {
  if (*nactive == 0) return;
  const int nq = tp / 4, G = 256 / nq;
  const int cq = threadIdx.x % nq, rg = threadIdx.x / nq;
  if (rg >= G) return;
  bool act[4];
  double b[4];
  bool any = false;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    act[v] = active[4 * cq + v] != 0;
    b[v] = act[v] ? beta[4 * cq + v] : 0.0;
    any = any || act[v];
  }
  if (!any) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
#pragma unroll 2
  for (int64_t r = r0 + rg; r < r1; r += G) {
    const int64_t e = r * tp + 4 * cq;
    const f64x4v z = *reinterpret_cast<const f64x4v*>(Z + e);
    f64x4v p = *reinterpret_cast<const f64x4v*>(P + e);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (act[v]) p[v] = z[v] + b[v] * p[v];
    *reinterpret_cast<f64x4v*>(P + e) = p;
  }
}

// colmap = active columns in increasing order, then -1 (one lane: tp <= 256)
__global__ void k_colmap(const int* __restrict__ active, int tp, int* __restrict__ colmap) {
  if (threadIdx.x != 0) return;
  int m = 0;
  for (int c = 0; c < tp; ++c)
    if (active[c]) colmap[m++] = c;
  for (; m < tp; ++m) colmap[m] = -1;
}

__global__ void k_swap_count(int* __restrict__ nactive, int* __restrict__ nactive_next) {
  *nactive = *nactive_next;
  *nactive_next = 0;
}

// ---------------------------------------------------------------------------
// Woodbury apply Z = (R - L Y) / sigma^2 with Y = C^-1 L^T R, both products on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64: A lane l = (row l%16, k l/16),
// B lane l = (k l/16, column l%16), D lane l = rows l/16 + 4v, column l%16).
// ---------------------------------------------------------------------------

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// part[chunk][l][c] = sum over the chunk's rows i of L[l][i] R[i][c], l < kpad,
// c < tp.  Workgroup (group of kLtrWaves waves, chunk); a wave owns LB consecutive
// blocks of 16 l and every 16-column tile of R, which the workgroup's waves read from
// LDS (one l-block per wave measured faster than two once R came from LDS).  The
// l-groups of one chunk are neighbours in launch order, so the chunk of R comes from
// HBM once.  XC = 1: R has 16 NT + 1 meaningful columns (y and 16 NT probes) in
// 16 (NT + 1); the NT tiles run on the matrix cores and column 16 NT on the vector ALU
// (one FP64 FMA per L value instead of a sixteen-column MFMA tile that carries one
// column), and the padding columns of part are written as zero.
template <int NT>
constexpr int ltr_lblocks() { return 1; }
constexpr int kLtrWaves = 8;

template <int NT, int XC>
__global__ __launch_bounds__(64 * kLtrWaves) void k_ltr_mfma(const double* __restrict__ lf, const double* __restrict__ R,
                                                  int64_t n, int kpad, int tp, int64_t rows,
                                                  double* __restrict__ part, const int* __restrict__ nactive) {
  if (nactive != nullptr && *nactive == 0) return;
  constexpr int LB = ltr_lblocks<NT>();
  // R rows of 16 (NT + XC) doubles (tp), 16 rows per group, two LDS buffers
  constexpr int TPC = 16 * (NT + XC);
  __shared__ __attribute__((aligned(16))) double rs[2][16 * TPC];
  // the wave index through the scalar unit, so the l-block tests below are uniform branches
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int mb0 = (blockIdx.x * kLtrWaves + wave) * LB;
  const int64_t i0 = (int64_t)blockIdx.y * rows, i1 = min(n, i0 + rows);
  const int m = lane & 15, kq = lane >> 4;
  const int nlb = kpad / 16;
  bool on[LB];
#pragma unroll
  for (int b = 0; b < LB; ++b) on[b] = (mb0 + b) * 16 < kpad;
  f64x4 acc[LB][NT];
  double xacc[LB];
#pragma unroll
  for (int b = 0; b < LB; ++b) {
    xacc[b] = 0.0;
#pragma unroll
    for (int nb = 0; nb < NT; ++nb) acc[b][nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  // Per group of 16 rows (four K-steps): the group's R rows were copied global -> LDS
  // (global_load_lds, 1 KB per wave instruction, shared by the workgroup) and its L
  // operands loaded into registers during the previous group; L comes operand-ordered
  // (lf: zero past n and k) and needs no masks.  A chunk holds a multiple of 16 rows
  // except the last, which ends at n; R has n_pad >= rup(n, 16) rows, and rows past
  // the chunk are zeroed by a select.
  constexpr int U = 4;
  const int ng = (int)((i1 - i0 + 15) / 16);
  auto issue = [&](int g, double (&av)[LB][U]) {
    const int64_t i = i0 + 16 * g;
    const u32x4* src = reinterpret_cast<const u32x4*>(R + i * tp);
    u32x4* dst = reinterpret_cast<u32x4*>(rs[g & 1]);
    for (int un = wave; un < TPC / 8; un += kLtrWaves)
      __builtin_amdgcn_global_load_lds(src + un * 64 + lane, (__attribute__((address_space(3))) void*)(dst + un * 64),
                                       16, 0, 0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int b = 0; b < LB; ++b) av[b][u] = on[b] ? lf[((i / 4 + u) * nlb + mb0 + b) * 64 + lane] : 0.0;
  };
  auto group = [&](int g, const double (&av)[LB][U], double (&an)[LB][U]) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // group g's rows are in LDS; every wave is done with group g - 1's
    if (g + 1 < ng) issue(g + 1, an);
    const int64_t i = i0 + 16 * g;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = i + 4 * u + kq < i1;
      const double* rr = rs[g & 1] + (4 * u + kq) * TPC;
      double bv[NT], xv = 0.0;
#pragma unroll
      for (int nb = 0; nb < NT; ++nb) {
        const double t = rr[nb * 16 + m];
        bv[nb] = in ? t : 0.0;
      }
      if constexpr (XC != 0) {
        const double t = rr[16 * NT];
        xv = in ? t : 0.0;
      }
#pragma unroll
      for (int b = 0; b < LB; ++b)
        if (on[b]) {
#pragma unroll
          for (int nb = 0; nb < NT; ++nb)
            acc[b][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[b][u], bv[nb], acc[b][nb], 0, 0, 0);
          if constexpr (XC != 0) xacc[b] = fma(av[b][u], xv, xacc[b]);
        }
    }
  };
  double a0[LB][U], a1[LB][U];
  if (ng > 0) issue(0, a0);
  for (int g = 0; g < ng; g += 2) {
    group(g, a0, a1);
    if (g + 1 < ng) group(g + 1, a1, a0);
  }
#pragma unroll
  for (int b = 0; b < LB; ++b) {
    if (!on[b]) continue;
    double* out = part + ((int64_t)blockIdx.y * kpad + (mb0 + b) * 16) * tp;
#pragma unroll
    for (int nb = 0; nb < NT; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(int64_t)(kq + 4 * v) * tp + nb * 16 + m] = acc[b][nb][v];
    if constexpr (XC != 0) {
      // lane (m, kq) holds row l = m over the chunk rows i = kq (mod 4): add the
      // four lane groups in a fixed order ((0 + 1) + (2 + 3))
      double x = xacc[b];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      for (int cc = kq; cc < 16; cc += 4) out[(int64_t)m * tp + 16 * NT + cc] = cc == 0 ? x : 0.0;
    }
  }
}

// T[l][c] = sum over chunks of part, l < k: 64 entries per workgroup, its 16
// waves take chunks q = wave (mod 16), then a fixed-order sum over the waves
__global__ __launch_bounds__(1024) void k_ltr_sum(const double* __restrict__ part, int nchunk, int k, int kpad, int tp,
                                                  double* __restrict__ T, const int* __restrict__ nactive) {
  if (nactive != nullptr && *nactive == 0) return;
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const bool in = e < k * tp;
  const int l = in ? e / tp : 0, c = in ? e % tp : 0;
  double s = 0.0;
  if (in) {
#pragma unroll 4
    for (int q = wave; q < nchunk; q += 16) s += part[((int64_t)q * kpad + l) * tp + c];
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && in) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w][lane];
    T[e] = t;
  }
}

// Y = C^-1 T (k x k times k x tp), and zero rows k .. rup(k, 64) - 1 (k_zapply_mfma
// copies Y to LDS in whole chunks of up to 64 rows)
__global__ void k_cinv_apply(const double* __restrict__ Cinv, const double* __restrict__ T, int k, int tp,
                             double* __restrict__ Y, const int* __restrict__ nactive) {
  if (nactive != nullptr && *nactive == 0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (k + 63) / 64 * 64 * tp) return;
  const int l = e / tp, c = e % tp;
  if (l >= k) {
    Y[e] = 0.0;
    return;
  }
  double s = 0.0;
  // unrolled so that the loads of several terms are in flight together (same order)
#pragma unroll 8
  for (int m = 0; m < k; ++m) s += Cinv[l * k + m] * T[m * tp + c];
  Y[e] = s;
}

// rows of Y per LDS chunk in k_zapply_mfma: 64, 32 or 16 (a divisor of 64), so that a
// chunk of rows x tp doubles fits in 32 KB
__host__ __device__ constexpr int zy_rows(int tp) { return tp <= 64 ? 64 : (tp <= 128 ? 32 : 16); }
constexpr int kZyLdsDoubles = 4096;

// Z = (R - L Y) / sigma^2 on 64 rows per workgroup (16 per wave), plus the
// per-block partial r.z of every column.  XC = 1 as in k_ltr_mfma: column 16 NT of
// L Y on the vector ALU, and in the padding columns (where Y is zero) z = r / sigma^2.
// Y is copied once per workgroup into LDS, LC rows at a time, so the loop's only
// global loads are L's; each K-group's L loads are issued one group ahead and stay
// in flight across the LDS reads and MFMAs of the current group.
template <int NT, int XC>
__global__ __launch_bounds__(256) void k_zapply_mfma(const double* __restrict__ L, const double* __restrict__ Y,
                                                     const double* __restrict__ R, int64_t n, int k, int tp,
                                                     double inv_s2, double* __restrict__ Z, double* __restrict__ part,
                                                     const int* __restrict__ nactive) {
  if (nactive != nullptr && *nactive == 0) return;
  constexpr int RED = 16 * 16 * NT + (XC ? 4 * 16 * 16 : 0);
  // the Y chunks during the K-loop (rows of tp doubles, as in Y), the r.z partials after it
  __shared__ __attribute__((aligned(16))) double smem[kZyLdsDoubles > RED ? kZyLdsDoubles : RED];
  double* ys = smem;
  const int LC = zy_rows(tp);
  double(*red)[16 * NT] = reinterpret_cast<double(*)[16 * NT]>(smem);
  double(*redx)[16][16] = reinterpret_cast<double(*)[16][16]>(smem + 16 * 16 * NT);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t ra = r0 + m;
  f64x4 acc[NT];
#pragma unroll
  for (int nb = 0; nb < NT; ++nb) acc[nb] = f64x4{0.0, 0.0, 0.0, 0.0};
  double xacc = 0.0;
  constexpr int U = 4;
  // L[l0 + 4u + kq][ra] from a clamped address, then a select (a lane-dependent
  // condition on the load itself would become a branch around it)
  auto load_l = [&](int l0, double (&av)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = l0 + 4 * u + kq;
      const bool in = l < k && ra < n;
      const double t = L[in ? (int64_t)l * n + ra : 0];
      av[u] = in ? t : 0.0;
    }
  };
  // K-groups of 16 l; group g uses the L values in one register set while the next
  // group's land in the other (a ping-pong, so no register copy waits on a load)
  auto group = [&](int g, const double (&cur)[U], double (&nxt)[U]) {
    const int l0 = 16 * g;
    load_l(l0 + 16, nxt);  // past k the clamped loads give zeros
    if (l0 % LC == 0) {
      // rows l0 .. l0 + LC - 1 of Y (zero past k; Y holds rup(k, 64) rows) are one
      // contiguous run: copied global -> LDS in 1 KB units, no registers in between
      __syncthreads();  // every wave is done with the previous chunk
      const u32x4* src = reinterpret_cast<const u32x4*>(Y + (int64_t)l0 * tp);
      u32x4* dst = reinterpret_cast<u32x4*>(ys);
      const int units = LC * tp / 128;
      for (int un = __builtin_amdgcn_readfirstlane(wave); un < units; un += 4)
        __builtin_amdgcn_global_load_lds(src + un * 64 + lane, (__attribute__((address_space(3))) void*)(dst + un * 64),
                                         16, 0, 0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* yr = ys + (l0 % LC + 4 * u + kq) * tp;
#pragma unroll
      for (int nb = 0; nb < NT; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[u], yr[nb * 16 + m], acc[nb], 0, 0, 0);
      if constexpr (XC != 0) xacc = fma(cur[u], yr[16 * NT], xacc);
    }
  };
  const int ng = (k + 15) / 16;
  double a0[U], a1[U];
  if (ng > 0) load_l(0, a0);
  for (int g = 0; g < ng; g += 2) {
    group(g, a0, a1);
    if (g + 1 < ng) group(g + 1, a1, a0);
  }
  __syncthreads();  // the LDS now holds the r.z partials
  // lane holds rows r0 + kq + 4v, column nb * 16 + m
#pragma unroll
  for (int nb = 0; nb < NT; ++nb) {
    double rz = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + kq + 4 * v;
      if (r < n) {
        const int64_t e = r * tp + nb * 16 + m;
        const double rv = R[e];
        const double z = (rv - acc[nb][v]) * inv_s2;
        Z[e] = z;
        rz += rv * z;
      }
    }
    red[wave * 4 + kq][nb * 16 + m] = rz;
  }
  if constexpr (XC != 0) {
    // row ra: the four lane groups' partial sums in a fixed order, then lane (m, kq)
    // takes columns 16 NT + kq + 4 j of that row
    double x = xacc;
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = kq + 4 * j;
      double rz = 0.0;
      if (ra < n) {
        const int64_t e = ra * tp + 16 * NT + cc;
        const double rv = R[e];
        const double z = (cc == 0 ? rv - x : rv) * inv_s2;
        Z[e] = z;
        rz = rv * z;
      }
      redx[wave][m][cc] = rz;
    }
  }
  if (part == nullptr) return;
  __syncthreads();
  for (int c = threadIdx.x; c < 16 * NT; c += 256) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += red[q][c];
    part[(int64_t)blockIdx.x * tp + c] = s;
  }
  if constexpr (XC != 0) {
    if (threadIdx.x < 16) {
      double s = 0.0;
      for (int w = 0; w < 4; ++w)
        for (int q = 0; q < 16; ++q) s += redx[w][q][threadIdx.x];
      part[(int64_t)blockIdx.x * tp + 16 * NT + threadIdx.x] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static unsigned nb_for(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

template <int NT, int XC>
static void ltr_launch(const Ctx& c, const double* Rsrc, double* part, const int* nact) {
  const Layout& L = *c.lay;
  const int kpad = (L.k + 15) / 16 * 16;
  constexpr int wl = kLtrWaves * ltr_lblocks<NT>();  // l-blocks per workgroup
  hipLaunchKernelGGL((k_ltr_mfma<NT, XC>), dim3((kpad / 16 + wl - 1) / wl, L.nchunk_ltr), dim3(64 * kLtrWaves), 0, c.st,
                     c.at<double>(L.lf_ltr), Rsrc, L.n, kpad, L.tp, L.ltr_rows, part, nact);
}

template <int NT, int XC>
static void zapply_launch(const Ctx& c, const Hyper& h, const double* Rsrc, double* Zdst, double* rz_part,
                          const int* nact) {
  const Layout& L = *c.lay;
  hipLaunchKernelGGL((k_zapply_mfma<NT, XC>), dim3(nb_for(L.n, 64)), dim3(256), 0, c.st, c.at<double>(L.L),
                     c.at<double>(L.Y), Rsrc, L.n, L.k, L.tp, 1.0 / h.s2, Zdst, rz_part, nact);
}

#define GPMLL_TP_CASES(M) M(1) M(2) M(3) M(4) M(5) M(6) M(8) M(12) M(16)

// the Woodbury products take the extra-column route when the tp columns hold
// 16 m + 1 meaningful ones (y and 16 m probes, m = tp / 16 - 1 <= 5); returns m, else 0
static int woodbury_xc_tiles(const Layout& L) {
  const int m = L.tp / 16 - 1;
  return (m >= 1 && m <= 5 && L.t == 16 * m + 1) ? m : 0;
}

// dst (k x tp) = L^T Rsrc
hipError_t launch_ltr(const Ctx& c, const double* Rsrc, double* dst, const int* nact) {
  const Layout& L = *c.lay;
  const int kpad = (L.k + 15) / 16 * 16;
  double* part = c.at<double>(L.ltr_part2);
  switch (woodbury_xc_tiles(L)) {
#define CASE(N) case N: ltr_launch<N, 1>(c, Rsrc, part, nact); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5)
#undef CASE
    default:
      switch (L.tp / 16) {
#define CASE(N) case N: ltr_launch<N, 0>(c, Rsrc, part, nact); break;
        GPMLL_TP_CASES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
      }
  }
  hipLaunchKernelGGL(k_ltr_sum, dim3(nb_for((int64_t)L.k * L.tp, 64)), dim3(1024), 0, c.st, part, L.nchunk_ltr, L.k,
                     kpad, L.tp, dst, nact);
  return hipGetLastError();
}

hipError_t launch_woodbury(const Ctx& c, const Hyper& h, const double* Rsrc, double* Zdst, const int* nact,
                           double* rz_part) {
  const Layout& L = *c.lay;
  if (L.k > 0) {
    hipError_t e = launch_ltr(c, Rsrc, c.at<double>(L.ltr), nact);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cinv_apply, dim3(nb_for((int64_t)(L.k + 63) / 64 * 64 * L.tp, 256)), dim3(256), 0, c.st,
                       c.at<double>(L.Cinv), c.at<double>(L.ltr), L.k, L.tp, c.at<double>(L.Y), nact);
  }
  switch (woodbury_xc_tiles(L)) {
#define CASE(N) case N: zapply_launch<N, 1>(c, h, Rsrc, Zdst, rz_part, nact); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5)
#undef CASE
    default:
      switch (L.tp / 16) {
#define CASE(N) case N: zapply_launch<N, 0>(c, h, Rsrc, Zdst, rz_part, nact); break;
        GPMLL_TP_CASES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
      }
  }
  return hipGetLastError();
}

hipError_t launch_cg_init(const Ctx& c, const Hyper& h) {
  const Layout& L = *c.lay;
  const int64_t rpb = (L.n + L.nred - 1) / L.nred;
  double* part = c.at<double>(L.dot_part);
  double* part2 = part + (int64_t)L.nred * L.tp;
  hipLaunchKernelGGL(k_coldot_part, dim3(L.nred), dim3(256), 0, c.st, c.at<double>(L.R), c.at<double>(L.R), L.n, L.tp,
                     rpb, part);
  // Z0 = P^-1 B; the z-apply partials have one row per 64-row tile
  hipError_t e = launch_woodbury(c, h, c.at<double>(L.R), c.at<double>(L.Z0), nullptr, part2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, c.st, c.at<int>(L.nactive));
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, c.st, c.at<int>(L.nactive) + 1);
  // the z-apply partial count differs from nred: reduce them with their own count
  hipLaunchKernelGGL(k_cg_start, dim3(L.tp), dim3(256), 0, c.st, part, L.nred, part2, (int)nb_for(L.n, 64), L.tp, L.t,
                     c.at<double>(L.bnorm), c.at<double>(L.rho), c.at<double>(L.rho0), c.at<int>(L.active),
                     c.at<int>(L.iters), c.at<int>(L.nactive));
  const int64_t cnt = L.n_pad * L.tp;
  hipLaunchKernelGGL(k_copy, dim3(nb_for(cnt, 256)), dim3(256), 0, c.st, c.at<double>(L.Z0), c.at<double>(L.Pd), cnt);
  return hipGetLastError();
}

// one CG iteration after the K_hat product has been reduced into W with p.w partials
hipError_t launch_cg_after_product(const Ctx& c, const Hyper& h, int it, double tol) {
  const Layout& L = *c.lay;
  const int64_t rpb = (L.n + L.nred - 1) / L.nred;
  double* part = c.at<double>(L.dot_part);
  int* nact = c.at<int>(L.nactive);
  int* nact_next = nact + 1;
  double* sc = c.at<double>(L.pw);  // alpha[tp] then beta[tp]
  double* alpha = sc;
  double* beta = sc + L.tp;
  const int nzblk = (int)nb_for(L.n, 64);
  hipLaunchKernelGGL(k_cg_alpha, dim3(L.tp), dim3(256), 0, c.st, part, (int)nb_for(L.n, 64), L.tp, it, L.max_iters,
                     c.at<double>(L.rho), c.at<int>(L.active), alpha, c.at<double>(L.alog), c.at<int>(L.flags) + 1,
                     nact);
  hipLaunchKernelGGL(k_cg_update, dim3(L.nred), dim3(256), 0, c.st, c.at<double>(L.Xs), c.at<double>(L.R),
                     c.at<double>(L.Pd), c.at<double>(L.W), alpha, c.at<int>(L.active), L.n, L.tp, rpb, part, nact);
  hipLaunchKernelGGL(k_cg_check, dim3(L.tp), dim3(256), 0, c.st, part, L.nred, L.tp, it, tol, c.at<double>(L.bnorm),
                     c.at<int>(L.active), c.at<int>(L.iters), c.at<double>(L.rnorm2), nact_next, nact);
  double* rzpart = part + (int64_t)L.nred * L.tp;
  hipError_t e = launch_woodbury(c, h, c.at<double>(L.R), c.at<double>(L.W), nact, rzpart);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cg_beta, dim3(L.tp), dim3(256), 0, c.st, rzpart, nzblk, L.tp, it, L.max_iters,
                     c.at<double>(L.rho), c.at<int>(L.active), beta, c.at<double>(L.blog), nact);
  hipLaunchKernelGGL(k_cg_p, dim3(L.nred), dim3(256), 0, c.st, c.at<double>(L.Pd), c.at<double>(L.W), beta,
                     c.at<int>(L.active), L.n, L.tp, rpb, nact);
  hipLaunchKernelGGL(k_swap_count, dim3(1), dim3(1), 0, c.st, nact, nact_next);
  return hipGetLastError();
}

hipError_t launch_colmap(const Ctx& c) {
  const Layout& L = *c.lay;
  hipLaunchKernelGGL(k_colmap, dim3(1), dim3(64), 0, c.st, c.at<int>(L.active), L.tp, c.at<int>(L.colmap));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Posterior prediction (Sec. 2.1): one CG call on [y | k(X, x*_1) .. k(X, x*_m)]
// gives u = K_hat^-1 y and a_j = K_hat^-1 k(X, x*_j); the mean is a_j^T y and the
// latent variance s - k(X, x*_j)^T a_j.
// ---------------------------------------------------------------------------

// R = [y | s kappa(x~_i, x~*_j) for the chunk's test points | 0], the cross
// covariances also into Bk (kept through CG), Xs = 0; padding rows zero
__global__ void k_pred_rhs(const double* __restrict__ y, const double* __restrict__ xs,
                           const double* __restrict__ xstar, const double* __restrict__ mean, int64_t n,
                           int64_t n_pad, int tp, int ncols, Hyper h, double* __restrict__ R, double* __restrict__ Bk,
                           double* __restrict__ Xs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  double* row = R + i * tp;
  double* brow = Bk + i * tp;
  double* xrow = Xs + i * tp;
  for (int c = 0; c < tp; ++c) {
    row[c] = 0.0;
    brow[c] = 0.0;
    xrow[c] = 0.0;
  }
  if (i >= n) return;
  const int d = h.d;
  double xi[GP_MAX_D];
  for (int q = 0; q < d; ++q) xi[q] = xs[i * d + q];
  row[0] = y[i];
  brow[0] = y[i];
  for (int j = 0; j < ncols; ++j) {
    double r2 = 0.0;
    for (int q = 0; q < d; ++q) {
      const double df = xi[q] - (xstar[(int64_t)j * d + q] - mean[q]) * h.inv_ls[q];
      r2 = fma(df, df, r2);
    }
    const double kv = h.s * kappa64(h.kind, r2, h.alpha);
    row[1 + j] = kv;
    brow[1 + j] = kv;
  }
}

// dst[i][c] = src[i][0] for every column c
__global__ void k_bcast_col0(const double* __restrict__ src, double* __restrict__ dst, int64_t n, int tp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * tp) return;
  dst[e] = src[(e / tp) * tp];
}

// mean_j = sum_i Xs[i][1+j] y_i and var_j = s - sum_i Bk[i][1+j] Xs[i][1+j] from the
// per-block partials; one workgroup per test point
__global__ void k_pred_final(const double* __restrict__ part_mean, const double* __restrict__ part_var, int nblk,
                             int tp, double s, double* __restrict__ mean, double* __restrict__ var) {
  const int j = blockIdx.x;
  const double m = column_total(part_mean, nblk, tp, 1 + j);
  const double v = column_total(part_var, nblk, tp, 1 + j);
  if (threadIdx.x == 0) {
    mean[j] = m;
    if (var) var[j] = s - v;
  }
}

hipError_t launch_pred_rhs(const Ctx& c, const Hyper& h, const double* y, const double* xstar, int ncols) {
  const Layout& L = *c.lay;
  hipLaunchKernelGGL(k_pred_rhs, dim3(nb_for(L.n_pad, 256)), dim3(256), 0, c.st, y, c.at<double>(L.xs), xstar,
                     c.at<double>(L.mean), L.n, L.n_pad, L.tp, ncols, h, c.at<double>(L.R), c.at<double>(L.cprime),
                     c.at<double>(L.Xs));
  return hipGetLastError();
}

hipError_t launch_coldot(const Ctx& c, const double* A, const double* B, double* part);

hipError_t launch_pred_finish(const Ctx& c, const Hyper& h, int ncols, double* mean, double* var) {
  const Layout& L = *c.lay;
  double* part_mean = c.at<double>(L.dot_part);
  double* part_var = part_mean + (int64_t)L.nred * L.tp;
  // y in every column of W (free after CG), then column dots with the solutions
  hipLaunchKernelGGL(k_bcast_col0, dim3(nb_for(L.n * L.tp, 256)), dim3(256), 0, c.st, c.at<double>(L.cprime),
                     c.at<double>(L.W), L.n, L.tp);
  hipError_t e = launch_coldot(c, c.at<double>(L.Xs), c.at<double>(L.W), part_mean);
  if (e != hipSuccess) return e;
  e = launch_coldot(c, c.at<double>(L.cprime), c.at<double>(L.Xs), part_var);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pred_final, dim3(ncols), dim3(256), 0, c.st, part_mean, part_var, L.nred, L.tp, h.s, mean,
                     var);
  return hipGetLastError();
}

hipError_t launch_coldot(const Ctx& c, const double* A, const double* B, double* part) {
  const Layout& L = *c.lay;
  const int64_t rpb = (L.n + L.nred - 1) / L.nred;
  hipLaunchKernelGGL(k_coldot_part, dim3(L.nred), dim3(256), 0, c.st, A, B, L.n, L.tp, rpb, part);
  return hipGetLastError();
}

}  // namespace gpmll
