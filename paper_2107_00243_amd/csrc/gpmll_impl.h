// Internal declarations of the gpmll HIP library (gfx950).
//
// Data layout in device memory (all inside the caller's workspace):
//   xs      n_pad x d         FP64  centred, lengthscale-scaled inputs x~ = (x - mean) / ls
//   xfrag   tile-precision copy of x~ arranged for the MFMA operand loads
//   rowterm / colterm         per-point FP32 terms of the distance expansion
//   L       n x rank          FP64  pivoted Cholesky factor, column-major
//   CG block arrays           n_pad x tp FP64, row-major (tp = columns padded to 16)
//   vfrag   tile-precision copy of the search directions for the MFMA B operand
//   wpart   split-K partial products, FP32 (FP64 for FP64 tiles)
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/gpmll.h"

namespace gpmll {

constexpr int kRowBlock = 256;      // rows per workgroup of the tile kernels; n is padded to this
constexpr int kSlqQrMax = 128;      // longest Lanczos tridiagonal diagonalised by QR; longer: quadrature
constexpr int kWgSlots = 512;       // resident tile workgroups on MI355X: 2 per CU x 256 CUs
constexpr int kColChunk = 32;       // K-dimension of one tile-times-V step (MFMA K for BF16)
constexpr int kRedBlock = 256;      // threads of the reduction kernels
constexpr int kChunkRows = 2048;    // rows per partial of the Gram reduction L^T L

// Row groups of 16 rows per wave of the FP32 / FP64 tile kernels for NTT
// 16-column tiles of right-hand sides; a workgroup covers 64 * RG rows.
constexpr __host__ __device__ int fp_row_groups(size_t elem_bytes, int ntt) {
  return elem_bytes == 8 ? (ntt <= 4 ? 2 : 1) : (ntt <= 5 ? 4 : (ntt <= 8 ? 2 : 1));
}

// Hyperparameters as the kernels consume them.
struct Hyper {
  int kind;      // gp_kernel
  int d;
  double inv_ls[GP_MAX_D];
  double s;      // outputscale
  double s2;     // noise variance
  double log2s;  // log2(s)
  double alpha;  // rational quadratic shape (1 for the other kernels)
};

// Kernel correlation kappa(r^2) and the derivative factor g(r^2) with
// d kappa / d ls_j = g * dtilde_j^2 / ls_j (FP64, used by the FP64 tiles, the
// pivoted Cholesky and the preconditioner derivative).
__device__ inline void kappa_g64(int kind, double r2, double* kap, double* g, double alpha) {
  const double sqrt3 = 1.7320508075688772, sqrt5 = 2.23606797749979;
  if (kind == GP_KERNEL_RBF) {
    double e = exp(-0.5 * r2);
    *kap = e;
    *g = e;
  } else if (kind == GP_KERNEL_RATQUAD) {
    // kappa = b^-alpha with b = 1 + r^2 / (2 alpha); -2 d kappa / d r^2 = b^(-alpha-1)
    const double b = 1.0 + r2 / (2.0 * alpha);
    const double k = exp(-alpha * log(b));
    *kap = k;
    *g = k / b;
  } else if (kind == GP_KERNEL_MATERN32) {
    double r = sqrt(r2);
    double e = exp(-sqrt3 * r);
    *kap = (1.0 + sqrt3 * r) * e;
    *g = 3.0 * e;
  } else {
    double r = sqrt(r2);
    double e = exp(-sqrt5 * r);
    *kap = (1.0 + sqrt5 * r + (5.0 / 3.0) * r2) * e;
    *g = (5.0 / 3.0) * (1.0 + sqrt5 * r) * e;
  }
}

__device__ inline double kappa64(int kind, double r2, double alpha) {
  double k, g;
  kappa_g64(kind, r2, &k, &g, alpha);
  return k;
}

// Workspace carving.  Offsets are bytes from the workspace base, 256-aligned.
// Pieces of each search-direction value in the BF16x3 tiles: hi + lo (16 bits),
// or hi + lo + lo2 (24 bits, one more MFMA per tile and step).  Two-piece
// directions delay CG (their rounding acts like noise on the product and spoils
// the early Krylov steps: 43 iterations instead of the 33 of FP64 tiles on the
// n = 100,000 RBF workload), three-piece ones in the first kBf16V3Iters iterations
// of a call restore the FP64 iteration count (measured: 8 are not enough there, 12
// are; 16 leave a margin); later iterations take two.  Launches of more than eight
// tiles always take two (three would overflow the LDS stages).
#ifndef GPMLL_BF16_V3_ITERS
#define GPMLL_BF16_V3_ITERS 16
#endif
constexpr int kBf16V3Iters = GPMLL_BF16_V3_ITERS;
__device__ __host__ constexpr bool bf16_v3_fits(int ntt) { return ntt <= 8; }

struct Layout {
  int64_t n, n_pad;
  int d, p, t, tp, k, ell, max_iters, prec;
  int bprec;            // precision of the derivative sweep operands (FP64 or FP32)
  int kd;               // K-extent of the staged distance operand (elements)
  int bkd;              // K-extent of the derivative sweep's distance operand
  int bow;              // row width of the derivative sweep's per-row outputs
  int nsplit;           // column splits of the tile kernels
  int64_t cols_per_split;
  int nchunk;           // row chunks of the Gram reduction
  int nchunk_ltr;       // row chunks of the L^T R reduction
  int64_t ltr_rows;     // rows per chunk of the L^T R reduction (multiple of 16)
  int nrb;              // row blocks of kRowBlock rows
  int nred;             // blocks of the row-parallel reductions (<= 1024)
  // preconditioner block (offsets independent of the estimator options)
  size_t xs, mean, mean_part, L, diag, ispiv, piv, amax, C, Rc, Rinv, Cinv, logdetP, scal_small, flags, ltr_part;
  size_t freq;          // m x d spectral samples of the random Fourier feature preconditioner
  size_t landmarks;     // k prescribed pivot rows of the Nystrom preconditioner
  size_t famp;          // m per-frequency amplitudes of weighted Fourier features
  // L in the operand order of the L^T R MFMAs (each wave load one contiguous 512-byte
  // run): lf_ltr[(i/4, l/16)][lane (i%4, l%16)], rup(n, 64) x rup(k, 16) entries,
  // zero past n and k; written with the preconditioner
  size_t lf_ltr;
  size_t precond_end;
  // estimator block
  size_t xfa, xfb, rowterm, colterm, H, Y, ltr, ltr_raw, ltr_part2;
  size_t Xs, R, Z0, Pd, W, vfrag, vx, vscale, wpart;
  size_t rho, rho0, bnorm, rnorm2, pw, active, nactive, iters, colmap, alog, blog;
  size_t dot_part, gamma, slq_work;
  size_t cprime, bxa, bxb, brt, bct, bafrag, bcfrag, bxaug, bwd_part, pg_small, omega, pg_part;
  size_t sqrt_work;     // 6 k x k FP64 of the square-root probes (probe_mode 1 only)
  size_t total;
};

Layout make_layout(int64_t n, int d, int ard, int num_probes, int max_iters, int rank, int prec,
                   int probe_mode = 0);

// 32-wide K chunks of the BF16x3 M-tile contraction over t columns split as
// (hi, hi, lo) x (hi, lo, hi), rounded up to a compiled chunk count
inline int bwd_nkm(int t) {
  const int tq = (t + 7) / 8 * 8;
  const int nkm = (3 * tq + 31) / 32;
  static const int ok[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 14, 16, 18, 20, 22, 24};
  for (int v : ok)
    if (v >= nkm) return v;
  return 24;
}

struct Ctx {
  const Layout* lay;
  char* ws;
  hipStream_t st;
  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// Small integer slots: scal_small[0] pivoted-Cholesky stop flag, [1] achieved rank.
// flags[0] GP_FLAG_* bits, [1] deferred gp_status, [2] clamped Ritz values.

hipError_t launch_prep(const Ctx& c, const double* X, const Hyper& h);
// greedy pivots, or (forced != null) the k prescribed distinct rows in that order
hipError_t launch_pivchol(const Ctx& c, const Hyper& h, const int32_t* forced = nullptr);
hipError_t launch_precond_finish(const Ctx& c, const Hyper& h);
// Fourier features from the frequencies at lay.freq into the L slot (rank 2m), with
// amplitude sqrt(s/m) (random features) or the amplitudes at lay.famp (weighted)
hipError_t launch_rff(const Ctx& c, const Hyper& h, bool weighted = false);

// preconditioner families: the low-rank factor in the L slot comes from
enum PrecondKind { kPivChol = 0, kRff = 1 };
hipError_t launch_probes(const Ctx& c, const double* y, const Hyper& h, uint64_t seed);
// probes b_i = P_hat^1/2 w_i (symmetric square root; C^1/2 by a coupled Newton-Schulz
// iteration on the k x k matrix C, then (C^1/2 + sigma I)^-1 by Cholesky)
hipError_t launch_probes_sqrt(const Ctx& c, const double* y, const Hyper& h, uint64_t seed);
hipError_t launch_cg_init(const Ctx& c, const Hyper& h);

// posterior prediction: right-hand sides [y | k(X, x*_j), j < ncols] (and their copy
// kept through CG), then mean_j and latent var_j from the solutions
hipError_t launch_pred_rhs(const Ctx& c, const Hyper& h, const double* y, const double* xstar, int ncols);
hipError_t launch_pred_finish(const Ctx& c, const Hyper& h, int ncols, double* mean, double* var);

// forgets the forward pass recorded for a workspace (every call that writes into a
// workspace other than the estimator itself calls this first)
void gpmll_forget_forward(const void* ws);

// GP_OK when the current device is gfx950 (cached per device); records the HIP
// error behind a GP_EHIP for gp_last_hip_error.
int gpmll_check_device();
void gpmll_set_hip_error(int e);

// Staging and tile launches shared with the batched path (the layout view there
// describes the concatenation of all problems' padded row blocks).
hipError_t launch_stage_x(const Ctx& c, const Hyper& h);
// Staged right-hand side columns of one product: ntt 16-column tiles on the
// matrix cores (-1: all of tp) and, for the split precisions, xc = 1 more column
// (staged column 16 ntt) contracted on the vector ALU.
struct TilePlan {
  int ntt = -1;
  int xc = 0;
  int vp = 2;  // BF16x3: pieces of each staged search-direction value (2 or 3)
};
// the plan for ncols staged columns (compiled tile counts only)
TilePlan tile_plan(const Layout& L, int ncols);
// V staging: ncols staged columns taken through colmap (null: the first ncols
// columns), laid out as the plan's tiles (and extra column).
hipError_t launch_stage_v(const Ctx& c, const double* V, int ldv, int ncols, const Hyper& h,
                          const int* colmap = nullptr, TilePlan plan = TilePlan{});
// Tile launch over the plan's staged columns.
hipError_t launch_khat_tiles(const Ctx& c, const Hyper& h, const int* nact, TilePlan plan = TilePlan{});
// W (columns through colmap, as staged) = s * sum of split partials + sigma^2 V,
// and per-64-row-block partials of V.W at dot_part[block * ldpart + column].
hipError_t launch_khat_reduce(const Ctx& c, const double* V, int ldv, double* W, int ldw, int ncols, const Hyper& h,
                              double* dot_part, const int* nact, const int* colmap = nullptr, int ldpart = 0);
// colmap[0 .. tp) = the active columns in increasing order, then -1 (from the CG masks)
hipError_t launch_colmap(const Ctx& c);

// FP32 / FP64 tiles over a table of int4 {first row, column begin, column end,
// output slot}; kernel values carry outputscale 1 (the caller scales).  With a
// gate, item i is skipped while gate_count[gate[i]] == 0.
struct ItemTable {
  const int4* items = nullptr;
  int nitems = 0;
  const int* gate = nullptr;
  const int* gate_count = nullptr;
};
hipError_t launch_khat_tiles_items(const Ctx& c, const Hyper& h, const ItemTable& it, const int* nact);

}  // namespace gpmll
