// Internal declarations of the batched path: many independent problems of
// different sizes evaluated by one call, each phase one launch for all problems.
//
// Layout: every problem's rows are padded to a multiple of kBRows and the
// padded blocks are concatenated (N rows in total).  Per-row arrays (scaled
// inputs, CG blocks, staged tile operands) use the concatenated row index;
// every kBRows-row block belongs to exactly one problem (blkprob).  Per-problem
// scalars are [B][tp] (CG) or [B][K][K] (small dense).  The pivoted Cholesky
// factor of problem b is column-major n_pad_b x K at element offset loff_b.
#pragma once

#include "gpmll_impl.h"

namespace gpmll {

constexpr int kBRows = 256;         // rows per block of the batched layout
constexpr int kBMaxRank = 256;      // largest preconditioner rank of the batched path
constexpr int kBMaxProbes = 64;     // largest probe count of the batched path (tp <= 80)
constexpr int64_t kBColsPerSplit = 1024;  // columns per work item of the K_hat V tiles
constexpr int64_t kBBwdCols = 2048;       // columns per work item of the derivative sweep

struct BDesc {
  int64_t xoff;     // first row of the problem in the caller's unpadded X and y
  int64_t off;      // first row in the padded concatenation
  int64_t n;        // points
  int64_t n_pad;    // rows reserved, multiple of kBRows
  int64_t loff;     // element offset of the problem's L (column-major n_pad x K)
  int32_t blk0;     // first kBRows-row block
  int32_t nblk;     // its blocks
  int32_t nsplit;   // column splits of its tile product (output slots 0 .. nsplit-1)
  int32_t k;        // preconditioner rank requested for it: min(rank, n)
  int32_t bitem0;   // first work item of the derivative sweep
  int32_t nbitem;   // its work items
  double s, s2, sigma;
  uint64_t seed;
  double inv_ls[GP_MAX_D];
};

struct BLayout {
  int B, d, p, t, tp, K, ell, max_iters, prec, kind, ard;
  int64_t N;            // rows of the padded concatenation
  int nblk;             // N / kBRows
  int maxsplit, nitems, nbitems;
  int dm;               // compiled dimension bound of the derivative sweep (4, 8, 16, 32)
  Layout view;          // tile-kernel view of the concatenation (n = n_pad = N)
  size_t desc, items, item_prob, bitems, blkprob;
  size_t xs, L, diag, ispiv, piv, kach, stop, C, Rc, Rinv, Cinv, logdetP, H;
  size_t Tb, Y, ltr_part;
  size_t R, Xs, Z0, Pd, W;
  size_t rho, rho0, bnorm, rnorm, alpha, beta, active, iters, nactive, pact, alog, blog;
  size_t part, part2, gamma, flags, logp_aux;
  size_t cprime, bwd_part, pgs, pg_psi, pg_part;
  size_t total;
};

// flags[b * 4 + 0] GP_FLAG_* bits, [1] deferred gp_status, [2] clamped Ritz values

hipError_t bl_prep(const BLayout& L, char* ws, hipStream_t st, const double* X);
hipError_t bl_precond(const BLayout& L, char* ws, hipStream_t st);
hipError_t bl_probes(const BLayout& L, char* ws, hipStream_t st, const double* y);
hipError_t bl_cg_init(const BLayout& L, char* ws, hipStream_t st);
hipError_t bl_cg_after_product(const BLayout& L, char* ws, hipStream_t st, int it, double tol);
hipError_t bl_reduce(const BLayout& L, char* ws, hipStream_t st);
hipError_t bl_slq_logp(const BLayout& L, char* ws, hipStream_t st, const double* y, double* logp);
hipError_t bl_backward(const BLayout& L, char* ws, hipStream_t st, int precond_grad, double* grad);
hipError_t bl_zero_flags(const BLayout& L, char* ws, hipStream_t st);

}  // namespace gpmll
