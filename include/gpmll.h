/*
 * gpmll — preconditioned Gaussian-process log marginal likelihood and its
 * gradient on AMD Instinct MI355X (gfx950).
 *
 * Method: Wenger, Pleiss, Hennig, Cunningham, Gardner, "Preconditioning for
 * Scalable Gaussian Process Hyperparameter Optimization" (ICML 2022),
 * Algorithm 1 (log-marginal likelihood) and Algorithm 2 (its derivative),
 * Section 4.4, with the partial pivoted Cholesky preconditioner (Section 2.2,
 * "Preconditioning"; supplement S5.3) and the log-determinant decomposition of
 * Section 3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named *_dev are device pointers (hipMalloc / torch CUDA tensors);
 *   pointers named *_host are host pointers.  The library never allocates
 *   device memory: every device array it needs lives in the caller's workspace
 *   (see gp_workspace_size).  It owns no device memory between calls.
 * - X_dev is n x d, row-major, FP64.  y_dev is n FP64.
 * - theta_host holds natural (positive) hyperparameters in the order
 *   [ls_1 .. ls_p | s | sigma^2], p = d for ARD kernels and p = 1 otherwise:
 *   k(x, x') = s * kappa(r), r^2 = sum_j ((x_j - x'_j) / ls_j)^2, and
 *   K_hat = K + sigma^2 I (Section 2.1).
 * - All work is enqueued on `stream`, in order.  Results written to *_dev
 *   outputs are valid once the stream reaches them.  A call returns after
 *   enqueueing unless it has to read a device value on the host: the
 *   convergence poll of CG (gp_options.sync_every > 0) and the optional
 *   statistics (stats != NULL) do that.
 * - Calls that share a workspace must not overlap; calls on distinct
 *   workspaces may run concurrently on distinct streams.
 * - Every function returns GP_OK (0) or a negative gp_status; gp_strerror
 *   gives the text.  On an error nothing further is enqueued; work enqueued
 *   before the error was detected may still run.
 * - Results are deterministic: fixed inputs, seed and build on the same GPU give
 *   bitwise-identical outputs (fixed-order reductions, no float atomics).
 */
#ifndef GPMLL_H
#define GPMLL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gp_status {
  GP_OK = 0,
  GP_EINVAL = -1,        /* null pointer, n < 1, d out of range, theta <= 0 or NaN, sizes */
  GP_EWORKSPACE = -2,    /* workspace smaller than gp_workspace_size */
  GP_ENOTSPD = -3,       /* p^T K_hat p <= 0 in CG, or the k x k Woodbury matrix not SPD */
  GP_EHIP = -4,          /* a HIP runtime call failed; see gp_last_hip_error */
  GP_EUNSUPPORTED = -5   /* device is not gfx950, or an option the build lacks */
} gp_status;

typedef enum gp_kernel {
  GP_KERNEL_RBF = 0,        /* kappa = exp(-r^2 / 2) */
  GP_KERNEL_MATERN32 = 1,   /* kappa = (1 + sqrt3 r) exp(-sqrt3 r) */
  GP_KERNEL_MATERN52 = 2,   /* kappa = (1 + sqrt5 r + 5 r^2 / 3) exp(-sqrt5 r) */
  GP_KERNEL_RATQUAD = 3     /* kappa = (1 + r^2 / (2 alpha))^-alpha, alpha = gp_problem.kernel_shape
                               (a fixed constant of the kernel, not part of theta) */
} gp_kernel;

typedef enum gp_precision {
  GP_PREC_FP64 = 0,         /* kernel tiles and products in FP64 */
  GP_PREC_FP32 = 1,         /* kernel tiles in FP32, FP32 MFMA products */
  GP_PREC_BF16X3 = 2,       /* split BF16 (hi + lo) MFMA products, FP32 accumulation */
  GP_PREC_FP16X3 = 3        /* distance as BF16X3; tile x V in split FP16 (hi + lo), with the kernel
                               values scaled by 2^15 and each column of V by a power of two so that
                               both fit the FP16 range (exact scalings, undone in FP64) */
} gp_precision;

/* Flags reported in gp_stats.flags. */
#define GP_FLAG_NOT_CONVERGED 1   /* a CG column hit max_iters before its tolerance */
#define GP_FLAG_RANK_DEFICIENT 2  /* pivoted Cholesky stopped early (rank_achieved < rank) */
#define GP_FLAG_RITZ_CLAMPED 4    /* a Ritz value was clamped to 1e-300 before the log */

/* Limits of this build. */
#define GP_MAX_D 32
#define GP_MAX_PROBES 255
#define GP_MAX_RANK 1024

/* The regression problem.  All device arrays stay owned by the caller. */
typedef struct gp_problem {
  const double* X_dev;   /* n x d row-major FP64 */
  const double* y_dev;   /* n FP64 */
  int64_t n;             /* number of points, >= 1 */
  int32_t d;             /* input dimension, 1 .. GP_MAX_D */
  int32_t kernel;        /* gp_kernel */
  int32_t ard;           /* 1: d lengthscales; 0: one shared lengthscale */
  double kernel_shape;   /* GP_KERNEL_RATQUAD: alpha > 0; ignored by the other kernels */
} gp_problem;

/* Estimator options (Algorithms 1 and 2). */
typedef struct gp_options {
  int32_t precision;     /* gp_precision of the K_hat tiles (0..3); recurrences are FP64 */
  int32_t num_probes;    /* ell, 1 .. GP_MAX_PROBES */
  int32_t max_iters;     /* CG iteration cap per column, >= 1 */
  double cg_tol;         /* a column stops when ||r|| <= cg_tol * ||b|| (>= 0) */
  uint64_t seed;         /* probe seed (SplitMix64 counter stream) */
  int32_t precond_grad;  /* 0: full frozen-pivot dP/dtheta; 1: only the s and sigma^2 terms */
  int32_t sync_every;    /* poll the convergence flag on the host every q iterations (q >= 1),
                            or 0 to enqueue all max_iters iterations without a host wait
                            (iterations after convergence exit at once on the device) */
  int32_t probe_mode;    /* 0: b_i = sigma eps_i + L eta_i; 1: b_i = P_hat^1/2 w_i with the symmetric
                            square root (rho0_i = n); both have E[b b^T] = P_hat.  Single
                            problems only (batches: GP_EUNSUPPORTED) */
} gp_options;

/* Statistics copied to the host when a stats pointer is given (this waits for
 * the stream).  The optional arrays are filled when non-NULL. */
typedef struct gp_stats {
  int32_t num_columns;       /* t = 1 + num_probes */
  int32_t iters_max;         /* max CG iterations over columns */
  int32_t rank_achieved;     /* k' <= rank */
  int32_t flags;             /* GP_FLAG_* */
  int32_t ritz_clamped;      /* number of clamped Ritz values */
  int32_t reserved;
  double logdet_precond;     /* log det P_hat */
  double datafit;            /* y^T u, u ~ K_hat^-1 y */
  double logdet_estimate;    /* log det P_hat + mean_i gamma_i */
  int32_t* col_iters_host;   /* [t] iterations per column, or NULL */
  double* gammas_host;       /* [num_probes] per-probe quadrature gamma_i, or NULL */
  double* rel_residual_host; /* [t] final recurrence ||r|| / ||b|| per column, or NULL */
  int32_t* pivots_host;      /* [rank] pivot rows, -1 after an early stop, or NULL */
} gp_stats;

/* Host handle of a preconditioner whose device arrays live in a workspace. */
typedef struct gp_precond gp_precond;

/* Device views of a built preconditioner (valid while its workspace lives). */
typedef struct gp_precond_view {
  const double* L_dev;        /* n x rank, column-major (column j contiguous) */
  const int32_t* pivots_dev;  /* [rank], -1 after an early stop */
  const double* logdet_dev;   /* log det(sigma^2 I + L L^T), one FP64 */
  int64_t n;
  int32_t rank;
} gp_precond_view;

/*
 * gp_workspace_size — device bytes the caller must provide to the calls below
 * for this problem shape, options and preconditioner rank (0 <= rank <=
 * min(n, GP_MAX_RANK)).  The size is also valid for gp_khat_matvec with
 * num_rhs <= 1 + num_probes.  Returns GP_EINVAL on bad shapes.
 */
int gp_workspace_size(const gp_problem* prob, const gp_options* opt, int32_t rank,
                      size_t* bytes);

/*
 * gp_precond_build — partial pivoted Cholesky preconditioner
 * P_hat = sigma^2 I + L L^T (Section 2.2, "Preconditioning"; supplement S5.3):
 * `rank` greedy steps on the residual diagonal of K (noise excluded), ties to
 * the lowest index, stopping early only when the largest residual diagonal is
 * <= 1e-12 * s; then C = sigma^2 I_k + L^T L, its Cholesky factor and
 * log det P_hat = (n - k) log sigma^2 + log det C (matrix determinant lemma).
 * Everything is FP64.  The device arrays are written into `ws`; *out receives
 * a small host handle (free it with gp_precond_free).  A later gp_mll_* call
 * given this handle must pass the same problem, theta and workspace.
 */
int gp_precond_build(const gp_problem* prob, const double* theta_host, int32_t rank,
                     void* ws_dev, size_t ws_bytes, hipStream_t stream, gp_precond** out);

/*
 * gp_precond_build_nystrom — randomized Nystrom preconditioner
 * P_hat = sigma^2 I + K_{:S} K_SS^-1 K_{S:} (Table 1, "randomized Nystrom";
 * supplement S5, randomized Nystrom approximation quality) on `rank` landmark
 * rows S given by the caller (drawn with probabilities proportional to K_ii^2,
 * which is uniform for these stationary kernels).  With as many landmarks as
 * the rank, no truncation of K_SS^+ is needed and the factor is the partial
 * Cholesky of gp_precond_build with its pivots prescribed in the order of S:
 * same handle, view (the pivots read S), breakdown rule (a landmark whose
 * residual diagonal is <= 1e-12 * s stops the factor, GP_FLAG_RANK_DEFICIENT)
 * and derivative (landmarks held fixed; precond_grad as for the pivoted
 * Cholesky).  landmarks_host: host int32[rank], distinct rows in [0, n); it is
 * copied before the call returns (the call waits for that copy).
 * Errors: GP_EINVAL for rank < 1, a null, repeated or out-of-range landmark, or
 * as gp_precond_build; GP_EWORKSPACE; GP_EHIP.
 */
int gp_precond_build_nystrom(const gp_problem* prob, const double* theta_host, int32_t rank,
                             const int32_t* landmarks_host, void* ws_dev, size_t ws_bytes,
                             hipStream_t stream, gp_precond** out);

/*
 * gp_precond_build_rff — random Fourier feature preconditioner
 * P_hat = sigma^2 I + Z Z^T (Table 1, "RFF"; supplement S5, RFF approximation
 * quality), an alternative to gp_precond_build with the same handle, workspace
 * layout and later use:
 *   Z = sqrt(s / m) [cos(Phi) | sin(Phi)]   (n x rank, rank = 2m, column-major),
 *   Phi = X~ W^T,  X~ = (X - column mean) / ls,
 * so that Z Z^T = (s/m) sum_j cos(w_j . (x~_a - x~_b)), whose expectation over w_j
 * drawn from the kernel's spectral density is K.  Then C, its factors and
 * log det P_hat as in gp_precond_build.  freq_dev is a device array of m x d
 * FP64 (row-major, row j = w_j): samples of the kernel's spectral density at
 * unit lengthscale (RBF: standard normal; Matern-nu: multivariate Student t
 * with 2 nu degrees of freedom).  They are copied into the workspace in stream
 * order, so freq_dev may be released once the stream has passed this call.
 * gp_mll_grad with this handle differentiates P_hat with the frequencies held
 * fixed (precond_grad = 1 keeps only the s and sigma^2 terms, as for the
 * pivoted Cholesky).  The pivots of the view read -1.
 * Errors: GP_EINVAL for an odd rank, rank < 2, a null freq_dev, or as
 * gp_precond_build; GP_EWORKSPACE; GP_EHIP.
 */
int gp_precond_build_rff(const gp_problem* prob, const double* theta_host, int32_t rank,
                         const double* freq_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream,
                         gp_precond** out);

/*
 * gp_precond_build_qff — quadrature Fourier feature preconditioner of the RBF
 * kernel (Table 1, "QFF"; Mutny & Krause 2018): the form of
 * gp_precond_build_rff with deterministic frequencies and weights, the tensor
 * Gauss rule of the standard normal spectral density with q = nodes_per_dim
 * points per dimension (probabilists' Hermite nodes, weights summing to 1).
 * Of each +-pair of grid nodes one is kept, with its weight doubled, so the
 * rank is q^d: Z = sqrt(s) [sqrt(w_j) cos(Phi_j) | sqrt(w_j) sin(Phi_j)] and
 * Z Z^T -> K exponentially fast in q.  The workspace and later gp_mll_* calls
 * use rank = q^d.  Derivatives hold nodes and weights fixed.
 * Errors: GP_EINVAL for odd q, q < 2, q > 64, q^d > min(n, GP_MAX_RANK), or as
 * gp_precond_build; GP_EUNSUPPORTED for a kernel other than GP_KERNEL_RBF;
 * GP_EWORKSPACE; GP_EHIP.  The call waits for its small host-to-device copy.
 */
int gp_precond_build_qff(const gp_problem* prob, const double* theta_host, int32_t nodes_per_dim,
                         void* ws_dev, size_t ws_bytes, hipStream_t stream, gp_precond** out);

/* gp_precond_view_of — device views of a built preconditioner. */
int gp_precond_view_of(const gp_precond* P, gp_precond_view* view);

/* gp_precond_free — releases the host handle only (the device arrays belong to
 * the workspace).  NULL is accepted. */
void gp_precond_free(gp_precond* P);

/*
 * gp_mll_eval — estimate of log p(y | theta), Algorithm 1 with the
 * preconditioned probes b_i = sigma eps_i + L eta_i (E[b b^T] = P_hat):
 * one preconditioned CG call on [y | b_1 .. b_ell] with on-the-fly K_hat
 * tiles (Section 4.4), the Lanczos tridiagonal from the CG coefficients
 * (supplement S1.2), Lanczos quadrature gamma_i = rho0_i sum_j tau_1j^2
 * log theta_j with rho0_i = b_i^T P_hat^-1 b_i, and
 *   log p ~ -1/2 (y^T u + log det P_hat + mean_i gamma_i + n log 2 pi).
 * P may be NULL (the preconditioner of opt-independent `rank` is then built in
 * `ws`).  Writes one FP64 to logp_dev.
 */
int gp_mll_eval(const gp_problem* prob, const double* theta_host, const gp_options* opt,
                int32_t rank, gp_precond* P, void* ws_dev, size_t ws_bytes,
                hipStream_t stream, double* logp_dev, gp_stats* stats);

/*
 * gp_mll_grad — the estimate of gp_mll_eval plus the gradient of Algorithm 2,
 * reusing the forward solves a_i = K_hat^-1 b_i and c_i = P_hat^-1 b_i:
 *   d/dtheta log p ~ 1/2 u^T dK_hat u
 *                    - 1/2 [ tr(P_hat^-1 dP_hat)
 *                            + mean_i (a_i^T dK_hat c_i - c_i^T dP_hat c_i) ]
 * with dK_hat tiles recomputed on the fly and tr(P_hat^-1 dP_hat) by the matrix
 * inversion lemma (supplement S3.3).  dP_hat holds the pivots fixed
 * (precond_grad = 0) or keeps only the s and sigma^2 terms (precond_grad = 1).
 * Writes one FP64 to logp_dev and p + 2 FP64 to grad_dev, ordered like theta.
 * Reuse: when the previous call on this workspace was a gp_mll_eval with the
 * same problem, theta, options, rank, preconditioner handle and stream, the
 * forward pass is not repeated: its solves and CG coefficients are read from
 * the workspace and only log p and the derivative are computed (the results
 * are bitwise those of a full call).  A gp_mll_grad after a gp_mll_grad always
 * runs the whole evaluation.  Any other call
 * on the workspace (preconditioner builds, gp_khat_matvec, gp_khat_profile,
 * gp_predict, batch calls) and gp_precond_free of the handle end the reuse; the
 * caller must not change X, y or the workspace in between (the record compares
 * pointers and values of the arguments, not the contents of device arrays).
 */
int gp_mll_grad(const gp_problem* prob, const double* theta_host, const gp_options* opt,
                int32_t rank, gp_precond* P, void* ws_dev, size_t ws_bytes,
                hipStream_t stream, double* logp_dev, double* grad_dev, gp_stats* stats);

/*
 * gp_predict — GP posterior at test points (Sec. 2.1: the posterior of f under
 * the zero-mean prior given y): for each test point x*_j
 *   mean_j = k(x*_j, X) K_hat^-1 y,
 *   var_j  = s - k(x*_j, X) K_hat^-1 k(X, x*_j)   (latent f; add sigma^2 for y*),
 * from preconditioned CG on [y | k(X, x*_j) for a chunk of test points] with the
 * same on-the-fly K_hat tiles, preconditioner and stopping rule as gp_mll_eval.
 * Test points go in chunks of opt->num_probes per CG call, so the workspace of
 * gp_workspace_size(prob, opt, rank) serves any nstar.  Xstar_dev: nstar x d
 * row-major FP64 device array; mean_dev: FP64[nstar]; var_dev: FP64[nstar] or
 * NULL.  opt->seed and precond_grad are unused.  P: NULL or a preconditioner
 * built in ws_dev for the same problem, theta and rank.  The call waits for
 * the stream at its end to report deferred errors (GP_ENOTSPD).
 * Errors: GP_EINVAL (null pointers, nstar < 1, bad shapes or theta),
 * GP_EWORKSPACE, GP_ENOTSPD, GP_EHIP.
 */
int gp_predict(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t rank,
               gp_precond* P, const double* Xstar_dev, int64_t nstar, void* ws_dev, size_t ws_bytes,
               hipStream_t stream, double* mean_dev, double* var_dev);

/*
 * gp_khat_matvec — W = K_hat V (the product inside every CG iteration) with
 * tiles of the given precision: V_dev and W_dev are n x num_rhs row-major FP64
 * (1 <= num_rhs <= 1 + GP_MAX_PROBES).  Uses the workspace for staging.
 */
int gp_khat_matvec(const gp_problem* prob, const double* theta_host, int32_t precision,
                   const double* V_dev, int32_t num_rhs, double* W_dev, void* ws_dev,
                   size_t ws_bytes, hipStream_t stream);

/*
 * gp_khat_profile — measurement helper: times the K_hat V tile kernel alone, in
 * the launch configuration gp_mll_eval uses for the same problem and options.
 * Fills the search-direction block of the workspace with a fixed pattern and
 * issues `reps` tile launches as CG iterations 0 .. reps-1 would with every
 * column active: with GP_PREC_BF16X3 tiles the first 16 split the search
 * directions in three BF16 pieces and the rest in two, as the solver does (a
 * different kernel instance; other precisions have one).  Each run of launches
 * with one split is staged and warmed up first, then bracketed by hipEvents on
 * `stream`; the call waits for them and writes the mean milliseconds per launch
 * over all `reps` launches to *ms_per_launch (host).  Also reports the
 * workgroup grid.
 */
int gp_khat_profile(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t reps,
                    void* ws_dev, size_t ws_bytes, hipStream_t stream, double* ms_per_launch,
                    int64_t* grid_x, int64_t* grid_y);

/*
 * gp_khat_matvec_noalloc — gp_khat_matvec for callers that cannot allocate
 * device memory (code under stream or graph capture, tight serving loops,
 * harnesses that forbid allocation): the same product W = K_hat V with the
 * same arguments minus the workspace.  Its staging arrays live in a device
 * array of GP_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from
 * the library's load until the process ends; the call allocates and frees
 * nothing.  Shapes whose arrays exceed that size are rejected with
 * GP_EWORKSPACE before any device work (fewer column splits are taken first,
 * so results may differ from gp_khat_matvec in rounding order only; roughly
 * n <= 130,000 for d = 16 and 65 right-hand sides in the split precisions).
 * Every call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (different streams or host threads) race and must be serialised by the
 * caller.  V_dev, W_dev: caller-owned n x num_rhs row-major FP64 device arrays.
 * Errors: GP_EINVAL (null pointers, bad shapes, precision or theta),
 * GP_EWORKSPACE (shape too large for the array), GP_EUNSUPPORTED, GP_EHIP.
 */
#define GP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int gp_khat_matvec_noalloc(const gp_problem* prob, const double* theta_host, int32_t precision,
                           const double* V_dev, int32_t num_rhs, double* W_dev, hipStream_t stream);

/*
 * Ragged batches of independent problems
 * --------------------------------------
 * One call evaluates Algorithm 1 (and, for the _grad form, Algorithm 2) for
 * every problem of a batch; each phase of the method is one launch for all
 * problems, and every problem keeps its own hyperparameters, preconditioner,
 * CG scalars and per-column convergence mask (the many-right-hand-sides CG of
 * Section 4.4, across problems).  Problem b gives exactly the result of
 * gp_mll_eval / gp_mll_grad on that problem alone with seed + b and rank
 * min(rank, n_b), up to rounding order.
 *
 * X_dev holds the problems' points one after another (sum_b n_b rows of d
 * FP64, row-major), y_dev their targets; problem b is rows
 * offsets_host[b] .. offsets_host[b+1] - 1.  offsets_host is a host array of
 * batch + 1 entries starting at 0 and strictly increasing.  All problems share
 * d, kernel, ard and the options.
 */
typedef struct gp_batch {
  const double* X_dev;
  const double* y_dev;
  const int64_t* offsets_host;
  int32_t batch;    /* number of problems, 1 .. 65536 */
  int32_t d;        /* 1 .. GP_MAX_D */
  int32_t kernel;   /* gp_kernel */
  int32_t ard;      /* 1: d lengthscales per problem, 0: one */
} gp_batch;

/* Per-batch statistics (optional; asking for them synchronises the stream). */
typedef struct gp_batch_stats {
  int32_t iters_max;      /* largest CG iteration count over all problems and columns */
  int32_t flags_any;      /* OR of the per-problem GP_FLAG_* bits */
  int32_t* iters_host;    /* NULL or int32[batch]: per-problem largest column iteration count */
  int32_t* flags_host;    /* NULL or int32[batch]: per-problem GP_FLAG_* bits */
  int32_t* rank_host;     /* NULL or int32[batch]: per-problem achieved preconditioner rank */
} gp_batch_stats;

/* Limits of the batched path. */
#define GP_BATCH_MAX_RANK 256
#define GP_BATCH_MAX_PROBES 64

/*
 * gp_batch_workspace_size — bytes of device workspace for gp_batch_mll_eval /
 * gp_batch_mll_grad with these problems, options and rank.  Only
 * offsets_host, batch, d, kernel and ard of *batch are read.
 * Errors: GP_EINVAL for bad sizes or options; GP_EUNSUPPORTED for a precision
 * other than GP_PREC_FP64 / GP_PREC_FP32, num_probes > GP_BATCH_MAX_PROBES or
 * rank > GP_BATCH_MAX_RANK.
 */
int gp_batch_workspace_size(const gp_batch* batch, const gp_options* opt, int32_t rank, size_t* bytes);

/*
 * gp_batch_mll_eval — log p for every problem of the batch.
 *   theta_host  batch x (p + 2) natural hyperparameters, row b for problem b.
 *   rank        requested pivoted-Cholesky rank; problem b uses min(rank, n_b).
 *   ws_dev      256-byte aligned device workspace of at least
 *               gp_batch_workspace_size bytes, owned by the caller.
 *   logp_dev    device FP64[batch] output.
 *   stats       NULL, or statistics filled after a stream synchronisation.
 * The call copies its small problem tables (sizes, offsets, hyperparameters,
 * work items) from the host into the workspace and waits for that copy once.
 * Deferred errors (GP_ENOTSPD in any problem) are reported only when stats is
 * non-NULL.  Errors as gp_batch_workspace_size, plus GP_EINVAL for null
 * pointers or theta <= 0 / NaN, GP_EWORKSPACE, GP_EHIP.
 */
int gp_batch_mll_eval(const gp_batch* batch, const double* theta_host, const gp_options* opt, int32_t rank,
                      void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev, gp_batch_stats* stats);

/*
 * gp_batch_mll_grad — as gp_batch_mll_eval, plus the gradient of every
 * problem's estimate with respect to its natural theta (Algorithm 2 with the
 * solves reused, as gp_mll_grad) into grad_dev: device FP64[batch x (p + 2)],
 * row b for problem b.  The kernel-derivative sweep runs in FP64.
 */
int gp_batch_mll_grad(const gp_batch* batch, const double* theta_host, const gp_options* opt, int32_t rank,
                      void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev, double* grad_dev,
                      gp_batch_stats* stats);

/* gp_strerror — static text for a gp_status. */
const char* gp_strerror(int status);

/* gp_last_hip_error — the hipError_t behind the last GP_EHIP on this thread. */
int gp_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GPMLL_H */
