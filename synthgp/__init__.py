"""Seeded synthetic GP-regression workloads.

This module only draws inputs: point sets X, targets y and hyperparameters
theta, plus the solver settings of each workload.  It holds none of the
estimator's arithmetic (no kernel matrix, no solve, no trace estimate), so
that both the CPU reference and the GPU path can take their inputs from it.

Targets are drawn from the GP prior through random Fourier features
(Rahimi & Recht 2007): for a stationary kernel with spectral density p(w),
    f(x) = sqrt(2 s / F) * sum_f cos(w_f . x + b_f),  w_f ~ p,  b_f ~ U[0, 2 pi)
has covariance s * kappa(r) up to O(F^-1/2); y = f + sigma * N(0, 1).
The spectral density of the RBF kernel with lengthscales ls is N(0, diag(ls)^-2);
that of a Matern-nu kernel is a multivariate t with 2 nu degrees of freedom,
    w = z * sqrt(2 nu / u) / ls,  z ~ N(0, I),  u ~ chi^2(2 nu)
(Rasmussen & Williams 2006, Sec. 4.2); the rational quadratic kernel with shape
alpha is a Gamma(alpha, rate alpha) scale mixture of RBF kernels, so
    w = z * sqrt(tau) / ls,  tau ~ Gamma(alpha, rate alpha).

Theta layout everywhere: [ls_1 .. ls_p | s | sigma^2] with p = d for ARD
kernels and p = 1 for isotropic ones; all entries are natural (positive)
parameters.
"""
from __future__ import annotations

import dataclasses
import numpy as np

KERNELS = ("rbf", "matern32", "matern52", "ratquad:<alpha>")
PRECISIONS = ("fp64", "fp32", "bf16x3")


@dataclasses.dataclass
class GPProblem:
    name: str
    X: np.ndarray            # (n, d) float64, C-contiguous
    y: np.ndarray            # (n,) float64
    theta: np.ndarray        # (p + 2,) float64, natural parameters
    kernel: str              # one of KERNELS
    ard: bool
    rank: int                # pivoted-Cholesky rank k
    num_probes: int          # number of probe vectors (ell)
    tol: float               # relative CG residual tolerance
    max_iters: int
    precision: str           # tile precision, one of PRECISIONS
    probe_seed: int = 1
    recipe: str = ""

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def rff_targets(rng, X, ls, s, sigma2, kernel, num_features=4096):
    """One approximate GP-prior draw at X plus N(0, sigma2) noise (module docstring)."""
    n, d = X.shape
    ls = np.broadcast_to(np.asarray(ls, dtype=np.float64), (d,))
    z = rng.standard_normal((num_features, d))
    if kernel == "rbf":
        w = z / ls
    elif kernel.startswith("ratquad"):
        alpha = float(kernel.split(":", 1)[1]) if ":" in kernel else 1.0
        tau = rng.gamma(alpha, 1.0 / alpha, size=(num_features, 1))
        w = z * np.sqrt(tau) / ls
    else:
        nu = {"matern32": 1.5, "matern52": 2.5}[kernel]
        u = rng.chisquare(2.0 * nu, size=(num_features, 1))
        w = z * np.sqrt(2.0 * nu / u) / ls
    b = rng.uniform(0.0, 2.0 * np.pi, size=num_features)
    f = np.zeros(n)
    # chunk over points to bound memory at n = 300k
    for lo in range(0, n, 8192):
        hi = min(n, lo + 8192)
        f[lo:hi] = np.cos(X[lo:hi] @ w.T + b).sum(axis=1)
    f *= np.sqrt(2.0 * s / num_features)
    return f + np.sqrt(sigma2) * rng.standard_normal(n)


def spectral_frequencies(kernel, m, d, seed=0):
    """m samples (m, d) of the kernel's spectral density at unit lengthscale, the
    random input of the random Fourier feature preconditioner: N(0, I) for the
    RBF kernel, z * sqrt(2 nu / u) with z ~ N(0, I), u ~ chi^2(2 nu) for Matern-nu,
    z * sqrt(tau), tau ~ Gamma(alpha, rate alpha) for the rational quadratic
    (module docstring)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x52FF]))
    z = rng.standard_normal((m, d))
    if kernel == "rbf":
        return z
    if kernel.startswith("ratquad"):
        alpha = float(kernel.split(":", 1)[1]) if ":" in kernel else 1.0
        return z * np.sqrt(rng.gamma(alpha, 1.0 / alpha, size=(m, 1)))
    nu = {"matern32": 1.5, "matern52": 2.5}[kernel]
    u = rng.chisquare(2.0 * nu, size=(m, 1))
    return z * np.sqrt(2.0 * nu / u)


def uniform_landmarks(n, k, seed=0):
    """k distinct rows of n drawn uniformly without replacement, the random input of
    the randomized Nystrom preconditioner (column probabilities proportional to
    K_ii^2 are uniform for a stationary kernel)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x4E59]))
    return rng.choice(n, size=k, replace=False).astype(np.int32)


def plain_rbf_1000(n=1000, seed=0):
    """Uniform[0,1]^3 inputs, isotropic RBF (ls 0.3, s 1, sigma^2 0.1), FP64 tiles."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 3))
    theta = np.array([0.3, 1.0, 0.1])
    y = rff_targets(rng, X, theta[0], theta[1], theta[2], "rbf")
    return GPProblem("plain_rbf_fp64", X, y, theta, "rbf", False, rank=10, num_probes=16,
                     tol=1e-6, max_iters=200, precision="fp64",
                     recipe="X~U[0,1]^3; RBF iso ls=0.3 s=1 s2=0.1; y=RFF(4096)+noise")


def matern52_ard_20k(n=20000, seed=0):
    """N(0, I_8) inputs, Matern-5/2 ARD (ls ~ LogU[0.5, 2]), sigma^2 0.01, FP32 tiles.
    CG tolerance 1e-6 with a cap of 500 iterations: with the rank-50 preconditioner
    the columns need 284-300 iterations at this tolerance with FP64 tiles and
    332-355 with FP32 tiles at n = 20000, so a cap of 200 stops every column short."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8))
    ls = _loguniform(rng, 0.5, 2.0, 8)
    theta = np.concatenate([ls, [1.0, 0.01]])
    y = rff_targets(rng, X, ls, 1.0, 0.01, "matern52")
    return GPProblem("matern52_ard_fp32", X, y, theta, "matern52", True, rank=50,
                     num_probes=32, tol=1e-6, max_iters=500, precision="fp32",
                     recipe="X~N(0,I_8); Matern52 ARD ls~LogU[0.5,2] s=1 s2=0.01; y=RFF(4096)+noise")


def rbf_ard_100k(n=100000, seed=0, precision="bf16x3"):
    """Uniform[0,1]^16 inputs, RBF ARD (ls ~ LogU[0.1, 1]), sigma^2 1e-3,
    y = sin(2 pi X w) + 0.1 N(0, 1) with w ~ N(0, I)/4."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 16))
    ls = _loguniform(rng, 0.1, 1.0, 16)
    theta = np.concatenate([ls, [1.0, 1e-3]])
    w = rng.standard_normal(16) / 4.0
    y = np.sin(2.0 * np.pi * (X @ w)) + 0.1 * rng.standard_normal(n)
    return GPProblem("rbf_ard_100k", X, y, theta, "rbf", True, rank=100, num_probes=64,
                     tol=1e-6, max_iters=200, precision=precision,
                     recipe="X~U[0,1]^16; RBF ARD ls~LogU[0.1,1] s=1 s2=1e-3; "
                            "y=sin(2pi Xw)+0.1N, w~N(0,I)/4")


def batched_rbf_64(num_problems=64, n_lo=500, n_hi=8000, seed=0):
    """64 independent problems, n_b ~ U{500..8000}, X ~ N(0, I_4), isotropic RBF with
    ls ~ LogU[0.2, 2], sigma^2 ~ LogU[1e-3, 1e-1], s 1; FP64 tiles (FP32 tiles miss
    the gradient bar on the worst-conditioned problems).  Rank 20, 16
    probes, CG tolerance 1e-6 with a cap of 2500 iterations (the slowest problems
    need about 1650 at this tolerance with FP64 tiles, 1950 with FP32 tiles)."""
    rng = np.random.default_rng(seed)
    out = []
    sizes = rng.integers(n_lo, n_hi + 1, size=num_problems)
    for b, nb in enumerate(sizes):
        X = rng.standard_normal((int(nb), 4))
        ls = float(_loguniform(rng, 0.2, 2.0, 1)[0])
        s2 = float(_loguniform(rng, 1e-3, 1e-1, 1)[0])
        theta = np.array([ls, 1.0, s2])
        y = rff_targets(rng, X, ls, 1.0, s2, "rbf")
        out.append(GPProblem(f"batched_rbf_{b}", X, y, theta, "rbf", False, rank=20,
                             num_probes=16, tol=1e-6, max_iters=2500, precision="fp64",
                             recipe="X~N(0,I_4); RBF iso ls~LogU[0.2,2] s=1 s2~LogU[1e-3,1e-1]; "
                                    "y=RFF(4096)+noise"))
    return out


def gmm_matern32_300k(n=300000, seed=0, precision="bf16x3"):
    """10-component Gaussian mixture in R^20 (means ~ N(0, 4I), unit covariances),
    Matern-3/2 ARD with truth ls ~ LogU[1, 4], s 1, sigma^2 1e-2; y = RFF(4096) + noise.
    The returned theta is the optimiser's start (ls 1, s 1, sigma^2 0.1)."""
    rng = np.random.default_rng(seed)
    d = 20
    means = 2.0 * rng.standard_normal((10, d))
    comp = rng.integers(0, 10, size=n)
    X = means[comp] + rng.standard_normal((n, d))
    ls_true = _loguniform(rng, 1.0, 4.0, d)
    y = rff_targets(rng, X, ls_true, 1.0, 1e-2, "matern32")
    theta0 = np.concatenate([np.ones(d), [1.0, 0.1]])
    return GPProblem("gmm_matern32_300k", X, y, theta0, "matern32", True, rank=200,
                     num_probes=64, tol=1e-6, max_iters=400, precision=precision,
                     recipe="X~GMM(10, means N(0,4I), unit cov) in R^20; Matern32 ARD "
                            "truth ls~LogU[1,4] s=1 s2=1e-2; y=RFF(4096)+noise; "
                            "start ls=1 s=1 s2=0.1")


def random_problem(n, d, kernel="rbf", ard=True, rank=8, num_probes=8, seed=0,
                   ls_range=(0.3, 1.5), sigma2=0.05, s=1.0, dist="uniform",
                   precision="fp64", tol=1e-8, max_iters=200):
    """Small generic problem used by the parity and property tests."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        X = rng.uniform(0.0, 1.0, size=(n, d))
    else:
        X = rng.standard_normal((n, d))
    p = d if ard else 1
    ls = _loguniform(rng, ls_range[0], ls_range[1], p)
    theta = np.concatenate([ls, [s, sigma2]])
    y = rff_targets(rng, X, ls if ard else ls[0], s, sigma2, kernel, num_features=1024)
    return GPProblem(f"random_{kernel}_{n}x{d}", X, y, theta, kernel, ard, rank=rank,
                     num_probes=num_probes, tol=tol, max_iters=max_iters, precision=precision,
                     recipe=f"X~{dist}; {kernel} ard={ard}; y=RFF(1024)+noise")


TABLE_S1_KERNELS = ("matern32", "rbf", "ratquad:1.0")


def table_s1(kernel="rbf", d=1, n=10000, seed=0):
    """The synthetic experiment of Table S1: n = 10,000 iid standard normal points in
    d dimensions, sigma^2 = 1e-2.  The paper leaves the remaining parameters open:
    isotropic lengthscale 1, outputscale 1, rational quadratic shape 1, and y drawn
    from the GP through random features plus noise."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x51, int(d)]))
    X = rng.standard_normal((n, d))
    theta = np.array([1.0, 1.0, 1e-2])
    y = rff_targets(rng, X, 1.0, 1.0, 1e-2, kernel)
    return GPProblem(f"table_s1_{kernel}_d{d}", X, y, theta, kernel, False, rank=128, num_probes=128,
                     tol=1e-10, max_iters=3000, precision="fp64",
                     recipe=f"X~N(0,I_{d}), n={n}; {kernel} iso ls=1 s=1 s2=1e-2; y=RFF(4096)+noise")
