"""CPU FP64 reference ("oracle") for the preconditioned GP log-marginal-likelihood
estimator and its derivative (Wenger, Pleiss, Hennig, Cunningham, Gardner:
"Preconditioning for Scalable Gaussian Process Hyperparameter Optimization").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module: only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the HIP path.

Two parts:

* exact_mll: the exact targets, Eq. (1) (log marginal likelihood) and Eq. (2)
  (its derivative), by a dense FP64 Cholesky factorisation (LAPACK potrf);
  predict: the posterior mean and latent variance at test points, likewise.
* estimate_mll: the stochastic estimator of Algorithms 1 and 2 (Section 4.4),
  step by step in the paper's order, with dense or row-blocked matrix products:
  partial pivoted Cholesky preconditioner P = sigma^2 I + L L^T (Section 2.2,
  "Preconditioning"; supplement S5.3), solves with P through the matrix
  inversion lemma, preconditioned CG on [y | probes] (one call with many right
  hand sides, footnote to Section 4.4), the Lanczos tridiagonal from the CG
  coefficients (supplement S1.2), Lanczos quadrature for the log (Section 2.2,
  SLQ), the log-determinant decomposition (Section 3) and the derivative
  decomposition (Section 3.3) with the trace of P^-1 dP computed by the matrix
  inversion lemma (supplement S3.3).  The random Fourier feature preconditioner
  of Table 1 (reading R-rff) can replace the pivoted Cholesky one.

Readings taken where the paper is silent or loose (each is listed with its reason
in the design notes):

R-probe  Probes for the preconditioned quadrature are b_i = sigma*eps_i + L*eta_i
         with Rademacher eps_i (length n) and eta_i (length k), so E[b b^T] = P.
         Quadrature weight of probe i is rho0_i = b_i^T P^-1 b_i (the first r^T z
         of preconditioned CG): gamma_i = rho0_i * sum_j tau_1j^2 log(theta_j).
         This makes (1/ell) sum_i gamma_i unbiased for tr log(P^-1/2 K P^-T/2).
R-sqrt   The alternative probe b_i = P^1/2 w_i with the symmetric square root of P
         and Rademacher w_i (length n, the eps stream): E[b b^T] = P as under
         R-probe, and rho0_i = w_i^T w_i = n exactly, the (n/ell) normalisation of
         the paper's Hutchinson form.
R-quad   The quadrature sums over the m Ritz values of the m x m tridiagonal
         produced by m CG steps (indices 1..m).
R-grad   The derivative probes reuse the forward solves: with a_i = K^-1 b_i and
         c_i = P^-1 b_i, gamma'_i = a_i^T dK c_i - c_i^T dP c_i, whose expectation
         is tr(K^-1 dK) - tr(P^-1 dP), the residual trace of Section 3.3.
R-dP     dP/dtheta of the pivoted Cholesky factor is taken with the pivots held
         fixed; the rank-k partial pivoted Cholesky equals the Nystrom
         approximation K_{:S} K_SS^-1 K_{S:} on its pivot set S.  Mode 1 keeps only
         the outputscale and noise terms (dP/dls = 0); any fixed choice keeps the
         estimator unbiased because the deterministic term and the control
         variate cancel in expectation.
R-chol   Greedy pivoting on the residual diagonal, ties to the lowest index; run
         exactly k steps, stopping early only when the largest residual diagonal
         is <= 1e-12 * s; L factors K without the noise term.
R-cg     x0 = 0; a column stops after the iteration whose updated recurrence
         residual satisfies ||r|| <= tol * ||b||; its alpha/beta stream ends there.
R-rq     Rational quadratic kernel (used with the RBF and Matern-3/2 kernels in
         Table S1): kappa = (1 + r^2 / (2 alpha))^-alpha with the shape alpha a
         fixed kernel constant (kind "ratquad:<alpha>"), not a hyperparameter
         of theta; the paper does not optimise it.
R-kern   k(x, x') = s * kappa(r), r^2 = sum_j ((x_j - x'_j) / ls_j)^2, noise
         sigma^2 on the diagonal; theta = [ls | s | sigma^2] natural parameters.
R-ritz   Ritz values below 1e-300 are clamped to 1e-300 before the log.
R-nys    Randomized Nystrom preconditioner (Table 1; supplement S5, randomized
         Nystrom approximation quality): the landmark rows S are an input, drawn
         with probabilities proportional to K_ii^2 (uniform for a stationary
         kernel) without replacement and with s = k landmarks, so no rank-k
         truncation of K_SS^+ is needed: P = sigma^2 I + K_{:S} K_SS^-1 K_{S:}, the
         partial Cholesky with the pivots prescribed in the order of S.  Its
         derivative holds S fixed, exactly as R-dP.
R-qff    Quadrature Fourier features (Table 1, "QFF", RBF kernel): the frequencies
         of R-rff are the nodes of a tensor Gauss-Hermite rule with q (even)
         points per dimension for the standard normal spectral density; of each
         +-pair of nodes one is kept with its weight doubled, and feature j has
         amplitude sqrt(s w_j) instead of sqrt(s/m).  Rank q^d.
R-rff    Random Fourier feature preconditioner (Table 1, "RFF"): m = k/2 frequency
         samples w_j of the kernel's spectral density at unit lengthscale are an
         input; Z = sqrt(s/m) [cos(Phi) | sin(Phi)] with Phi = X~ W^T and
         X~ = (X - column mean) / ls, so Z Z^T = (s/m) sum_j cos(w_j.(x~_a - x~_b))
         (the origin of the phases is invisible in Z Z^T; the data mean fixes Z).
         dP/dtheta holds the frequencies fixed.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np
import scipy.linalg as sla

KIND = {"rbf": 0, "matern32": 1, "matern52": 2}
SQRT3 = math.sqrt(3.0)
SQRT5 = math.sqrt(5.0)
LOG2PI = math.log(2.0 * math.pi)
PIVOT_BREAKDOWN = 1e-12
RITZ_FLOOR = 1e-300


# ----------------------------------------------------------------------------
# Kernels (Section 2.1; forms of Rasmussen & Williams 2006, Sec. 4.2)
# ----------------------------------------------------------------------------

def split_theta(theta, d, ard):
    theta = np.asarray(theta, dtype=np.float64)
    p = d if ard else 1
    if theta.shape != (p + 2,):
        raise ValueError(f"theta must have {p + 2} entries, got {theta.shape}")
    ls = np.broadcast_to(theta[:p], (d,)).copy()
    return ls, float(theta[p]), float(theta[p + 1])


def scaled_differences(X1, X2, ls):
    """(x_p - x_q) / ls per dimension, by direct differences: shape (n1, n2, d)."""
    return (X1[:, None, :] - X2[None, :, :]) / ls


def sqdist(X1, X2, ls):
    """r^2 by direct differences (no inner-product expansion)."""
    D = scaled_differences(X1, X2, ls)
    return np.einsum("pqj,pqj->pq", D, D)


def ratquad_shape(kind):
    """alpha of a rational quadratic kind "ratquad:<alpha>" (None for other kinds)."""
    if not kind.startswith("ratquad"):
        return None
    alpha = float(kind.split(":", 1)[1]) if ":" in kind else 1.0
    if not alpha > 0.0:
        raise ValueError(kind)
    return alpha


def kappa(kind, r2):
    """Correlation kappa(r) of the stationary kernel, k = s * kappa."""
    if kind == "rbf":
        return np.exp(-0.5 * r2)
    alpha = ratquad_shape(kind)
    if alpha is not None:
        return (1.0 + r2 / (2.0 * alpha)) ** (-alpha)
    r = np.sqrt(r2)
    if kind == "matern32":
        return (1.0 + SQRT3 * r) * np.exp(-SQRT3 * r)
    if kind == "matern52":
        return (1.0 + SQRT5 * r + (5.0 / 3.0) * r2) * np.exp(-SQRT5 * r)
    raise ValueError(kind)


def gfun(kind, r2):
    """g(r) with d kappa / d ls_j = g(r) * dtilde_j^2 / ls_j (dtilde = scaled diff)."""
    if kind == "rbf":
        return np.exp(-0.5 * r2)
    alpha = ratquad_shape(kind)
    if alpha is not None:
        return (1.0 + r2 / (2.0 * alpha)) ** (-alpha - 1.0)
    r = np.sqrt(r2)
    if kind == "matern32":
        return 3.0 * np.exp(-SQRT3 * r)
    if kind == "matern52":
        return (5.0 / 3.0) * (1.0 + SQRT5 * r) * np.exp(-SQRT5 * r)
    raise ValueError(kind)


def kernel_matrix(X1, X2, theta, kind, ard):
    """K(X1, X2) = s * kappa(r) (no noise)."""
    ls, s, _ = split_theta(theta, X1.shape[1], ard)
    return s * kappa(kind, sqdist(X1, X2, ls))


def khat_dense(X, theta, kind, ard):
    """K_hat = K(X, X) + sigma^2 I (Section 2.1)."""
    ls, s, s2 = split_theta(theta, X.shape[1], ard)
    K = kernel_matrix(X, X, theta, kind, ard)
    K[np.diag_indices_from(K)] += s2
    return K


def _row_block(n, d, budget=4e7):
    return max(1, int(budget // max(1, n * d)))


def _over_blocks(fn, starts, workers):
    """fn(start) for every block start, in order; with workers > 1 the blocks run
    on a thread pool (NumPy releases the interpreter lock in its array loops), and
    the results still come back in block order."""
    if workers <= 1:
        return [fn(lo) for lo in starts]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, starts))


_NATIVE = None


def _native():
    """The plain-C matrix-free products (oracle/khat_native.c), compiled with gcc
    next to their source on first use (or when the source is newer)."""
    global _NATIVE
    if _NATIVE is None:
        import ctypes
        import os
        here = os.path.dirname(os.path.abspath(__file__))
        src = os.path.join(here, "khat_native.c")
        lib = os.path.join(here, "liboracle_khat.so")
        if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            build_native(src, lib)
        h = ctypes.CDLL(lib)
        P = ctypes.POINTER(ctypes.c_double)
        h.oracle_khat_matvec.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), P]
        h.oracle_dkhat_lowrank.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_int32,
                                           ctypes.c_double, ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int64, P]
        _NATIVE = h
    return _NATIVE


def build_native(src=None, lib=None):
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    src = src or os.path.join(here, "khat_native.c")
    lib = lib or os.path.join(here, "liboracle_khat.so")
    tmp = lib + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, lib)
    return lib


def _native_kind(kind):
    alpha = ratquad_shape(kind)
    if alpha is not None:
        return 3, alpha
    return KIND[kind], 0.0


def _dptr(a):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def khat_matvec(X, theta, kind, ard, V, rows=None, workers=1, native=False):
    """K_hat[rows, :] @ V with K_hat rows built block by block (matrix-free for large n).
    workers: threads over row blocks (each output row is computed the same way).
    native: the same product by the plain-C loops of khat_native.c."""
    n, d = X.shape
    ls, s, s2 = split_theta(theta, d, ard)
    V = np.asarray(V, dtype=np.float64)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    if native:
        import ctypes
        Xc = np.ascontiguousarray(X, dtype=np.float64)
        V2 = np.ascontiguousarray(V.reshape(n, -1))
        rr = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty((rr.size, V2.shape[1]))
        code, alpha = _native_kind(kind)
        rc = _native().oracle_khat_matvec(n, d, _dptr(Xc), _dptr(ls), s, s2, code, alpha, V2.shape[1],
                                          _dptr(V2), rr.size, rr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          _dptr(out))
        if rc != 0:
            raise ValueError("oracle_khat_matvec failed")
        return out.reshape((rr.size,) + V.shape[1:])
    out = np.empty((rows.size,) + V.shape[1:])
    blk = _row_block(n, d)

    def block(lo):
        r = rows[lo:lo + blk]
        Kb = s * kappa(kind, sqdist(X[r], X, ls))
        out[lo:lo + blk] = Kb @ V
        out[lo:lo + blk] += s2 * V[r]

    _over_blocks(block, range(0, rows.size, blk), workers)
    return out


def dkhat_contract(X, theta, kind, ard, m_rows, workers=1):
    """sum_pq M_pq dK_hat_pq / dtheta for every theta, with M given block-of-rows
    at a time by m_rows(rows) -> (|rows|, n).  Order of the result follows theta.
    workers: threads over row blocks; the block sums are added in block order."""
    n, d = X.shape
    ls, s, s2 = split_theta(theta, d, ard)
    p = d if ard else 1
    blk = _row_block(n, d)

    def block(lo):
        part = np.zeros(p + 2)
        r = np.arange(lo, min(n, lo + blk))
        Dt = scaled_differences(X[r], X, ls)
        r2 = np.einsum("pqj,pqj->pq", Dt, Dt)
        M = m_rows(r)
        W = s * gfun(kind, r2) * M
        per_dim = np.einsum("pq,pqj->j", W, Dt * Dt) / ls
        if ard:
            part[:p] = per_dim
        else:
            part[0] = per_dim.sum()
        part[p] = np.sum(kappa(kind, r2) * M)
        part[p + 1] = np.sum(M[np.arange(r.size), r])
        return part

    out = np.zeros(p + 2)
    for part in _over_blocks(block, range(0, n, blk), workers):
        out += part
    return out


def dkhat_contract_lowrank(X, theta, kind, ard, A, C, row_range=None):
    """dkhat_contract for M = A C^T by the plain-C loops of khat_native.c
    (row_range = (p0, p1): only the rows p0 <= p < p1 of M)."""
    n, d = X.shape
    ls, s, _ = split_theta(theta, d, ard)
    p = d if ard else 1
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    Ac = np.ascontiguousarray(A, dtype=np.float64)
    Cc = np.ascontiguousarray(C, dtype=np.float64)
    raw = np.zeros(d + 2)
    code, alpha = _native_kind(kind)
    p0, p1 = (0, n) if row_range is None else row_range
    rc = _native().oracle_dkhat_lowrank(n, d, _dptr(Xc), _dptr(ls), s, code, alpha, Ac.shape[1], _dptr(Ac),
                                        _dptr(Cc), int(p0), int(p1), _dptr(raw))
    if rc != 0:
        raise ValueError("oracle_dkhat_lowrank failed")
    out = np.zeros(p + 2)
    if ard:
        out[:p] = raw[:d]
    else:
        out[0] = raw[:d].sum()
    out[p:] = raw[d:]
    return out


def dkernel_cols(X, theta, kind, ard, cols):
    """dK[:, cols]/dtheta for the kernel parameters (ls..., s): list of (n, |cols|)."""
    n, d = X.shape
    ls, s, _ = split_theta(theta, d, ard)
    Dt = scaled_differences(X, X[cols], ls)
    r2 = np.einsum("pqj,pqj->pq", Dt, Dt)
    g = s * gfun(kind, r2)
    mats = []
    if ard:
        for j in range(d):
            mats.append(g * Dt[:, :, j] ** 2 / ls[j])
    else:
        mats.append(g * r2 / ls[0])
    mats.append(kappa(kind, r2))
    return mats


# ----------------------------------------------------------------------------
# Exact targets: Eq. (1) and Eq. (2) via dense Cholesky
# ----------------------------------------------------------------------------

def exact_mll(X, y, theta, kind, ard, grad=True):
    """Exact log p(y | theta) (Eq. 1) and, if grad, its gradient (Eq. 2) in FP64."""
    n, d = X.shape
    Kh = khat_dense(X, theta, kind, ard)
    R = sla.cholesky(Kh, lower=True, overwrite_a=False, check_finite=True)
    logdet = 2.0 * np.sum(np.log(np.diag(R)))
    u = sla.cho_solve((R, True), y)
    datafit = float(y @ u)
    logp = -0.5 * (datafit + logdet + n * LOG2PI)
    if not grad:
        return {"logp": logp, "logdet": logdet, "datafit": datafit, "u": u}
    Kinv = sla.cho_solve((R, True), np.eye(n))
    del Kh, R
    # dL/dtheta = sum_pq dK_hat_pq (u_p u_q / 2 - Kinv_pq / 2)
    grad = dkhat_contract(X, theta, kind, ard,
                          lambda r: 0.5 * np.outer(u[r], u) - 0.5 * Kinv[r])
    return {"logp": logp, "grad": grad, "logdet": logdet, "datafit": datafit, "u": u}


def predict(X, y, theta, kind, ard, Xstar):
    """GP posterior at test points (Sec. 2.1: the posterior of f given y under the
    zero-mean prior): mean k(X*, X) K_hat^-1 y and latent variance
    k(x*, x*) - k(x*, X) K_hat^-1 k(X, x*) (noise not added), by a dense FP64
    Cholesky factorisation of K_hat."""
    Kh = khat_dense(X, theta, kind, ard)
    R = sla.cholesky(Kh, lower=True)
    Ks = kernel_matrix(X, np.asarray(Xstar, dtype=np.float64), theta, kind, ard)   # n x n*
    u = sla.cho_solve((R, True), y)
    A = sla.cho_solve((R, True), Ks)
    _, s, _ = split_theta(theta, X.shape[1], ard)
    return Ks.T @ u, s - np.sum(Ks * A, axis=0)


def bareiss_det(A):
    """Exact determinant of a rational matrix by fraction-free Bareiss elimination."""
    M = [[Fraction(v) for v in row] for row in A]
    n = len(M)
    sign, prev = 1, Fraction(1)
    for k in range(n - 1):
        if M[k][k] == 0:
            swap = next((i for i in range(k + 1, n) if M[i][k] != 0), None)
            if swap is None:
                return Fraction(0)
            M[k], M[swap] = M[swap], M[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = (M[i][j] * M[k][k] - M[i][k] * M[k][j]) / prev
        prev = M[k][k]
    return sign * M[n - 1][n - 1]


# ----------------------------------------------------------------------------
# Counter-based Rademacher signs: SplitMix64 (Steele, Lea & Flood 2014)
# ----------------------------------------------------------------------------

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """Output number `counter` (0-based) of SplitMix64 started from state `seed`:
    mix(seed + (counter + 1) * golden_gamma), with the 64-bit finaliser whose
    shifts are 30, 27, 31."""
    with np.errstate(over="ignore"):
        c = np.asarray(counter, dtype=np.uint64)
        z = np.uint64(seed) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def rademacher(seed, stream, col, count):
    """Signs for probe column `col`: entry i is +1 when the top bit of SplitMix64
    output (stream << 56 | col << 32 | i) is clear, else -1.  stream 0 feeds the
    n-vector eps, stream 1 the k-vector eta."""
    base = (np.uint64(stream) << np.uint64(56)) | (np.uint64(col) << np.uint64(32))
    ctr = base + np.arange(count, dtype=np.uint64)
    top = splitmix64(seed, ctr) >> np.uint64(63)
    return 1.0 - 2.0 * top.astype(np.float64)


def probe_signs(seed, n, k, ell):
    E = np.stack([rademacher(seed, 0, i, n) for i in range(ell)], axis=1) if ell else np.zeros((n, 0))
    H = np.stack([rademacher(seed, 1, i, k) for i in range(ell)], axis=1) if ell else np.zeros((k, 0))
    return E, H


# ----------------------------------------------------------------------------
# Partial pivoted Cholesky and the diagonal-plus-low-rank preconditioner
# ----------------------------------------------------------------------------

def pivoted_cholesky(X, theta, kind, ard, k, order=None):
    """Greedy partial pivoted Cholesky of K (noise excluded), R-chol.
    Returns L (n, k) with zero columns after an early stop, pivots, achieved rank.
    order: k distinct rows taken as the pivots in that order instead of the
    greedy choice (the randomized Nystrom preconditioner, reading R-nys)."""
    n, d = X.shape
    ls, s, _ = split_theta(theta, d, ard)
    if order is not None:
        order = np.asarray(order, dtype=np.int64)
        if order.shape != (k,) or len(set(order.tolist())) != k or order.min() < 0 or order.max() >= n:
            raise ValueError("order must hold k distinct rows")
    L = np.zeros((n, k))
    diag = np.full(n, s)
    piv = []
    for j in range(k):
        i = int(np.argmax(diag)) if order is None else int(order[j])
        if not diag[i] > PIVOT_BREAKDOWN * s:
            break
        piv.append(i)
        kcol = s * kappa(kind, sqdist(X, X[i:i + 1], ls)[:, 0])
        col = kcol - L[:, :j] @ L[i, :j]
        pivot_val = math.sqrt(diag[i])
        L[:, j] = col / pivot_val
        L[i, j] = pivot_val
        L[piv[:-1], j] = 0.0
        diag -= L[:, j] ** 2
        diag[piv] = 0.0
    return L, np.array(piv, dtype=np.int64), len(piv)


class Preconditioner:
    """P = sigma^2 I + L L^T, solves by the matrix inversion lemma and its
    log-determinant by the matrix determinant lemma."""

    def __init__(self, L, sigma2):
        self.L = L
        self.s2 = float(sigma2)
        n, k = L.shape
        self.C = self.s2 * np.eye(k) + L.T @ L
        self.Rc = sla.cholesky(self.C, lower=True) if k else np.zeros((0, 0))
        self.logdet = (n - k) * math.log(self.s2) + 2.0 * float(np.sum(np.log(np.diag(self.Rc))))

    def Cinv(self, V):
        return sla.cho_solve((self.Rc, True), V) if self.L.shape[1] else V[:0]

    def solve(self, V):
        """P^-1 V = sigma^-2 (V - L C^-1 L^T V)."""
        if self.L.shape[1] == 0:
            return V / self.s2
        return (V - self.L @ self.Cinv(self.L.T @ V)) / self.s2

    def dense(self):
        n = self.L.shape[0]
        return self.s2 * np.eye(n) + self.L @ self.L.T


# ----------------------------------------------------------------------------
# Random Fourier feature preconditioner P = sigma^2 I + Z Z^T (Table 1, "RFF";
# supplement S5, RFF approximation quality; Rahimi & Recht 2007), reading R-rff
# ----------------------------------------------------------------------------

def _rff_phases(X, theta, ard, freqs):
    n, d = X.shape
    ls, s, _ = split_theta(theta, d, ard)
    freqs = np.asarray(freqs, dtype=np.float64)
    if freqs.ndim != 2 or freqs.shape[1] != d:
        raise ValueError("freqs must be (m, d)")
    Xt = (X - X.mean(axis=0)) / ls
    return Xt, ls, s, Xt @ freqs.T


def rff_features(X, theta, ard, freqs, weights=None):
    """Z (n, 2m): column j is sqrt(s w_j) cos(Phi_j), column m + j is sqrt(s w_j) sin(Phi_j),
    w_j = 1/m for random features (R-rff) or the quadrature weights (R-qff)."""
    _, _, s, Phi = _rff_phases(X, theta, ard, freqs)
    a = _feature_amplitudes(s, Phi.shape[1], weights)
    return np.concatenate([a * np.cos(Phi), a * np.sin(Phi)], axis=1)


def _feature_amplitudes(s, m, weights):
    w = np.full(m, 1.0 / m) if weights is None else np.asarray(weights, dtype=np.float64)
    if w.shape != (m,):
        raise ValueError("one weight per frequency")
    return np.sqrt(s * w)


def rff_feature_derivatives(X, theta, ard, freqs, weights=None):
    """dZ/dtheta for the kernel parameters in theta order (lengthscales, then s),
    frequencies and weights held fixed: dPhi_ij/dls_q = -w_jq x~_iq / ls_q,
    d cos = -sin dPhi, d sin = cos dPhi, dZ/ds = Z / (2 s)."""
    n, d = X.shape
    Xt, ls, s, Phi = _rff_phases(X, theta, ard, freqs)
    a = _feature_amplitudes(s, Phi.shape[1], weights)
    C, S = np.cos(Phi), np.sin(Phi)
    per_dim = []
    for q in range(d):
        dPhi = -np.outer(Xt[:, q], freqs[:, q]) / ls[q]
        per_dim.append(np.concatenate([-a * S * dPhi, a * C * dPhi], axis=1))
    out = per_dim if ard else [sum(per_dim)]
    out.append(np.concatenate([a * C, a * S], axis=1) / (2.0 * s))
    return out


def qff_frequencies(d, q):
    """Quadrature Fourier features of the RBF kernel (Table 1, "QFF"; Mutny & Krause
    2018), reading R-qff: the q-point Gauss-Hermite rule of N(0, 1) (probabilists'
    Hermite nodes, weights normalised to sum 1) in every dimension, tensor product,
    one frequency of each +-pair (first coordinate among the q/2 negative nodes),
    lexicographic order, weight doubled.  Returns (freqs (q^d/2, d), weights)."""
    if q < 2 or q % 2:
        raise ValueError("q must be even")
    x, w = np.polynomial.hermite_e.hermegauss(q)
    w = w / math.sqrt(2.0 * math.pi)
    freqs, weights = [], []
    for J in itertools.product(range(q // 2), *([range(q)] * (d - 1))):
        freqs.append([x[j] for j in J])
        weights.append(2.0 * float(np.prod([w[j] for j in J])))
    return np.array(freqs, dtype=np.float64).reshape(-1, d), np.array(weights)


def precond_sqrt_apply(L, sigma2, W):
    """P^1/2 W for P = sigma^2 I + L L^T with the symmetric square root (R-sqrt):
    P^1/2 = sigma I + L V D V^T L^T with L^T L = V diag(lam) V^T and
    D = diag(1 / (sigma + sqrt(sigma^2 + lam)))."""
    sigma = math.sqrt(sigma2)
    if L.shape[1] == 0:
        return sigma * W
    lam, V = np.linalg.eigh(L.T @ L)
    lam = np.maximum(lam, 0.0)
    D = 1.0 / (sigma + np.sqrt(sigma2 + lam))
    return sigma * W + L @ (V @ (D[:, None] * (V.T @ (L.T @ W))))


# ----------------------------------------------------------------------------
# Preconditioned CG, one column at a time (R-cg), and the Lanczos tridiagonal
# ----------------------------------------------------------------------------

def pcg(matvec, b, psolve, tol, max_iters, callback=None):
    """Preconditioned CG for K_hat x = b from x0 = 0.  Returns x, the step lengths
    alpha_j, the conjugacy coefficients beta_j, rho0 = b^T P^-1 b and the final
    recurrence residual norm.  callback(x) sees every iterate."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    z = psolve(r)
    p = z.copy()
    rho = float(r @ z)
    rho0 = rho
    alphas, betas = [], []
    if bnorm == 0.0:
        return x, np.array(alphas), np.array(betas), rho0, 0.0
    for _ in range(max_iters):
        w = matvec(p)
        pw = float(p @ w)
        if not pw > 0.0:
            raise FloatingPointError("p^T K_hat p <= 0: K_hat not positive definite")
        alpha = rho / pw
        x += alpha * p
        r -= alpha * w
        alphas.append(alpha)
        if callback is not None:
            callback(x.copy())
        if np.linalg.norm(r) <= tol * bnorm:
            break
        z = psolve(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        betas.append(beta)
        p = z + beta * p
        rho = rho_new
    return x, np.array(alphas), np.array(betas), rho0, float(np.linalg.norm(r))


def pcg_block(matvec, Bmat, psolve, tol, max_iters):
    """The same recurrences as pcg, run on every column of Bmat at once: one
    product with K_hat per iteration serves all still-active columns, and a
    column that has met its tolerance is frozen.  Returns the solutions, the
    per-column (alphas, betas), rho0 and final recurrence residual norms."""
    n, t = Bmat.shape
    Xs = np.zeros_like(Bmat)
    R = Bmat.copy()
    bnorm = np.linalg.norm(Bmat, axis=0)
    Z = psolve(R)
    Pd = Z.copy()
    rho = np.einsum("ij,ij->j", R, Z)
    rho0 = rho.copy()
    alphas = [[] for _ in range(t)]
    betas = [[] for _ in range(t)]
    active = bnorm > 0.0
    for _ in range(max_iters):
        idx = np.flatnonzero(active)
        if idx.size == 0:
            break
        W = matvec(Pd[:, idx])
        pw = np.einsum("ij,ij->j", Pd[:, idx], W)
        if not np.all(pw > 0.0):
            raise FloatingPointError("p^T K_hat p <= 0: K_hat not positive definite")
        alpha = rho[idx] / pw
        Xs[:, idx] += alpha * Pd[:, idx]
        R[:, idx] -= alpha * W
        for j, c in enumerate(idx):
            alphas[c].append(alpha[j])
        done = np.linalg.norm(R[:, idx], axis=0) <= tol * bnorm[idx]
        active[idx[done]] = False
        idx = idx[~done]
        if idx.size == 0:
            break
        Zi = psolve(R[:, idx])
        rho_new = np.einsum("ij,ij->j", R[:, idx], Zi)
        beta = rho_new / rho[idx]
        for j, c in enumerate(idx):
            betas[c].append(beta[j])
        Pd[:, idx] = Zi + beta * Pd[:, idx]
        rho[idx] = rho_new
    coeffs = [(np.array(alphas[c]), np.array(betas[c])) for c in range(t)]
    return Xs, coeffs, rho0, np.linalg.norm(R, axis=0)


def lanczos_tridiag(alphas, betas):
    """Lanczos tridiagonal of the preconditioned operator from m CG steps
    (supplement S1.2, citing Saad 2003, Sec. 6.7.3):
      T_11 = 1/a_0,  T_jj = 1/a_j + b_{j-1}/a_{j-1},  T_{j,j+1} = sqrt(b_{j-1})/a_{j-1}."""
    m = len(alphas)
    diag = np.empty(m)
    off = np.empty(max(0, m - 1))
    diag[0] = 1.0 / alphas[0]
    for j in range(1, m):
        diag[j] = 1.0 / alphas[j] + betas[j - 1] / alphas[j - 1]
        off[j - 1] = math.sqrt(betas[j - 1]) / alphas[j - 1]
    return diag, off


def slq_log(alphas, betas, rho0):
    """Lanczos quadrature for b^T P^-1/2 log(P^-1/2 K P^-T/2) P^-T/2 b with nodes
    theta_j (Ritz values) and weights tau_1j^2 from the eigendecomposition of T
    (Algorithm 1, scaled by rho0 per R-probe).  Returns (gamma, #clamped)."""
    if len(alphas) == 0:
        return 0.0, 0
    diag, off = lanczos_tridiag(alphas, betas)
    if len(diag) == 1:
        lam, tau1 = diag.copy(), np.ones(1)
    else:
        # implicit QL/QR driver: the relatively robust representation driver can
        # fail to converge on Lanczos matrices with near-duplicate Ritz values
        lam, vec = sla.eigh_tridiagonal(diag, off, lapack_driver="stev")
        tau1 = vec[0, :]
    clamped = int(np.sum(lam < RITZ_FLOOR))
    lam = np.maximum(lam, RITZ_FLOOR)
    return float(rho0 * np.sum(tau1 ** 2 * np.log(lam))), clamped


# ----------------------------------------------------------------------------
# Algorithms 1 and 2 with the readings above
# ----------------------------------------------------------------------------

def _precond_terms(X, theta, kind, ard, L, piv, kp, P, Cs, mode):
    """tr(P^-1 dP/dtheta) by the matrix-inversion-lemma formula of supplement S3.3
    and the control variates c_i^T dP c_i, for every theta (R-dP)."""
    n, d = X.shape
    ls, s, s2 = split_theta(theta, d, ard)
    p = d if ard else 1
    Lk = L[:, :kp]
    ell = Cs.shape[1]
    tr = np.zeros(p + 2)
    ctrl = np.zeros((p + 2, ell))
    # noise: dP/dsigma^2 = I
    LCinv = P.Cinv(Lk.T).T if kp else np.zeros((n, 0))          # L C^-1
    tr[p + 1] = (n - np.sum(LCinv * Lk)) / s2
    ctrl[p + 1] = np.sum(Cs * Cs, axis=0)
    if kp == 0:
        return tr, ctrl
    LS = Lk[piv[:kp], :]                                          # lower triangular
    dcols = dkernel_cols(X, theta, kind, ard, piv[:kp])           # dK[:, S] per kernel theta
    LtC = Lk.T @ Cs
    LtL = Lk.T @ Lk
    for idx, dKS in enumerate(dcols):
        if mode == 1 and idx < p:
            continue
        E = sla.solve_triangular(LS, dKS.T, lower=True).T        # dK_{:S} L_S^-T
        F = sla.solve_triangular(LS, sla.solve_triangular(LS, dKS[piv[:kp], :].T, lower=True).T,
                                 lower=True)                     # L_S^-1 dK_SS L_S^-T
        F = 0.5 * (F + F.T)
        diag_dP = 2.0 * np.sum(E * Lk, axis=1) - np.sum((Lk @ F) * Lk, axis=1)
        dP_L = E @ LtL + Lk @ (E.T @ Lk) - Lk @ (F @ LtL)
        tr[idx] = (np.sum(diag_dP) - np.sum(LCinv * dP_L)) / s2
        EtC = E.T @ Cs
        ctrl[idx] = 2.0 * np.sum(LtC * EtC, axis=0) - np.sum(LtC * (F @ LtC), axis=0)
    return tr, ctrl


def _precond_terms_rff(X, theta, ard, freqs, Z, P, Cs, mode, weights=None):
    """tr(P^-1 dP/dtheta) and the control variates c_i^T dP c_i for the RFF
    preconditioner, dP = dZ Z^T + Z dZ^T, with P^-1 = sigma^-2 (I - Z C^-1 Z^T)
    (matrix inversion lemma, as in supplement S3.3)."""
    n, d = X.shape
    _, _, s2 = split_theta(theta, d, ard)
    p = d if ard else 1
    ell = Cs.shape[1]
    tr = np.zeros(p + 2)
    ctrl = np.zeros((p + 2, ell))
    ZCinv = P.Cinv(Z.T).T
    tr[p + 1] = (n - np.sum(ZCinv * Z)) / s2
    ctrl[p + 1] = np.sum(Cs * Cs, axis=0)
    ZtC = Z.T @ Cs
    ZtZ = Z.T @ Z
    for idx, dZ in enumerate(rff_feature_derivatives(X, theta, ard, freqs, weights)):
        if mode == 1 and idx < p:
            continue
        dP_Z = dZ @ ZtZ + Z @ (dZ.T @ Z)                         # dP Z
        tr[idx] = (2.0 * np.sum(dZ * Z) - np.sum(ZCinv * dP_Z)) / s2
        ctrl[idx] = 2.0 * np.sum(ZtC * (dZ.T @ Cs), axis=0)
    return tr, ctrl


def estimate_mll(X, y, theta, kind, ard, rank, num_probes, tol, max_iters, seed,
                 grad=True, precond_grad=0, signs=None, dense=None, precond="pivchol", freqs=None,
                 landmarks=None, qff_nodes=None, probe_mode=0, workers=1, native=False):
    """Preconditioned estimate of log p (Algorithm 1) and, if grad, of its
    derivative (Algorithm 2) under the readings in the module docstring.

    signs: optional (E, H) Rademacher arrays of shapes (n, ell), (rank, ell)
    replacing the SplitMix64 stream.  dense: force (True) or forbid (False) a
    dense K_hat; default dense for n <= 20000.  precond: "pivchol" (partial
    pivoted Cholesky of the given rank) or "rff" (R-rff; freqs (rank/2, d)).
    workers: threads over the row blocks of the matrix-free products; native: run
    the matrix-free products by the plain-C loops of khat_native.c."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, d = X.shape
    ls, s, s2 = split_theta(theta, d, ard)
    if dense is None:
        dense = n <= 20000
    Kh = khat_dense(X, theta, kind, ard) if dense else None

    def matvec(V):
        return Kh @ V if dense else khat_matvec(X, theta, kind, ard, V, workers=workers, native=native)

    # preconditioner (pivoted Cholesky or random Fourier features) and log det P
    weights = None
    if precond == "qff":
        if kind != "rbf":
            raise ValueError("quadrature Fourier features are built for the RBF kernel")
        freqs, weights = qff_frequencies(d, qff_nodes)
        if 2 * len(freqs) != rank:
            raise ValueError("the QFF preconditioner has rank q^d")
    if precond in ("rff", "qff"):
        if freqs is None or 2 * len(freqs) != rank:
            raise ValueError("the RFF preconditioner needs rank / 2 frequency rows")
        L = rff_features(X, theta, ard, freqs, weights)
        piv, kp = np.full(rank, -1, dtype=np.int64), rank
    elif precond == "nystrom":
        L, piv, kp = pivoted_cholesky(X, theta, kind, ard, rank, order=landmarks)
    elif precond == "pivchol":
        L, piv, kp = pivoted_cholesky(X, theta, kind, ard, rank)
    else:
        raise ValueError(precond)
    P = Preconditioner(L[:, :kp], s2)

    # probes b_i = sigma eps_i + L eta_i (R-probe), or P^1/2 w_i (R-sqrt)
    if signs is None:
        E, H = probe_signs(seed, n, rank, num_probes)
    else:
        E, H = signs
    ell = E.shape[1]
    if probe_mode == 1:
        B = precond_sqrt_apply(L[:, :kp], s2, E)
    else:
        B = math.sqrt(s2) * E + L @ H[:rank] if rank else math.sqrt(s2) * E
    rhs = np.concatenate([y[:, None], B], axis=1)

    # one CG call over all right hand sides (footnote to Section 4.4)
    t = rhs.shape[1]
    Xs, coeffs, rho0, resid = pcg_block(matvec, rhs, P.solve, tol, max_iters)
    iters = np.array([len(a) for a, _ in coeffs], dtype=np.int64)

    gammas = np.zeros(ell)
    clamped = 0
    for i in range(ell):
        a, b = coeffs[i + 1]
        gammas[i], cl = slq_log(a, b, rho0[i + 1])
        clamped += cl
    u = Xs[:, 0]
    datafit = float(y @ u)
    logdet_est = P.logdet + (gammas.mean() if ell else 0.0)
    logp = -0.5 * (datafit + logdet_est + n * LOG2PI)
    out = {"logp": logp, "datafit": datafit, "logdet_est": logdet_est, "logdet_P": P.logdet,
           "gammas": gammas, "rho0": rho0, "iters": iters, "coeffs": coeffs, "L": L,
           "piv": piv, "rank": kp, "solves": Xs, "B": B, "rel_resid": resid / np.maximum(
               np.linalg.norm(rhs, axis=0), 1e-300), "ritz_clamped": clamped}
    if not grad:
        return out

    # derivative (Algorithm 2, R-grad): M = A' C'^T with A' = [u | a_i],
    # C' = [u/2 | -c_i/(2 ell)]; c_i = P^-1 b_i
    Cs = P.solve(B)
    A1 = Xs
    C1 = np.concatenate([0.5 * u[:, None], -Cs / (2.0 * ell)], axis=1)
    if native and not dense:
        bil = dkhat_contract_lowrank(X, theta, kind, ard, A1, C1)
    else:
        bil = dkhat_contract(X, theta, kind, ard, lambda r: A1[r] @ C1.T, workers=workers)
    if precond in ("rff", "qff"):
        tr, ctrl = _precond_terms_rff(X, theta, ard, freqs, L, P, Cs, precond_grad, weights)
    else:
        tr, ctrl = _precond_terms(X, theta, kind, ard, L, piv, kp, P, Cs, precond_grad)
    g = bil - 0.5 * tr + ctrl.sum(axis=1) / (2.0 * ell)
    out.update({"grad": g, "bilinear": bil, "tr_precond": tr, "ctrl": ctrl, "precond_solves": Cs})
    return out
