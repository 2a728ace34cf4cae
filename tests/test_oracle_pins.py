"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: an
exact rational determinant, finite differences, a library routine for a special
case, an exact expectation over every Rademacher pattern, a closed-form variance,
or a convergence bound stated in the paper.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as sps
from scipy.spatial.distance import cdist

from oracle import gp_oracle as go
import synthgp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(n, d, kind="rbf", ard=True, seed=0, sigma2=0.05, ls=(0.4, 1.2), dist="uniform"):
    pr = synthgp.random_problem(n, d, kind, ard, seed=seed, sigma2=sigma2, ls_range=ls, dist=dist)
    return pr.X, pr.y, pr.theta


# ---------------------------------------------------------------- generator

def test_splitmix64_matches_reference_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = [int(go.splitmix64(0, i)) for i in range(len(vals))]
    assert got == vals


def test_rademacher_is_balanced_and_stream_separated():
    e = go.rademacher(7, 0, 3, 200000)
    assert set(np.unique(e)) == {-1.0, 1.0}
    assert abs(e.mean()) < 4.0 / math.sqrt(e.size)
    h = go.rademacher(7, 1, 3, 200000)
    assert abs(np.mean(e * h)) < 4.0 / math.sqrt(e.size)


# ---------------------------------------------------------------- kernels

def test_sqdist_matches_scipy_cdist():
    rng = np.random.default_rng(3)
    X1, X2 = rng.standard_normal((17, 5)), rng.standard_normal((9, 5))
    ls = np.array([0.5, 1.0, 2.0, 0.7, 1.3])
    np.testing.assert_allclose(go.sqdist(X1, X2, ls), cdist(X1 / ls, X2 / ls, "sqeuclidean"),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind,nu", [("matern32", 1.5), ("matern52", 2.5)])
def test_matern_closed_forms_match_bessel_definition(kind, nu):
    # Matern-nu: 2^(1-nu)/Gamma(nu) (sqrt(2 nu) r)^nu K_nu(sqrt(2 nu) r)
    r = np.linspace(1e-3, 6.0, 400)
    z = math.sqrt(2 * nu) * r
    ref = 2 ** (1 - nu) / sps.gamma(nu) * z ** nu * sps.kv(nu, z)
    np.testing.assert_allclose(go.kappa(kind, r * r), ref, rtol=1e-12, atol=1e-15)


def test_rbf_is_matern_limit():
    # Matern-nu -> RBF as nu -> infinity; nu = 60 agrees to ~1e-2 near r = 1
    r = np.linspace(0.05, 2.0, 50)
    nu = 60.0
    z = math.sqrt(2 * nu) * r
    mat = np.exp((1 - nu) * math.log(2) - sps.gammaln(nu) + nu * np.log(z)) * sps.kve(nu, z) * np.exp(-z)
    np.testing.assert_allclose(go.kappa("rbf", r * r), mat, rtol=2e-2)


@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52", "ratquad:0.8"])
@pytest.mark.parametrize("ard", [True, False])
def test_kernel_derivative_entries_match_finite_differences(kind, ard):
    X, _, theta = _problem(12, 3, kind, ard, seed=1)
    cols = np.array([0, 4, 7])
    mats = go.dkernel_cols(X, theta, kind, ard, cols)
    p = len(theta) - 2
    for i in range(p + 1):
        h = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (go.kernel_matrix(X, X[cols], tp, kind, ard) - go.kernel_matrix(X, X[cols], tm, kind, ard)) / (2 * h)
        np.testing.assert_allclose(mats[i], fd, rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------- exact targets

def test_cholesky_logdet_matches_exact_rational_determinant():
    X, y, theta = _problem(7, 2, "rbf", True, seed=2, sigma2=0.3)
    Kh = go.khat_dense(X, theta, "rbf", True)
    det = go.bareiss_det(Kh.tolist())
    assert det > 0
    exact_logdet = math.log(det.numerator) - math.log(det.denominator)
    got = go.exact_mll(X, y, theta, "rbf", True)["logdet"]
    assert abs(got - exact_logdet) <= 1e-13 * max(1.0, abs(exact_logdet))
    assert abs(np.linalg.slogdet(Kh)[1] - exact_logdet) <= 1e-12 * max(1.0, abs(exact_logdet))


def test_exact_solve_residual():
    X, y, theta = _problem(300, 3, "matern32", True, seed=3, sigma2=0.01)
    ex = go.exact_mll(X, y, theta, "matern32", True)
    Kh = go.khat_dense(X, theta, "matern32", True)
    assert np.linalg.norm(Kh @ ex["u"] - y) / np.linalg.norm(y) <= 1e-12


@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52"])
@pytest.mark.parametrize("ard", [True, False])
def test_exact_gradient_matches_central_differences(kind, ard):
    X, y, theta = _problem(40, 3, kind, ard, seed=4, sigma2=0.05)
    g = go.exact_mll(X, y, theta, kind, ard)["grad"]
    for i in range(len(theta)):
        h = 1e-5 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (go.exact_mll(X, y, tp, kind, ard)["logp"] - go.exact_mll(X, y, tm, kind, ard)["logp"]) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


# ---------------------------------------------------------------- preconditioner

def test_pivoted_cholesky_is_nystrom_on_its_pivots():
    X, _, theta = _problem(80, 2, "matern52", True, seed=5)
    L, piv, kp = go.pivoted_cholesky(X, theta, "matern52", True, 12)
    assert kp == 12 and len(set(piv.tolist())) == 12
    K = go.kernel_matrix(X, X, theta, "matern52", True)
    KS = K[:, piv]
    ny = KS @ np.linalg.solve(K[np.ix_(piv, piv)], KS.T)
    np.testing.assert_allclose(L @ L.T, ny, atol=1e-10)
    # L restricted to the pivot rows, in pivot order, is lower triangular
    LS = L[piv, :]
    assert np.all(np.triu(LS, 1) == 0.0)
    # residual diagonal stays non-negative
    assert np.min(np.diag(K - L @ L.T)) >= -1e-12


def test_pivoted_cholesky_trace_decreases_and_full_rank_reproduces_K():
    X, _, theta = _problem(30, 2, "rbf", True, seed=6, ls=(0.05, 0.1))
    K = go.kernel_matrix(X, X, theta, "rbf", True)
    traces = []
    for k in range(0, 31, 3):
        L, piv, kp = go.pivoted_cholesky(X, theta, "rbf", True, k)
        traces.append(np.trace(K - L @ L.T))
    assert all(b <= a + 1e-12 for a, b in zip(traces, traces[1:]))
    L, piv, kp = go.pivoted_cholesky(X, theta, "rbf", True, 30)
    assert kp == 30
    np.testing.assert_allclose(L @ L.T, K, atol=1e-10)


def test_pivoted_cholesky_rbf_1d_decays_exponentially():
    # supplement S5.3 (Cholesky approximation quality): exponential decay for a 1-D RBF kernel
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, size=(400, 1))
    theta = np.array([0.3, 1.0, 0.01])
    K = go.kernel_matrix(X, X, theta, "rbf", False)
    res = []
    for k in (2, 4, 6, 8, 10, 12):
        L, _, _ = go.pivoted_cholesky(X, theta, "rbf", False, k)
        res.append(np.trace(K - L @ L.T))
    ratios = [b / a for a, b in zip(res, res[1:])]
    assert max(ratios) < 0.1          # at least a factor 10 per two extra columns
    assert res[-1] < 1e-8 * res[0]


def test_pivot_breakdown_on_duplicate_points():
    X = np.repeat(np.array([[0.1, 0.2], [0.5, 0.9], [0.8, 0.3]]), 4, axis=0)
    theta = np.array([0.5, 1.0, 0.1])
    L, piv, kp = go.pivoted_cholesky(X, theta, "rbf", False, 6)
    assert kp == 3
    assert np.all(L[:, 3:] == 0.0)


def test_woodbury_solve_and_determinant_lemma():
    X, _, theta = _problem(60, 3, "rbf", True, seed=8, sigma2=0.02)
    L, _, kp = go.pivoted_cholesky(X, theta, "rbf", True, 9)
    P = go.Preconditioner(L, 0.02)
    Pd = P.dense()
    assert abs(P.logdet - np.linalg.slogdet(Pd)[1]) <= 1e-12 * abs(P.logdet)
    V = np.random.default_rng(1).standard_normal((60, 4))
    np.testing.assert_allclose(P.solve(V), np.linalg.solve(Pd, V), rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------- CG and Lanczos

def _tiny_system(n=30, seed=9, k=4, sigma2=0.05):
    X, _, theta = _problem(n, 2, "matern32", True, seed=seed, sigma2=sigma2)
    Kh = go.khat_dense(X, theta, "matern32", True)
    L, _, _ = go.pivoted_cholesky(X, theta, "matern32", True, k)
    return X, theta, Kh, go.Preconditioner(L, sigma2)


def test_pcg_converges_in_n_steps_and_obeys_theorem_s1():
    X, theta, Kh, P = _tiny_system()
    n = Kh.shape[0]
    Pd = P.dense()
    lam = sla.eigh(Kh, Pd, eigvals_only=True)
    kappa = lam.max() / lam.min()
    assert kappa < 1e3
    b = np.random.default_rng(0).standard_normal(n)
    xs = np.linalg.solve(Kh, b)
    rate = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    e0 = math.sqrt(xs @ Kh @ xs)
    iterates = []
    x, a, bb, rho0, _ = go.pcg(lambda v: Kh @ v, b.copy(), P.solve, 0.0, n, callback=iterates.append)
    assert len(a) == n
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-9
    for m, xm in enumerate(iterates, start=1):
        err = math.sqrt((xm - xs) @ Kh @ (xm - xs))
        assert err <= 2.0 * rate ** m * e0 * (1 + 1e-8) + 1e-12


def test_pcg_block_matches_single_column_pcg():
    X, theta, Kh, P = _tiny_system(n=40, seed=10)
    Bm = np.random.default_rng(2).standard_normal((40, 5))
    Xs, coeffs, rho0, _ = go.pcg_block(lambda V: Kh @ V, Bm, P.solve, 1e-9, 100)
    for c in range(5):
        x, a, b, r0, _ = go.pcg(lambda v: Kh @ v, Bm[:, c].copy(), P.solve, 1e-9, 100)
        # late CG coefficients amplify rounding differences (matrix-matrix vs
        # matrix-vector products); the early ones, the solution and the
        # quadrature value are stable
        assert abs(len(a) - len(coeffs[c][0])) <= 2
        np.testing.assert_allclose(Xs[:, c], x, rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(coeffs[c][0][:8], a[:8], rtol=1e-9)
        np.testing.assert_allclose(coeffs[c][1][:8], b[:8], rtol=1e-9)
        assert abs(rho0[c] - r0) <= 1e-12 * abs(r0)
        g1, _ = go.slq_log(coeffs[c][0], coeffs[c][1], rho0[c])
        g2, _ = go.slq_log(a, b, r0)
        assert abs(g1 - g2) <= 1e-7 * max(1.0, abs(g2))


def test_gauss_quadrature_moment_identity():
    # the m-point Lanczos (Gauss) rule from the CG coefficients integrates
    # polynomials of degree <= 2m-1 exactly: rho0 e1^T T^p e1 = b^T (P^-1 K)^p P^-1 b
    X, theta, Kh, P = _tiny_system(n=30, seed=11)
    b = np.random.default_rng(3).standard_normal(30)
    m = 5
    _, a, bb, rho0, _ = go.pcg(lambda v: Kh @ v, b.copy(), P.solve, 0.0, m)
    diag, off = go.lanczos_tridiag(a, bb)
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    v = P.solve(b)
    for p in range(2 * m):
        lhs = rho0 * np.linalg.matrix_power(T, p)[0, 0]
        rhs = b @ v
        assert abs(lhs - rhs) <= 1e-10 * abs(rhs), (p, lhs, rhs)
        v = P.solve(Kh @ v)


def test_slq_is_exact_when_m_equals_n():
    X, theta, Kh, P = _tiny_system(n=12, seed=12, k=3)
    b = np.random.default_rng(4).standard_normal(12)
    _, a, bb, rho0, _ = go.pcg(lambda v: Kh @ v, b.copy(), P.solve, 0.0, 12)
    gamma, clamped = go.slq_log(a, bb, rho0)
    w, V = np.linalg.eigh(P.dense())
    Pmh = V @ np.diag(w ** -0.5) @ V.T
    lam, Q = np.linalg.eigh(Pmh @ Kh @ Pmh)
    ref = b @ Pmh @ (Q @ np.diag(np.log(lam)) @ Q.T) @ Pmh @ b
    assert clamped == 0
    assert abs(gamma - ref) <= 1e-8 * max(1.0, abs(ref))


# ---------------------------------------------------------------- estimator special cases

def test_perfect_preconditioner_gives_exact_results_with_zero_variance():
    # k = n: P = K_hat, CG stops after one step, every gamma is 0 (Theorem 1 with g = 0)
    X, y, theta = _problem(10, 2, "rbf", True, seed=13, sigma2=0.2, ls=(0.05, 0.1))
    ex = go.exact_mll(X, y, theta, "rbf", True)
    for seed in (1, 2):
        es = go.estimate_mll(X, y, theta, "rbf", True, 10, 4, 1e-10, 50, seed)
        assert es["rank"] == 10
        assert np.all(es["iters"] == 1)
        assert np.max(np.abs(es["gammas"])) <= 1e-10
        assert abs(es["logp"] - ex["logp"]) <= 1e-10 * abs(ex["logp"])
        np.testing.assert_allclose(es["grad"], ex["grad"], rtol=1e-8, atol=1e-9)


def test_no_preconditioner_reduces_to_hutchinson_slq():
    X, y, theta = _problem(14, 2, "matern52", True, seed=14, sigma2=0.1)
    n = 14
    es = go.estimate_mll(X, y, theta, "matern52", True, 0, 6, 0.0, n, seed=5, grad=False)
    Kh = go.khat_dense(X, theta, "matern52", True)
    lam, Q = np.linalg.eigh(Kh)
    logK = Q @ np.diag(np.log(lam)) @ Q.T
    E, _ = go.probe_signs(5, n, 0, 6)
    hutch = np.mean([E[:, i] @ logK @ E[:, i] for i in range(6)])
    assert abs(es["logdet_est"] - hutch) <= 1e-8 * abs(hutch)


def _enumerate_estimates(X, y, theta, kind, ard, k, precond_grad=0):
    n = X.shape[0]
    vals, grads = [], []
    for bits in itertools.product((-1.0, 1.0), repeat=n + k):
        xi = np.array(bits)
        E = xi[:n, None]
        H = xi[n:, None]
        es = go.estimate_mll(X, y, theta, kind, ard, k, 1, 1e-13, n, 0,
                             grad=True, precond_grad=precond_grad, signs=(E, H))
        vals.append(es["logdet_est"])
        grads.append(es["grad"])
    return np.array(vals), np.array(grads), es


@pytest.mark.parametrize("precond_grad", [0, 1])
def test_estimators_are_unbiased_over_all_sign_patterns(precond_grad):
    # exact expectation over every Rademacher pattern (n + k = 9 signs)
    X, y, theta = _problem(7, 2, "rbf", True, seed=15, sigma2=0.1, ls=(0.3, 0.6))
    vals, grads, es = _enumerate_estimates(X, y, theta, "rbf", True, 2, precond_grad)
    ex = go.exact_mll(X, y, theta, "rbf", True)
    assert abs(vals.mean() - ex["logdet"]) <= 1e-9 * abs(ex["logdet"])
    np.testing.assert_allclose(grads.mean(axis=0), ex["grad"], rtol=1e-8, atol=1e-9)
    # not trivially exact per pattern
    assert vals.std() > 1e-6


def test_logdet_estimator_variance_matches_rademacher_closed_form():
    # gamma = xi^T A xi with A = R^T M R, R = [sigma I, L], M = P^-1/2 log(A~) P^-1/2;
    # Var over Rademacher xi of xi^T A xi = 2 (||A_s||_F^2 - sum_i (A_s)_ii^2)
    X, y, theta = _problem(7, 2, "rbf", True, seed=16, sigma2=0.1, ls=(0.3, 0.6))
    vals, _, es = _enumerate_estimates(X, y, theta, "rbf", True, 2)
    n, k = 7, 2
    L = es["L"]
    Pd = 0.1 * np.eye(n) + L @ L.T
    w, V = np.linalg.eigh(Pd)
    Pmh = V @ np.diag(w ** -0.5) @ V.T
    Kh = go.khat_dense(X, theta, "rbf", True)
    lam, Q = np.linalg.eigh(Pmh @ Kh @ Pmh)
    M = Pmh @ Q @ np.diag(np.log(lam)) @ Q.T @ Pmh
    R = np.concatenate([math.sqrt(0.1) * np.eye(n), L], axis=1)
    A = R.T @ M @ R
    As = 0.5 * (A + A.T)
    var = 2.0 * (np.sum(As ** 2) - np.sum(np.diag(As) ** 2))
    assert abs(vals.var() - var) <= 1e-8 * var


@pytest.mark.parametrize("mode", [0, 1])
def test_precond_trace_and_control_variates_match_dense_finite_differences(mode):
    X, y, theta = _problem(25, 2, "matern32", True, seed=17, sigma2=0.05)
    kind, ard, k = "matern32", True, 6
    L, piv, kp = go.pivoted_cholesky(X, theta, kind, ard, k)
    P = go.Preconditioner(L[:, :kp], 0.05)
    Cs = np.random.default_rng(5).standard_normal((25, 3))
    tr, ctrl = go._precond_terms(X, theta, kind, ard, L, piv, kp, P, Cs, mode)

    def nystrom(th):
        K = go.kernel_matrix(X, X, th, kind, ard)
        KS = K[:, piv]
        return KS @ np.linalg.solve(K[np.ix_(piv, piv)], KS.T)

    Pd = P.dense()
    p = len(theta) - 2
    for i in range(len(theta)):
        if i == p + 1:
            dP = np.eye(25)
        elif mode == 1 and i < p:
            dP = np.zeros((25, 25))
        else:
            h = 1e-6 * theta[i]
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            dP = (nystrom(tp) - nystrom(tm)) / (2 * h)
        ref_tr = np.trace(np.linalg.solve(Pd, dP))
        ref_ctrl = np.einsum("pi,pq,qi->i", Cs, dP, Cs)
        assert abs(tr[i] - ref_tr) <= 1e-6 * max(1.0, abs(ref_tr)), (i, tr[i], ref_tr)
        np.testing.assert_allclose(ctrl[i], ref_ctrl, rtol=1e-6, atol=1e-8)


def test_preconditioning_cuts_variance_as_in_table_s1():
    # trend pin (Table S1, RBF, d = 1): with a preconditioner of the probe count's
    # size, bias and variance of the log-likelihood estimate drop by orders of
    # magnitude against plain Hutchinson.  Smaller n and ell than the paper's.
    rng = np.random.default_rng(18)
    n = 600
    X = rng.standard_normal((n, 1))
    theta = np.array([1.0, 1.0, 1e-2])
    y = synthgp.rff_targets(rng, X, 1.0, 1.0, 1e-2, "rbf")
    ex = go.exact_mll(X, y, theta, "rbf", False)
    res = {}
    for k in (0, 16):
        vals = [go.estimate_mll(X, y, theta, "rbf", False, k, 16, 1e-10, 600, seed, grad=False)["logp"]
                for seed in range(10)]
        res[k] = (abs(np.mean(vals) - ex["logp"]) / abs(ex["logp"]), np.var(vals))
    assert res[16][1] < 1e-3 * res[0][1]
    assert res[16][0] < 1e-2 * res[0][0] + 1e-12


# ------------------------------------------------ random Fourier features (Table 1)

def test_rff_gram_is_the_shift_invariant_cosine_sum():
    X, _, theta = _problem(20, 3, "rbf", True, seed=21)
    W = synthgp.spectral_frequencies("rbf", 7, 3, seed=3)
    Z = go.rff_features(X, theta, True, W)
    ls, s = theta[:3], theta[3]
    D = (X[:, None, :] - X[None, :, :]) / ls              # direct differences
    ref = (s / 7) * np.cos(np.einsum("abq,jq->abj", D, W)).sum(axis=2)
    np.testing.assert_allclose(Z @ Z.T, ref, rtol=0, atol=1e-13)
    # the origin of the phases is invisible in Z Z^T
    Z2 = go.rff_features(X + 3.7, theta, True, W)
    np.testing.assert_allclose(Z2 @ Z2.T, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52"])
def test_rff_gram_approaches_the_kernel(kind):
    # Monte Carlo over the spectral density: each entry of Z Z^T averages m
    # cosines (variance <= s^2 / (2m)); 40,000 features bound every entry well
    # inside 0.03 s, while a wrong density (scale, degrees of freedom) misses by
    # far more
    X, _, theta = _problem(30, 3, kind, True, seed=22, ls=(0.5, 1.5))
    W = synthgp.spectral_frequencies(kind, 40000, 3, seed=4)
    Z = go.rff_features(X, theta, True, W)
    K = go.kernel_matrix(X, X, theta, kind, True)
    assert np.max(np.abs(Z @ Z.T - K)) < 0.03 * theta[3]


@pytest.mark.parametrize("ard", [True, False])
def test_rff_feature_derivatives_match_finite_differences(ard):
    X, _, theta = _problem(15, 3, "matern32", ard, seed=23)
    W = synthgp.spectral_frequencies("matern32", 5, 3, seed=5)
    dZ = go.rff_feature_derivatives(X, theta, ard, W)
    assert len(dZ) == len(theta) - 1
    for i in range(len(theta) - 1):
        h = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (go.rff_features(X, tp, ard, W) - go.rff_features(X, tm, ard, W)) / (2 * h)
        np.testing.assert_allclose(dZ[i], fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("mode", [0, 1])
def test_rff_precond_trace_and_control_variates_match_dense_finite_differences(mode):
    # tr(P^-1 dP) = d log det P (Jacobi's formula) and c^T dP c = d (c^T P c), both
    # by central differences of the dense P with the frequencies held fixed
    X, _, theta = _problem(25, 2, "rbf", True, seed=24, sigma2=0.05)
    W = synthgp.spectral_frequencies("rbf", 4, 2, seed=6)
    Z = go.rff_features(X, theta, True, W)
    P = go.Preconditioner(Z, 0.05)
    Cs = np.random.default_rng(7).standard_normal((25, 3))
    tr, ctrl = go._precond_terms_rff(X, theta, True, W, Z, P, Cs, mode)

    def dense_P(th):
        Zt = go.rff_features(X, th, True, W)
        return th[-1] * np.eye(25) + Zt @ Zt.T

    p = len(theta) - 2
    for i in range(len(theta)):
        if mode == 1 and i < p:
            assert tr[i] == 0.0 and np.all(ctrl[i] == 0.0)
            continue
        h = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Pp, Pm = dense_P(tp), dense_P(tm)
        ref_tr = (np.linalg.slogdet(Pp)[1] - np.linalg.slogdet(Pm)[1]) / (2 * h)
        ref_ctrl = (np.einsum("pi,pq,qi->i", Cs, Pp, Cs) - np.einsum("pi,pq,qi->i", Cs, Pm, Cs)) / (2 * h)
        assert abs(tr[i] - ref_tr) <= 1e-6 * max(1.0, abs(ref_tr)), (i, tr[i], ref_tr)
        np.testing.assert_allclose(ctrl[i], ref_ctrl, rtol=1e-6, atol=1e-6)


def test_rff_estimators_are_unbiased_over_all_sign_patterns():
    # exact expectation over every Rademacher pattern (n + k = 9 signs), RFF rank 2
    X, y, theta = _problem(7, 2, "matern52", True, seed=25, sigma2=0.1, ls=(0.3, 0.6))
    W = synthgp.spectral_frequencies("matern52", 1, 2, seed=8)
    n, k = 7, 2
    vals, grads = [], []
    for bits in itertools.product((-1.0, 1.0), repeat=n + k):
        xi = np.array(bits)
        es = go.estimate_mll(X, y, theta, "matern52", True, k, 1, 1e-13, n, 0, grad=True,
                             signs=(xi[:n, None], xi[n:, None]), precond="rff", freqs=W)
        vals.append(es["logdet_est"])
        grads.append(es["grad"])
    vals, grads = np.array(vals), np.array(grads)
    ex = go.exact_mll(X, y, theta, "matern52", True)
    assert abs(vals.mean() - ex["logdet"]) <= 1e-9 * abs(ex["logdet"])
    np.testing.assert_allclose(grads.mean(axis=0), ex["grad"], rtol=1e-8, atol=1e-9)
    assert vals.std() > 1e-6
    assert es["rank"] == 2 and np.all(es["piv"] == -1)


# ------------------------------------------------ randomized Nystrom (Table 1)

def test_nystrom_landmarks_reproduce_the_nystrom_formula():
    X, _, theta = _problem(40, 3, "matern52", True, seed=26)
    S = synthgp.uniform_landmarks(40, 9, seed=1)
    L, piv, kp = go.pivoted_cholesky(X, theta, "matern52", True, 9, order=S)
    assert kp == 9 and list(piv) == list(S)
    K = go.kernel_matrix(X, X, theta, "matern52", True)
    KS = K[:, S]
    np.testing.assert_allclose(L @ L.T, KS @ np.linalg.solve(K[np.ix_(S, S)], KS.T), rtol=0, atol=1e-12)
    LS = L[S, :]
    np.testing.assert_allclose(LS, np.tril(LS), atol=0)
    np.testing.assert_allclose(LS, np.linalg.cholesky(K[np.ix_(S, S)]), rtol=1e-12, atol=1e-14)


def test_nystrom_landmarks_stop_on_a_duplicate_point():
    X, _, theta = _problem(12, 2, "rbf", True, seed=27)
    X[5] = X[2]
    L, piv, kp = go.pivoted_cholesky(X, theta, "rbf", True, 4, order=[2, 5, 7, 9])
    assert kp == 1 and list(piv) == [2]
    assert np.all(L[:, 1:] == 0.0)


def test_nystrom_precond_terms_match_dense_finite_differences():
    X, y, theta = _problem(25, 2, "matern32", True, seed=28, sigma2=0.05)
    S = synthgp.uniform_landmarks(25, 5, seed=2)
    L, piv, kp = go.pivoted_cholesky(X, theta, "matern32", True, 5, order=S)
    P = go.Preconditioner(L[:, :kp], 0.05)
    Cs = np.random.default_rng(9).standard_normal((25, 3))
    tr, ctrl = go._precond_terms(X, theta, "matern32", True, L, piv, kp, P, Cs, 0)

    def dense_P(th):
        K = go.kernel_matrix(X, X, th, "matern32", True)
        KS = K[:, S]
        return th[-1] * np.eye(25) + KS @ np.linalg.solve(K[np.ix_(S, S)], KS.T)

    for i in range(len(theta)):
        h = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Pp, Pm = dense_P(tp), dense_P(tm)
        ref_tr = (np.linalg.slogdet(Pp)[1] - np.linalg.slogdet(Pm)[1]) / (2 * h)
        ref_ctrl = (np.einsum("pi,pq,qi->i", Cs, Pp, Cs) - np.einsum("pi,pq,qi->i", Cs, Pm, Cs)) / (2 * h)
        assert abs(tr[i] - ref_tr) <= 1e-6 * max(1.0, abs(ref_tr)), (i, tr[i], ref_tr)
        np.testing.assert_allclose(ctrl[i], ref_ctrl, rtol=1e-6, atol=1e-6)


def test_nystrom_estimators_are_unbiased_over_all_sign_patterns():
    X, y, theta = _problem(7, 2, "rbf", True, seed=29, sigma2=0.1, ls=(0.3, 0.6))
    S = np.array([4, 1], dtype=np.int32)
    n, k = 7, 2
    vals, grads = [], []
    for bits in itertools.product((-1.0, 1.0), repeat=n + k):
        xi = np.array(bits)
        es = go.estimate_mll(X, y, theta, "rbf", True, k, 1, 1e-13, n, 0, grad=True,
                             signs=(xi[:n, None], xi[n:, None]), precond="nystrom", landmarks=S)
        vals.append(es["logdet_est"])
        grads.append(es["grad"])
    vals, grads = np.array(vals), np.array(grads)
    ex = go.exact_mll(X, y, theta, "rbf", True)
    assert abs(vals.mean() - ex["logdet"]) <= 1e-9 * abs(ex["logdet"])
    np.testing.assert_allclose(grads.mean(axis=0), ex["grad"], rtol=1e-8, atol=1e-9)
    assert list(es["piv"]) == [4, 1]


# ------------------------------------------------ quadrature Fourier features (Table 1)

def test_qff_rule_integrates_gaussian_moments_exactly():
    # a q-point Gauss rule integrates polynomials up to degree 2q - 1 exactly:
    # E[w^2k] = (2k - 1)!! for the standard normal; degree 2q is not exact
    q = 6
    f, wt = go.qff_frequencies(1, q)
    x = np.concatenate([f[:, 0], -f[:, 0]])
    v = np.concatenate([wt, wt]) / 2.0
    assert abs(v.sum() - 1.0) < 1e-14
    for k in range(1, q):
        dfact = float(np.prod(np.arange(2 * k - 1, 0, -2)))
        assert abs(np.sum(v * x ** (2 * k)) - dfact) <= 1e-12 * dfact
    assert abs(np.sum(v * x ** (2 * q)) - float(np.prod(np.arange(2 * q - 1, 0, -2)))) > 1.0
    # every frequency of the half grid has its first coordinate negative (one of each pair)
    f2, w2 = go.qff_frequencies(3, 4)
    assert f2.shape == (32, 3) and np.all(f2[:, 0] < 0) and abs(w2.sum() - 1.0) < 1e-14


def test_qff_gram_converges_exponentially_to_the_rbf_kernel():
    X, _, theta = _problem(30, 2, "rbf", True, seed=40, ls=(0.5, 1.5))
    K = go.kernel_matrix(X, X, theta, "rbf", True)
    errs = []
    for q in (2, 4, 8, 12):
        f, w = go.qff_frequencies(2, q)
        Z = go.rff_features(X, theta, True, f, w)
        assert Z.shape == (30, q * q)
        errs.append(np.max(np.abs(Z @ Z.T - K)))
    assert errs[0] > 1e2 * errs[1] and errs[1] > 1e5 * errs[2]
    assert errs[3] < 1e-12


def test_qff_precond_terms_match_dense_finite_differences():
    X, _, theta = _problem(25, 2, "rbf", True, seed=41, sigma2=0.05)
    f, w = go.qff_frequencies(2, 4)
    Z = go.rff_features(X, theta, True, f, w)
    P = go.Preconditioner(Z, 0.05)
    Cs = np.random.default_rng(11).standard_normal((25, 3))
    tr, ctrl = go._precond_terms_rff(X, theta, True, f, Z, P, Cs, 0, w)

    def dense_P(th):
        Zt = go.rff_features(X, th, True, f, w)
        return th[-1] * np.eye(25) + Zt @ Zt.T

    for i in range(len(theta)):
        h = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Pp, Pm = dense_P(tp), dense_P(tm)
        ref_tr = (np.linalg.slogdet(Pp)[1] - np.linalg.slogdet(Pm)[1]) / (2 * h)
        ref_ctrl = (np.einsum("pi,pq,qi->i", Cs, Pp, Cs) - np.einsum("pi,pq,qi->i", Cs, Pm, Cs)) / (2 * h)
        assert abs(tr[i] - ref_tr) <= 1e-6 * max(1.0, abs(ref_tr)), (i, tr[i], ref_tr)
        np.testing.assert_allclose(ctrl[i], ref_ctrl, rtol=1e-6, atol=1e-6)


def test_qff_estimators_are_unbiased_over_all_sign_patterns():
    X, y, theta = _problem(7, 1, "rbf", False, seed=42, sigma2=0.1, ls=(0.3, 0.6))
    n, k = 7, 2
    vals, grads = [], []
    for bits in itertools.product((-1.0, 1.0), repeat=n + k):
        xi = np.array(bits)
        es = go.estimate_mll(X, y, theta, "rbf", False, k, 1, 1e-13, n, 0, grad=True,
                             signs=(xi[:n, None], xi[n:, None]), precond="qff", qff_nodes=2)
        vals.append(es["logdet_est"])
        grads.append(es["grad"])
    vals, grads = np.array(vals), np.array(grads)
    ex = go.exact_mll(X, y, theta, "rbf", False)
    assert abs(vals.mean() - ex["logdet"]) <= 1e-9 * abs(ex["logdet"])
    np.testing.assert_allclose(grads.mean(axis=0), ex["grad"], rtol=1e-8, atol=1e-9)


# ------------------------------------------------ posterior prediction (Sec. 2.1)

@pytest.mark.parametrize("kind,nu", [("rbf", None), ("matern32", 1.5), ("matern52", 2.5)])
def test_predict_matches_scikit_learn_gaussian_process_regressor(kind, nu):
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import RBF, ConstantKernel, Matern
    X, y, theta = _problem(60, 3, kind, True, seed=50, sigma2=0.05)
    Xs = np.random.default_rng(51).uniform(-0.2, 1.2, size=(25, 3))
    ls, s, s2 = theta[:3], theta[3], theta[4]
    base = RBF(length_scale=ls, length_scale_bounds="fixed") if kind == "rbf" else \
        Matern(length_scale=ls, length_scale_bounds="fixed", nu=nu)
    gpr = GaussianProcessRegressor(ConstantKernel(s, constant_value_bounds="fixed") * base, alpha=s2,
                                   optimizer=None, normalize_y=False).fit(X, y)
    mu_ref, sd_ref = gpr.predict(Xs, return_std=True)
    mu, var = go.predict(X, y, theta, kind, True, Xs)
    np.testing.assert_allclose(mu, mu_ref, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(np.sqrt(np.maximum(var, 0.0)), sd_ref, rtol=1e-7, atol=1e-8)


def test_predict_single_point_closed_form_and_limits():
    X = np.array([[0.3, -0.1]])
    y = np.array([1.7])
    theta = np.array([0.8, 1.3, 0.1])            # isotropic ls, s, sigma^2
    Xs = np.array([[0.3, -0.1], [1.0, 0.5], [30.0, 30.0]])
    mu, var = go.predict(X, y, theta, "rbf", False, Xs)
    k = 1.3 * np.exp(-0.5 * np.sum((Xs - X) ** 2, axis=1) / 0.8 ** 2)
    np.testing.assert_allclose(mu, k * 1.7 / (1.3 + 0.1), rtol=1e-14)
    np.testing.assert_allclose(var, 1.3 - k * k / (1.3 + 0.1), rtol=1e-14)
    assert abs(mu[2]) < 1e-100 and abs(var[2] - 1.3) < 1e-14   # far away: the prior


# ------------------------------------------------ rational quadratic kernel (Table S1)

def test_ratquad_matches_scikit_learn_and_tends_to_rbf():
    from sklearn.gaussian_process.kernels import RationalQuadratic
    X, _, _ = _problem(30, 3, "rbf", False, seed=70)
    for alpha in (0.5, 1.0, 3.0):
        theta = np.array([0.7, 1.0, 0.1])
        K = go.kernel_matrix(X, X, theta, f"ratquad:{alpha}", False)
        ref = RationalQuadratic(length_scale=0.7, alpha=alpha)(X)
        np.testing.assert_allclose(K, ref, rtol=1e-13, atol=1e-15)
    theta = np.array([0.7, 1.0, 0.1])
    Krbf = go.kernel_matrix(X, X, theta, "rbf", False)
    Kbig = go.kernel_matrix(X, X, theta, "ratquad:1e7", False)
    assert np.max(np.abs(Kbig - Krbf)) < 1e-6


def test_ratquad_derivatives_and_gradient_match_finite_differences():
    X, y, theta = _problem(12, 2, "rbf", True, seed=71)
    kind = "ratquad:1.7"
    ex = go.exact_mll(X, y, theta, kind, True)
    for i in range(len(theta)):
        h = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (go.exact_mll(X, y, tp, kind, True)["logp"] - go.exact_mll(X, y, tm, kind, True)["logp"]) / (2 * h)
        assert abs(ex["grad"][i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, ex["grad"][i], fd)


def test_ratquad_spectral_samples_reproduce_the_kernel():
    X, _, theta = _problem(25, 2, "rbf", True, seed=72, ls=(0.5, 1.5))
    W = synthgp.spectral_frequencies("ratquad:2.0", 40000, 2, seed=9)
    Z = go.rff_features(X, theta, True, W)
    assert np.max(np.abs(Z @ Z.T - go.kernel_matrix(X, X, theta, "ratquad:2.0", True))) < 0.03


def test_ratquad_predict_matches_scikit_learn():
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import ConstantKernel, RationalQuadratic
    X, y, theta = _problem(50, 2, "rbf", False, seed=73, sigma2=0.05)
    Xs = np.random.default_rng(74).uniform(-0.2, 1.2, size=(20, 2))
    kern = ConstantKernel(theta[1], constant_value_bounds="fixed") * RationalQuadratic(
        length_scale=theta[0], alpha=2.5, length_scale_bounds="fixed", alpha_bounds="fixed")
    gpr = GaussianProcessRegressor(kern, alpha=theta[2], optimizer=None).fit(X, y)
    mu_ref, sd_ref = gpr.predict(Xs, return_std=True)
    mu, var = go.predict(X, y, theta, "ratquad:2.5", False, Xs)
    np.testing.assert_allclose(mu, mu_ref, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(np.sqrt(np.maximum(var, 0.0)), sd_ref, rtol=1e-7, atol=1e-8)


# ------------------------------------------------ symmetric-square-root probes (R-sqrt)

def test_precond_sqrt_squares_to_the_preconditioner():
    rng = np.random.default_rng(90)
    L = rng.standard_normal((30, 5))
    L[:, 4] = L[:, 3]                       # rank-deficient L^T L is allowed
    S = go.precond_sqrt_apply(L, 0.07, np.eye(30))
    np.testing.assert_allclose(S, S.T, atol=1e-13)
    np.testing.assert_allclose(S @ S, 0.07 * np.eye(30) + L @ L.T, rtol=1e-12, atol=1e-12)
    assert np.all(np.linalg.eigvalsh(S) > 0)


def test_sqrt_probes_have_rho0_n_and_unbiased_estimators():
    X, y, theta = _problem(7, 2, "rbf", True, seed=91, sigma2=0.1, ls=(0.3, 0.6))
    n, k = 7, 2
    vals, grads = [], []
    for bits in itertools.product((-1.0, 1.0), repeat=n):
        xi = np.array(bits)
        es = go.estimate_mll(X, y, theta, "rbf", True, k, 1, 1e-13, n, 0, grad=True,
                             signs=(xi[:, None], np.ones((k, 1))), probe_mode=1)
        assert abs(es["rho0"][1] - n) < 1e-10
        vals.append(es["logdet_est"])
        grads.append(es["grad"])
    ex = go.exact_mll(X, y, theta, "rbf", True)
    assert abs(np.mean(vals) - ex["logdet"]) <= 1e-9 * abs(ex["logdet"])
    np.testing.assert_allclose(np.mean(grads, axis=0), ex["grad"], rtol=1e-8, atol=1e-9)


# ------------------------------------------------ matrix-free (row-blocked) products

def _sklearn_kernel(kind, ls, s):
    from sklearn.gaussian_process.kernels import RBF, ConstantKernel, Matern
    base = RBF(length_scale=ls, length_scale_bounds="fixed") if kind == "rbf" else \
        Matern(length_scale=ls, length_scale_bounds="fixed", nu={"matern32": 1.5, "matern52": 2.5}[kind])
    return ConstantKernel(s, constant_value_bounds="fixed") * base


@pytest.mark.parametrize("native", [False, True])
@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52"])
def test_khat_matvec_matches_a_library_kernel_across_row_blocks(kind, native):
    # n * d = 60,000 gives 666-row blocks: 4 full blocks and a ragged tail of 336 rows
    n, d = 3000, 20
    X, _, theta = _problem(n, d, kind, True, seed=81, sigma2=0.03, ls=(1.5, 4.0), dist="normal")
    assert n % go._row_block(n, d) != 0 and n // go._row_block(n, d) >= 3
    V = np.random.default_rng(82).standard_normal((n, 7))
    ls, s, s2 = theta[:d], theta[d], theta[d + 1]
    K = _sklearn_kernel(kind, ls, s)(X)
    ref = K @ V + s2 * V
    np.testing.assert_allclose(go.khat_matvec(X, theta, kind, True, V, native=native), ref, rtol=1e-11,
                               atol=1e-11)
    # a row subset, unsorted, with a repeat, crossing block edges
    rows = np.random.default_rng(83).choice(n, size=1500, replace=True)
    np.testing.assert_allclose(go.khat_matvec(X, theta, kind, True, V, rows=rows, native=native), ref[rows],
                               rtol=1e-11, atol=1e-11)
    # a single right-hand side as a vector, and a thread pool over the row blocks
    np.testing.assert_allclose(go.khat_matvec(X, theta, kind, True, V[:, 0], native=native, workers=3),
                               ref[:, 0], rtol=1e-11, atol=1e-11)


def test_dkhat_contract_matches_dense_derivative_matrices_across_row_blocks():
    n, d = 2100, 20
    X, _, theta = _problem(n, d, "matern52", True, seed=84, sigma2=0.02, ls=(1.5, 4.0), dist="normal")
    assert n // go._row_block(n, d) >= 2
    rng = np.random.default_rng(85)
    A, C = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    M = A @ C.T
    got = go.dkhat_contract(X, theta, "matern52", True, lambda r: M[r])
    got_threads = go.dkhat_contract(X, theta, "matern52", True, lambda r: M[r], workers=3)
    got_native = go.dkhat_contract_lowrank(X, theta, "matern52", True, A, C)
    # derivative matrices by central differences of a library kernel, one parameter at a time
    ref = np.zeros(d + 2)
    for j in range(d + 1):
        h = 1e-5 * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        Kp = _sklearn_kernel("matern52", tp[:d], tp[d])(X)
        Km = _sklearn_kernel("matern52", tm[:d], tm[d])(X)
        ref[j] = np.sum(M * (Kp - Km)) / (2.0 * h)
    ref[d + 1] = np.trace(M)
    for g in (got, got_threads, got_native):
        np.testing.assert_allclose(g, ref, rtol=2e-7, atol=1e-6 * np.max(np.abs(ref)))
    # row ranges of the plain-C contraction add up to the whole
    halves = (go.dkhat_contract_lowrank(X, theta, "matern52", True, A, C, row_range=(0, 777))
              + go.dkhat_contract_lowrank(X, theta, "matern52", True, A, C, row_range=(777, n)))
    np.testing.assert_allclose(halves, got_native, rtol=1e-12, atol=1e-12 * np.max(np.abs(got_native)))
    # isotropic form: one lengthscale, the sum of the per-dimension terms
    th_iso = np.concatenate([[2.5], theta[d:]])
    iso = go.dkhat_contract(X, th_iso, "matern52", False, lambda r: M[r])
    np.testing.assert_allclose(go.dkhat_contract_lowrank(X, th_iso, "matern52", False, A, C), iso, rtol=1e-11)


@pytest.mark.parametrize("kind,ard,native", [("rbf", True, False), ("matern32", False, False),
                                             ("rbf", True, True), ("ratquad:2.0", True, True)])
def test_matrix_free_estimator_equals_the_dense_one(kind, ard, native):
    # the row-blocked path (used where a dense K_hat does not fit) must give the dense
    # path's estimate: identical probes and pivots, the same numbers up to rounding
    # order.  A fixed number of CG steps (tol 0, the paper's fixed m) keeps a stop
    # decision near the tolerance from depending on that order.
    n, d = 2300, 20
    X, y, theta = _problem(n, d, kind, ard, seed=86, sigma2=0.05, ls=(1.5, 4.0), dist="normal")
    assert n // go._row_block(n, d) >= 2 and n % go._row_block(n, d) != 0
    a = go.estimate_mll(X, y, theta, kind, ard, 15, 6, 0.0, 12, 3, dense=True)
    b = go.estimate_mll(X, y, theta, kind, ard, 15, 6, 0.0, 12, 3, dense=False, native=native)
    np.testing.assert_array_equal(a["piv"], b["piv"])
    np.testing.assert_array_equal(a["iters"], b["iters"])
    assert abs(a["logp"] - b["logp"]) <= 1e-12 * abs(a["logp"])
    np.testing.assert_allclose(b["gammas"], a["gammas"], rtol=1e-10, atol=1e-10 * np.max(np.abs(a["gammas"])))
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-10, atol=1e-10 * np.max(np.abs(a["grad"])))
