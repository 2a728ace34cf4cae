"""Posterior prediction (gp_predict) on the HIP path against the oracle's dense
posterior, through the C-ABI.  Marked gpu."""
import sys

import numpy as np
import pytest

import synthgp
from oracle import gp_oracle as go

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_00243_amd import binding as B  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    B.load()


def run_predict(pr, Xs, precision, rank, num_probes=64, tol=1e-10, with_var=True, precond=None):
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, num_probes, 600, tol, 1, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank))
    Xsd = torch.tensor(np.ascontiguousarray(Xs), device=dev)
    mean = torch.zeros(Xs.shape[0], dtype=torch.float64, device=dev)
    var = torch.zeros(Xs.shape[0], dtype=torch.float64, device=dev) if with_var else None
    h = None
    if precond == "nystrom":
        h = B.gp_precond_build_nystrom(prob, pr.theta, rank, synthgp.uniform_landmarks(pr.n, rank, seed=3), ws)
    try:
        B.gp_predict(prob, pr.theta, opt, rank, h, Xsd, ws, mean, var)
    finally:
        if h is not None:
            B.gp_precond_free(h)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), (var.cpu().numpy() if with_var else None)


CASES = [
    ("rbf", True, 1500, 4),
    ("matern32", True, 1100, 6),
    ("matern52", False, 900, 3),
]


@pytest.mark.parametrize("kernel,ard,n,d", CASES)
@pytest.mark.parametrize("precision,mtol,vtol", [("fp64", 1e-8, 1e-8), ("fp32", 1e-4, 1e-4), ("bf16x3", 1e-3, 1e-3),
                                                 ("fp16x3", 1e-3, 1e-3)])
def test_predict_matches_the_dense_posterior(kernel, ard, n, d, precision, mtol, vtol):
    pr = synthgp.random_problem(n, d, kernel, ard=ard, seed=60 + d, ls_range=(0.4, 1.5), sigma2=0.05,
                                dist="normal")
    Xs = np.random.default_rng(61).standard_normal((150, d)) * 1.2      # chunks of 64 + 64 + 22
    say(f"[gpu] predict {kernel} ard={ard} n={n} d={d} n*=150 {precision}")
    mu, var = run_predict(pr, Xs, precision, 20)
    mu_ref, var_ref = go.predict(pr.X, pr.y, pr.theta, kernel, ard, Xs)
    em = np.max(np.abs(mu - mu_ref)) / np.max(np.abs(mu_ref))
    ev = np.max(np.abs(var - var_ref)) / pr.theta[-2]
    say(f"    mean err {em:.2e} (of max |mean|), var err {ev:.2e} (of s)")
    assert em < mtol and ev < vtol


def test_predict_with_a_prebuilt_preconditioner_and_without_variance():
    pr = synthgp.random_problem(1300, 3, "rbf", ard=True, seed=63, ls_range=(0.4, 1.5), sigma2=0.05, dist="normal")
    Xs = np.random.default_rng(64).standard_normal((70, 3))
    mu, var = run_predict(pr, Xs, "fp64", 24, num_probes=32, with_var=False, precond="nystrom")
    assert var is None
    mu_ref, _ = go.predict(pr.X, pr.y, pr.theta, "rbf", True, Xs)
    assert np.max(np.abs(mu - mu_ref)) / np.max(np.abs(mu_ref)) < 1e-8


def test_predict_at_training_points_and_far_away():
    # at a training point with small noise the mean is close to y and the variance
    # small; far from the data the posterior is the prior (mean 0, variance s)
    pr = synthgp.random_problem(800, 2, "matern52", ard=True, seed=65, ls_range=(0.5, 1.0), sigma2=1e-3,
                                dist="normal")
    Xs = np.concatenate([pr.X[:5], np.full((3, 2), 50.0)])
    mu, var = run_predict(pr, Xs, "fp64", 30, num_probes=16)
    mu_ref, var_ref = go.predict(pr.X, pr.y, pr.theta, "matern52", True, Xs)
    np.testing.assert_allclose(mu, mu_ref, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(var, var_ref, rtol=1e-6, atol=1e-9)
    assert np.all(np.abs(mu[5:]) < 1e-12) and np.allclose(var[5:], pr.theta[-2], rtol=1e-12)
