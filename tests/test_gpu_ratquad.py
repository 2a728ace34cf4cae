"""The rational quadratic kernel (Table S1's third kernel) on the HIP path against
the oracle, through the C-ABI: K_hat V tiles in every precision, the estimator
and its gradient, and posterior prediction.  Marked gpu."""
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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def relvec(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


MATVEC_TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 2e-4, "fp16x3": 1e-4}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("alpha", [0.5, 2.0])
@pytest.mark.parametrize("n,d,nrhs", [(1000, 3, 17), (777, 8, 33), (1300, 20, 65)])
def test_ratquad_khat_matvec_matches_oracle(precision, alpha, n, d, nrhs):
    kind = f"ratquad:{alpha}"
    pr = synthgp.random_problem(n, d, kind, ard=True, seed=n + d, ls_range=(0.5, 2.0), dist="normal")
    say(f"[gpu] ratquad khat_matvec n={n} d={d} rhs={nrhs} alpha={alpha} {precision}")
    dev = torch.device("cuda:0")
    V = np.random.default_rng(8).standard_normal((n, nrhs))
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, kind, True)
    opt = B.make_options(precision, max(1, nrhs - 1), 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, 0))
    Vd = torch.tensor(V, device=dev)
    Wd = torch.zeros_like(Vd)
    B.gp_khat_matvec(prob, pr.theta, precision, Vd, Wd, ws)
    ref = go.khat_matvec(pr.X, pr.theta, kind, True, V)
    scale = np.abs(go.khat_dense(pr.X, pr.theta, kind, True)) @ np.abs(V)
    err = np.max(np.abs(Wd.cpu().numpy() - ref) / scale)
    say(f"    max scaled error {err:.3e}")
    assert err < MATVEC_TOL[precision]


# split and FP32 tiles: about five times the measured distance over both shapes
# (FP32 1.4e-6 / 3.9e-5, BF16x3 1.4e-5 / 5.6e-4, FP16x3 1.0e-6 / 9.3e-5)
@pytest.mark.parametrize("precision,lp_tol,g_tol", [("fp64", 1e-7, 1e-5), ("fp32", 1e-5, 2e-4),
                                                     ("bf16x3", 1e-4, 5e-3), ("fp16x3", 1e-5, 5e-4)])
@pytest.mark.parametrize("alpha,ard", [(0.8, True), (3.0, False)])
def test_ratquad_estimator_and_gradient_match_oracle(alpha, ard, precision, lp_tol, g_tol):
    kind = f"ratquad:{alpha}"
    pr = synthgp.random_problem(1500, 4, kind, ard=ard, rank=20, num_probes=8, seed=80, ls_range=(0.4, 1.5),
                                sigma2=0.05, dist="normal", tol=1e-8, max_iters=400)
    say(f"[gpu] ratquad estimator alpha={alpha} ard={ard} {precision}")
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, kind, ard)
    opt = B.make_options(precision, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, pr.rank))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(pr.num_probes, pr.rank)
    B.gp_mll_grad(prob, pr.theta, opt, pr.rank, None, ws, logp, g, st)
    torch.cuda.synchronize()
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, kind, ard, pr.rank, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed)
    lp, gr = float(logp.cpu()[0]), g.cpu().numpy()
    say(f"    logp rel {rel(lp, ref['logp']):.2e}, grad rel {relvec(gr, ref['grad']):.2e}, "
        f"iters {st.iters_max} / {ref['iters'].max()}")
    assert rel(lp, ref["logp"]) < lp_tol
    assert relvec(gr, ref["grad"]) < g_tol
    if precision == "fp64":
        np.testing.assert_array_equal(st.pivots, ref["piv"])


def test_ratquad_gradient_against_the_exact_dense_gradient():
    # with n-step CG and a full-rank preconditioner the estimator is exact
    kind = "ratquad:1.5"
    pr = synthgp.random_problem(60, 2, kind, ard=True, rank=60, num_probes=2, seed=81, sigma2=0.1,
                                tol=1e-13, max_iters=60)
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, kind, True)
    opt = B.make_options("fp64", 2, 60, 1e-13, 1, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, 60))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    B.gp_mll_grad(prob, pr.theta, opt, 60, None, ws, logp, g)
    torch.cuda.synchronize()
    ex = go.exact_mll(pr.X, pr.y, pr.theta, kind, True)
    assert rel(float(logp.cpu()[0]), ex["logp"]) < 1e-9
    np.testing.assert_allclose(g.cpu().numpy(), ex["grad"], rtol=1e-7, atol=1e-9)


def test_ratquad_predict_matches_the_dense_posterior():
    kind = "ratquad:2.5"
    pr = synthgp.random_problem(1200, 3, kind, ard=True, seed=82, ls_range=(0.4, 1.5), sigma2=0.05, dist="normal")
    Xs = np.random.default_rng(83).standard_normal((40, 3))
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, kind, True)
    opt = B.make_options("fp64", 16, 600, 1e-10, 1, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, 20))
    mean = torch.zeros(40, dtype=torch.float64, device=dev)
    var = torch.zeros(40, dtype=torch.float64, device=dev)
    B.gp_predict(prob, pr.theta, opt, 20, None, torch.tensor(Xs, device=dev), ws, mean, var)
    mu_ref, var_ref = go.predict(pr.X, pr.y, pr.theta, kind, True, Xs)
    assert np.max(np.abs(mean.cpu().numpy() - mu_ref)) / np.max(np.abs(mu_ref)) < 1e-8
    assert np.max(np.abs(var.cpu().numpy() - var_ref)) < 1e-8
