"""The interface's limits and degenerate cases on the HIP path against the
oracle: d = GP_MAX_D, ell = GP_MAX_PROBES and rank = GP_MAX_RANK together (FP64,
BF16X3 and FP16X3 tiles); a single point (rank 0 and full rank in FP64, rank 0 in
the split and FP32 tiles).  Marked gpu."""
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


def run(pr, precision, rank, num_probes, tol, max_iters):
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, num_probes, max_iters, tol, 1, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(num_probes, rank)
    B.gp_mll_grad(prob, pr.theta, opt, rank, None, ws, logp, g, st)
    torch.cuda.synchronize()
    return float(logp.cpu()[0]), g.cpu().numpy(), st


@pytest.fixture(scope="module")
def max_case():
    pr = synthgp.random_problem(3000, B.MAX_D, "rbf", ard=True, seed=90, ls_range=(2.0, 6.0), sigma2=0.05,
                                dist="normal")
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, "rbf", True, B.MAX_RANK, B.MAX_PROBES, 1e-8, 300, 1)
    return pr, ref


# measured against the FP64 oracle: BF16x3 1.3e-7 / 1.4e-4, FP16x3 3.7e-8 / 1.5e-4
@pytest.mark.parametrize("precision,lp_tol,g_tol", [("fp64", 1e-7, 1e-5), ("bf16x3", 1e-6, 1e-3),
                                                    ("fp16x3", 2e-7, 1e-3)])
def test_maximum_dimension_probes_and_rank_together(max_case, precision, lp_tol, g_tol):
    pr, ref = max_case
    say(f"[gpu] limits n=3000 d={B.MAX_D} ell={B.MAX_PROBES} rank={B.MAX_RANK} {precision}")
    lp, gr, st = run(pr, precision, B.MAX_RANK, B.MAX_PROBES, 1e-8, 300)
    say(f"    logp rel {rel(lp, ref['logp']):.2e}, grad rel {relvec(gr, ref['grad']):.2e}, iters {st.iters_max}")
    assert st.rank_achieved == ref["rank"] == B.MAX_RANK
    assert rel(lp, ref["logp"]) < lp_tol
    assert relvec(gr, ref["grad"]) < g_tol


@pytest.mark.parametrize("rank", [0, 1])
def test_a_single_point_gives_the_exact_likelihood(rank):
    # n = 1: K_hat = s + sigma^2; with rank 1 the preconditioner is K_hat itself, with
    # rank 0 one CG step is exact; both estimates equal the closed form in expectation,
    # and exactly for rank 1
    X = np.array([[0.3, -0.7]])
    y = np.array([1.3])
    theta = np.array([0.9, 1.1, 0.6, 0.2])
    pr = synthgp.GPProblem("one_point", X, y, theta, "matern32", True, rank=rank, num_probes=4, tol=1e-12,
                           max_iters=5, precision="fp64")
    lp, gr, st = run(pr, "fp64", rank, 4, 1e-12, 5)
    ref = go.estimate_mll(X, y, theta, "matern32", True, rank, 4, 1e-12, 5, 1)
    assert rel(lp, ref["logp"]) < 1e-12
    np.testing.assert_allclose(gr, ref["grad"], rtol=1e-10, atol=1e-12)
    kh = theta[2] + theta[3]
    exact = -0.5 * (y[0] ** 2 / kh + np.log(kh) + np.log(2 * np.pi))
    if rank == 1:
        assert rel(lp, exact) < 1e-12
    assert st.iters_max <= 1


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3", "fp32"])
def test_a_single_point_in_split_and_single_precision_tiles(precision):
    # n = 1 pads to a whole 256-row tile block of zero operands; the one kernel value is
    # the exact diagonal s, so only the tile product's rounding separates the estimate
    # from the FP64 oracle's
    X = np.array([[0.3, -0.7]])
    y = np.array([1.3])
    theta = np.array([0.9, 1.1, 0.6, 0.2])
    say(f"[gpu] single point, {precision} tiles")
    lp, gr, st = run(synthgp.GPProblem("one_point", X, y, theta, "rbf", True, rank=0, num_probes=4, tol=1e-12,
                                       max_iters=5, precision=precision), precision, 0, 4, 1e-12, 5)
    ref = go.estimate_mll(X, y, theta, "rbf", True, 0, 4, 1e-12, 5, 1)
    assert rel(lp, ref["logp"]) < 1e-4
    assert relvec(gr, ref["grad"]) < 1e-3
    assert st.iters_max <= 2


def test_workspace_one_byte_short_is_rejected():
    pr = synthgp.random_problem(700, 3, "rbf", ard=True, seed=98, dist="normal")
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, "rbf", True)
    opt = B.make_options("fp64", 8, 100)
    need = B.gp_workspace_size(prob, opt, 16)
    ws = B.alloc_workspace(need - 1)
    lp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    for call in (lambda: B.gp_mll_grad(prob, pr.theta, opt, 16, None, ws, lp, g),
                 lambda: B.gp_mll_eval(prob, pr.theta, opt, 16, None, ws, lp),
                 lambda: B.gp_predict(prob, pr.theta, opt, 16, None, X[:4], ws, lp.repeat(4))):
        with pytest.raises(B.GPError) as e:
            call()
        assert e.value.code == B.GP_EWORKSPACE
    full = B.alloc_workspace(need)
    B.gp_mll_grad(prob, pr.theta, opt, 16, None, full, lp, g)      # the exact size is enough
    torch.cuda.synchronize()
    assert np.isfinite(float(lp.cpu()[0]))
