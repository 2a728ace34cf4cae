"""The Table S1 experiment on the HIP path (supplement, synthetic data): bias and
variance of the stochastic estimates of log p and of its derivatives with respect
to the outputscale, the lengthscale and the noise, with ell = 128 probes and no
preconditioner (rank 0) or a rank-128 partial Cholesky one.  Synthetic
n = 10,000, sigma^2 = 1e-2, d in {1, 2, 3}, the paper's three kernels (RBF,
Matern-3/2, rational quadratic); the problems of synthgp.table_s1.  Exact targets
from the oracle's dense Cholesky, stored by tests/golden/make_table_s1.py.
Relative errors est / exact - 1 per quantity (scale-free, so the outputscale and
noise parameterisation does not matter, and d/dsigma = 2 sigma d/dsigma^2 has the
relative error of d/dsigma^2); bias = |mean|, variance over the repetitions.
bench.py --table-s1 runs the paper's 25 repetitions; the tests run 6.  Marked gpu."""
import json
import os
import sys

import numpy as np
import pytest

import synthgp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_00243_amd import binding as B  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table_s1_exact.json")
COLUMNS = ("log p", "d/do", "d/dl", "d/dsigma")
REPS = 6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def table_s1_errors(pr, exact, rank, reps, seed0=0):
    """Relative errors (reps x 4) of log p and the outputscale, lengthscale and
    noise derivatives from gp_mll_grad with FP64 tiles and `reps` probe seeds."""
    dev = torch.device("cuda:0")
    X, y = torch.tensor(pr.X, device=dev), torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options("fp64", pr.num_probes, pr.max_iters, pr.tol, 1, 0, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(3, dtype=torch.float64, device=dev)
    ex = np.array([exact["logp"], exact["grad"][1], exact["grad"][0], exact["grad"][2]])
    errs, iters, flags = [], 0, 0
    for r in range(reps):
        opt.seed = seed0 + 1009 * rank + r
        st = B.Stats(pr.num_probes, rank)
        B.gp_mll_grad(prob, pr.theta, opt, rank, None, ws, logp, g, st)
        gr = g.cpu().numpy()
        est = np.array([float(logp.cpu()[0]), gr[1], gr[0], gr[2]])
        errs.append(est / ex - 1.0)
        iters = max(iters, int(st.iters_max))
        flags |= int(st.flags)
    del ws
    torch.cuda.empty_cache()
    return np.array(errs), iters, flags


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("kernel", synthgp.TABLE_S1_KERNELS)
def test_table_s1_bias_and_variance_at_rank_0_and_128(kernel, d):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    pr = synthgp.table_s1(kernel, d)
    exact = json.load(open(GOLDEN))["problems"][pr.name]
    assert np.allclose(exact["theta"], pr.theta) and exact["n"] == pr.n
    rows = {}
    for rank in (0, 128):
        e, iters, flags = table_s1_errors(pr, exact, rank, reps=REPS)
        assert flags & B.FLAG_NOT_CONVERGED == 0
        mean, var = e.mean(axis=0), e.var(axis=0, ddof=1)
        rows[rank] = (np.abs(mean), var, iters)
        say(f"[gpu] Table S1 {kernel} d={d} rank {rank:3d} (CG <= {iters}): "
            + "  ".join(f"{c} {abs(b):.0e}/{v:.0e}" for c, b, v in zip(COLUMNS, mean, var)))
        # with solves run to convergence both estimators are unbiased (Theorems 4
        # and 5): the mean error over the repetitions stays within a few standard
        # errors of zero (t with REPS - 1 degrees of freedom, |t| > 6 has
        # probability below 0.2 %), up to FP64 rounding of the whole evaluation
        # against the oracle's dense factorisation (1e-7 relative; where rank 128
        # makes the preconditioner exact the errors are that rounding alone, the
        # same in every repetition)
        assert np.all(np.abs(mean) <= 6.0 * np.sqrt(var / REPS) + 1e-7), (rank, mean, var)
    (b0, v0, it0), (b1, v1, it1) = rows[0], rows[128]
    # the preconditioned solves need fewer iterations in every case
    assert it1 < it0
    # in one dimension the rank-128 preconditioner captures the spectrum above
    # sigma^2, and every column's variance falls more than tenfold (measured: 30x
    # for the Matern-3/2 derivatives, whose pivoted Cholesky error decays
    # slowest, up to 1e20x for RBF); so it does for RBF in two dimensions. In two
    # and three dimensions the Matern-3/2 and rational quadratic spectra, and the
    # RBF one in three, keep many eigenvalues above sigma^2 beyond rank 128 and the
    # variance changes little: no claim is made there
    if d == 1 or kernel == "rbf" and d == 2:
        assert np.all(v1 < 0.1 * v0), (v0, v1)
