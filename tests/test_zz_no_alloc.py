"""The no-allocation K_hat V entry point (its staging arrays in the library's
own device array) against the workspace entry point, through the C ABI."""
import sys

import numpy as np
import pytest

import synthgp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_00243_amd import binding as B  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(pr, precision, nrhs, seed):
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    V = torch.tensor(np.random.default_rng(seed).standard_normal((pr.n, nrhs)), device=dev)
    opt = B.make_options(precision, max(1, nrhs - 1), 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, 0))
    W_ws = torch.zeros_like(V)
    B.gp_khat_matvec(prob, pr.theta, precision, V, W_ws, ws)
    W_na = torch.full_like(V, float("nan"))
    B.gp_khat_matvec_noalloc(prob, pr.theta, precision, V, W_na)
    torch.cuda.synchronize()
    return W_ws.cpu().numpy(), W_na.cpu().numpy(), V.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_noalloc_matvec_matches_the_workspace_entry_point_on_consecutive_calls(precision):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    # a larger call, then a smaller one that reuses (and must not see) its leftovers
    cases = [(synthgp.random_problem(4100, 8, "matern52", ard=True, seed=3, dist="normal"), 33),
             (synthgp.random_problem(1200, 5, "rbf", ard=False, seed=4), 17)]
    for k, (pr, nrhs) in enumerate(cases):
        say(f"[gpu] noalloc matvec call {k}: n={pr.n} d={pr.d} rhs={nrhs} {precision}")
        W_ws, W_na, _ = both(pr, precision, nrhs, seed=10 + k)
        # same layout geometry (the arrays fit without fewer column splits), same
        # kernels: the same numbers
        np.testing.assert_array_equal(W_na, W_ws)


def test_noalloc_matvec_with_fewer_column_splits():
    # n = 60,000 with 65 columns: the partial sums of the workspace entry point's
    # splits exceed the library's array, so fewer splits are taken (rounding order
    # differs; the scale is sum_j |K_ij| |V_jc|, bounded here by (s n + sigma^2) max|V|)
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    pr = synthgp.rbf_ard_100k(n=60000)
    say(f"[gpu] noalloc matvec n={pr.n} rhs=65 bf16x3 (fewer splits)")
    W_ws, W_na, V = both(pr, "bf16x3", 65, seed=12)
    assert np.all(np.isfinite(W_na))
    err = np.max(np.abs(W_na - W_ws), axis=0) / np.max(np.abs(W_ws), axis=0)
    say(f"    max column-relative difference {err.max():.2e}")
    assert err.max() < 1e-5
