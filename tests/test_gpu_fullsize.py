"""The HIP path at the full sizes of the benchmark workloads against the CPU
oracle's references (tests/golden/oracle_<workload>.json, written by
tests/golden/make_full_size.py from the oracle alone): the same-probe estimate
of Algorithms 1 and 2, and where a dense factor fits, the exact Eq. (1) and
Eq. (2) targets.  Marked gpu."""
import json
import math
import os
import sys

import numpy as np
import pytest

import synthgp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2107_00243_amd import binding as B  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def reference(workload):
    return json.load(open(os.path.join(GOLDEN, f"oracle_{workload}.json")))


def rel(a, b):
    return abs(a - b) / abs(b)


def relvec(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def run(pr, precision):
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, pr.rank))
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(pr.num_probes, pr.rank)
    B.gp_mll_grad(prob, pr.theta, opt, pr.rank, None, ws, logp, g, st)
    torch.cuda.synchronize()
    out = {"logp": float(logp.cpu()[0]), "grad": g.cpu().numpy(), "stats": st}
    del ws
    torch.cuda.empty_cache()
    return out


# Same-probe bars: FP64 tiles differ from the oracle by rounding order only; the
# FP32 and split tiles by their product error (about 1e-6 relative per kernel
# value), which moves log p by far less than 1e-6 and the gradient by less than
# 1e-4 (measured: 1e-8 and 3e-5 at n = 20,000 with FP32 tiles).
SAME_PROBE = {"fp64": (1e-8, 1e-6), "fp32": (1e-6, 1e-4), "bf16x3": (1e-6, 1e-4), "fp16x3": (1e-6, 1e-4)}


@pytest.mark.parametrize("workload,precision", [
    ("plain_rbf_1000", "fp64"),
    ("matern52_ard_20k", "fp32"),
    ("matern52_ard_20k", "fp64"),
])
def test_dense_workloads_against_the_oracle_and_the_exact_targets(workload, precision):
    ref = reference(workload)
    pr = getattr(synthgp, workload)()
    assert ref["n"] == pr.n and np.allclose(ref["theta"], pr.theta) and ref["max_iters"] == pr.max_iters
    say(f"[gpu] {workload} n={pr.n} {precision} against the oracle reference")
    out = run(pr, precision)
    st = out["stats"]
    est, ex = ref["estimate"], ref["exact"]
    assert st.flags & B.FLAG_NOT_CONVERGED == 0
    assert list(st.pivots[:pr.rank]) == est["pivots"]
    lp_tol, g_tol = SAME_PROBE[precision]
    e_lp, e_g = rel(out["logp"], est["logp"]), relvec(out["grad"], est["grad"])
    say(f"    same-probe oracle: log p rel {e_lp:.2e}, gradient rel {e_g:.2e}, CG iterations "
        f"{int(st.iters_max)} (oracle {max(est['col_iters'])})")
    assert e_lp < lp_tol and e_g < g_tol
    # the exact targets: the estimator's own error at this probe count and rank
    x_lp, x_g = rel(out["logp"], ex["logp"]), relvec(out["grad"], ex["grad"])
    x_fit = rel(st.datafit, ex["datafit"])
    x_det = rel(st.logdet_estimate, ex["logdet"])
    say(f"    exact (Eq. 1, Eq. 2): log p rel {x_lp:.2e}, data fit rel {x_fit:.2e}, log det rel {x_det:.2e}, "
        f"gradient rel {x_g:.2e}")
    # log p is an average over probes: its error must sit within four standard
    # errors of that average (the spread of the per-probe log-det terms)
    gam = np.asarray(est["gammas"])
    se = 0.5 * np.std(gam, ddof=1) / math.sqrt(len(gam))
    assert abs(out["logp"] - ex["logp"]) <= 4.0 * se + 1e-6 * abs(ex["logp"])
    assert x_fit < 1e-6


# n = 100,000: same-probe bars about five times the distances measured between the
# split tiles and the FP64 tiles of the same evaluation (3e-9 to 1e-8 on log p,
# 3e-6 on the gradient)
C3_BARS = {"fp64": (1e-8, 1e-6), "bf16x3": (5e-8, 2e-5), "fp16x3": (5e-8, 2e-5)}


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x3"])
def test_rbf_ard_100k_against_the_matrix_free_oracle(precision):
    # the headline workload at its full size against the oracle's matrix-free FP64
    # run of the same probes (about 45 minutes on six CPU threads); the exact
    # Eq. (1) / Eq. (2) targets are out of reach there (a dense factor of K_hat
    # would take 80 GB)
    ref = reference("rbf_ard_100k")
    pr = synthgp.rbf_ard_100k()
    assert ref["n"] == pr.n and np.allclose(ref["theta"], pr.theta)
    say(f"[gpu] rbf_ard_100k n={pr.n} {precision} against the matrix-free oracle")
    out = run(pr, precision)
    st = out["stats"]
    est = ref["estimate"]
    assert st.flags & B.FLAG_NOT_CONVERGED == 0
    assert list(st.pivots[:pr.rank]) == est["pivots"]
    e_lp, e_g = rel(out["logp"], est["logp"]), relvec(out["grad"], est["grad"])
    gam = np.asarray(est["gammas"])
    say(f"    log p rel {e_lp:.2e}, gradient rel {e_g:.2e}, CG {int(st.iters_max)} (oracle {max(est['col_iters'])}), "
        f"probe terms rel {np.max(np.abs(st.gammas - gam)) / np.max(np.abs(gam)):.2e}")
    lp_tol, g_tol = C3_BARS[precision]
    assert e_lp < lp_tol and e_g < g_tol
