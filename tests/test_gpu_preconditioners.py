"""Parity of the other diagonal-plus-low-rank preconditioners of Table 1 on the
HIP path against the CPU oracle, through the C-ABI: random Fourier features
("RFF") and the randomized Nystrom approximation on given landmarks.  Marked gpu."""
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
    return torch.device("cuda:0")


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def relvec(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def run_rff(pr, precision, rank, W, num_probes=None, tol=None, max_iters=None, precond_grad=0, grad=True):
    num_probes = pr.num_probes if num_probes is None else num_probes
    tol = pr.tol if tol is None else tol
    max_iters = pr.max_iters if max_iters is None else max_iters
    say(f"[gpu] rff estimator {pr.name} n={pr.n} d={pr.d} {pr.kernel} ard={pr.ard} prec={precision} "
        f"k={rank} ell={num_probes} mode={precond_grad}")
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    Wd = torch.tensor(np.ascontiguousarray(W), device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, num_probes, max_iters, tol, pr.probe_seed, precond_grad, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank))
    h = B.gp_precond_build_rff(prob, pr.theta, rank, Wd, ws)
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(num_probes, rank)
    try:
        if grad:
            B.gp_mll_grad(prob, pr.theta, opt, rank, h, ws, logp, g, st)
        else:
            B.gp_mll_eval(prob, pr.theta, opt, rank, h, ws, logp, st)
        torch.cuda.synchronize()
        v = B.gp_precond_view_of(h)
        n = pr.n
        Wg = np.frombuffer(ws.cpu().numpy().tobytes(), dtype=np.uint8)  # whole workspace on host
        base = ws.data_ptr()
        Z = Wg[v.L_dev - base: v.L_dev - base + n * rank * 8].view(np.float64).reshape(rank, n).T
        piv = Wg[v.pivots_dev - base: v.pivots_dev - base + rank * 4].view(np.int32)
        ldp = float(Wg[v.logdet_dev - base: v.logdet_dev - base + 8].view(np.float64)[0])
    finally:
        B.gp_precond_free(h)
    return {"logp": float(logp.cpu()[0]), "grad": g.cpu().numpy(), "stats": st, "Z": Z,
            "piv": piv, "logdet_P": ldp}


# RFF preconditioners of small rank are weak (Table 1: error rate k^-1/2), so
# the cases keep CG well inside its cap: a column that stops at the cap leaves
# a finite-precision Lanczos run whose rounding the two sides do not share.
CASES = [
    # name, n, d, kernel, ard, rank, sigma^2, CG iterations of the oracle
    ("rbf_1d", 1500, 1, "rbf", False, 64, 0.05),          # 17
    ("rbf_ard_2d", 1500, 2, "rbf", True, 64, 0.05),       # 138 (quadrature path)
    ("matern32_ard_6d", 1100, 6, "matern32", True, 24, 0.5),  # 175
    ("matern52_iso_3d", 900, 3, "matern52", False, 10, 0.5),  # 116
    ("ratquad_ard_2d", 1200, 2, "ratquad:1.5", True, 64, 0.2),  # 47 (Gamma-mixture frequencies)
]


def _case(n, d, kernel, ard, rank, s2, seed):
    ls = (0.5, 1.0) if d == 1 else ((0.5, 1.5) if d == 2 else (0.4, 1.5))
    pr = synthgp.random_problem(n, d, kernel, ard=ard, rank=rank, num_probes=8, seed=seed,
                                ls_range=ls, sigma2=s2, dist="normal", tol=1e-8, max_iters=400)
    W = synthgp.spectral_frequencies(kernel, rank // 2, d, seed=seed)
    return pr, W


@pytest.mark.parametrize("name,n,d,kernel,ard,rank,s2", CASES)
def test_rff_features_and_logdet_match_oracle(name, n, d, kernel, ard, rank, s2):
    pr, W = _case(n, d, kernel, ard, rank, s2, seed=32)
    out = run_rff(pr, "fp64", rank, W, grad=False)
    Zr = go.rff_features(pr.X, pr.theta, ard, W)
    np.testing.assert_allclose(out["Z"], Zr, rtol=0, atol=1e-12 * np.sqrt(pr.theta[-2]))
    ldp = go.Preconditioner(Zr, pr.theta[-1]).logdet
    assert rel(out["logdet_P"], ldp) < 1e-11
    assert np.all(out["piv"] == -1)
    assert out["stats"].rank_achieved == rank
    assert out["stats"].flags & B.FLAG_RANK_DEFICIENT == 0


# Same-probe bars (log p, gradient) per case and tile precision, about five times
# the measured distance from the oracle: the split and FP32 tiles perturb every
# product by their rounding (about 1e-5 and 1e-6 of |K||V|), which the long CG runs
# of these weak preconditioners carry into the quadrature (measured: BF16x3 up to
# 5e-4 on log p for the two-dimensional RBF case, FP16x3 and FP32 below 4e-5).
RFF_BARS = {
    ("rbf_1d", "bf16x3"): (1e-3, 1e-2), ("rbf_1d", "fp16x3"): (5e-5, 2e-3), ("rbf_1d", "fp32"): (1e-4, 1e-3),
    ("rbf_ard_2d", "bf16x3"): (1e-3, 1e-2), ("rbf_ard_2d", "fp16x3"): (1e-4, 5e-3),
    ("rbf_ard_2d", "fp32"): (2e-4, 1e-3),
    ("matern32_ard_6d", "bf16x3"): (2e-7, 2e-4), ("matern32_ard_6d", "fp16x3"): (2e-7, 2e-4),
    ("matern32_ard_6d", "fp32"): (5e-8, 1e-5),
    ("matern52_iso_3d", "bf16x3"): (5e-6, 5e-4), ("matern52_iso_3d", "fp16x3"): (1e-7, 5e-4),
    ("matern52_iso_3d", "fp32"): (5e-7, 5e-5),
    ("ratquad_ard_2d", "bf16x3"): (1e-4, 5e-3), ("ratquad_ard_2d", "fp16x3"): (5e-6, 5e-4),
    ("ratquad_ard_2d", "fp32"): (1e-6, 5e-5),
}


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x3", "fp32"])
@pytest.mark.parametrize("name,n,d,kernel,ard,rank,s2", CASES)
def test_rff_estimator_matches_oracle(name, n, d, kernel, ard, rank, s2, precision):
    lp_tol, g_tol = (1e-7, 1e-5) if precision == "fp64" else RFF_BARS[(name, precision)]
    pr, W = _case(n, d, kernel, ard, rank, s2, seed=32)
    out = run_rff(pr, precision, rank, W)
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, kernel, ard, rank, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed, grad=True, precond="rff", freqs=W)
    say(f"    logp {out['logp']:.12e} oracle {ref['logp']:.12e} rel {rel(out['logp'], ref['logp']):.2e}; "
        f"grad rel {relvec(out['grad'], ref['grad']):.2e}")
    assert rel(out["logp"], ref["logp"]) < lp_tol
    assert relvec(out["grad"], ref["grad"]) < g_tol
    assert out["stats"].flags & B.FLAG_NOT_CONVERGED == 0
    if precision == "fp64":
        # past the loss of orthogonality the step at which the recurrence residual
        # crosses the tolerance depends on rounding order (the results above do not)
        assert abs(out["stats"].iters_max - int(ref["iters"].max())) <= 1 + 0.05 * int(ref["iters"].max())


@pytest.mark.parametrize("mode", [0, 1])
def test_rff_precond_grad_modes_match_oracle(mode):
    pr, W = _case(1100, 6, "matern32", True, 24, 0.5, seed=33)   # 129 CG iterations
    out = run_rff(pr, "fp64", 24, W, precond_grad=mode)
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, "matern32", True, 24, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed, grad=True, precond_grad=mode, precond="rff", freqs=W)
    assert relvec(out["grad"], ref["grad"]) < 1e-5
    assert rel(out["logp"], ref["logp"]) < 1e-7


def test_rff_rejects_bad_arguments():
    pr, W = _case(200, 2, "rbf", True, 8, 0.1, seed=34)
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, "rbf", True)
    opt = B.make_options("fp64", 4, 50)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, 8))
    Wd = torch.tensor(W, device=dev)
    for rank in (7, 0):
        with pytest.raises(B.GPError):
            B.gp_precond_build_rff(prob, pr.theta, rank, Wd, ws)


# ---------------------------------------------------------------- randomized Nystrom

NYS_CASES = [
    # name, n, d, kernel, ard, rank, sigma^2, CG iterations of the oracle
    ("rbf_ard_4d", 1500, 4, "rbf", True, 40, 0.02),            # 208 (quadrature path)
    ("matern32_ard_6d", 1100, 6, "matern32", True, 24, 0.1),   # 48
    ("matern52_iso_3d", 900, 3, "matern52", False, 16, 0.05),  # 139
    ("ratquad_ard_3d", 1000, 3, "ratquad:1.5", True, 20, 0.2),  # 59
]


def _nys_case(n, d, kernel, ard, rank, s2, seed=35):
    pr = synthgp.random_problem(n, d, kernel, ard=ard, rank=rank, num_probes=8, seed=seed,
                                ls_range=(0.4, 1.5), sigma2=s2, dist="normal", tol=1e-8, max_iters=400)
    return pr, synthgp.uniform_landmarks(n, rank, seed=seed)


def run_nystrom(pr, precision, rank, S, precond_grad=0, grad=True):
    say(f"[gpu] nystrom estimator {pr.name} n={pr.n} d={pr.d} {pr.kernel} ard={pr.ard} prec={precision} "
        f"k={rank} mode={precond_grad}")
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, pr.kernel, pr.ard)
    opt = B.make_options(precision, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, precond_grad, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank))
    h = B.gp_precond_build_nystrom(prob, pr.theta, rank, S, ws)
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(pr.num_probes, rank)
    try:
        if grad:
            B.gp_mll_grad(prob, pr.theta, opt, rank, h, ws, logp, g, st)
        else:
            B.gp_mll_eval(prob, pr.theta, opt, rank, h, ws, logp, st)
        torch.cuda.synchronize()
        v = B.gp_precond_view_of(h)
        n = pr.n
        Wg = np.frombuffer(ws.cpu().numpy().tobytes(), dtype=np.uint8)
        base = ws.data_ptr()
        L = Wg[v.L_dev - base: v.L_dev - base + n * rank * 8].view(np.float64).reshape(rank, n).T
        piv = Wg[v.pivots_dev - base: v.pivots_dev - base + rank * 4].view(np.int32)
        ldp = float(Wg[v.logdet_dev - base: v.logdet_dev - base + 8].view(np.float64)[0])
    finally:
        B.gp_precond_free(h)
    return {"logp": float(logp.cpu()[0]), "grad": g.cpu().numpy(), "stats": st, "L": L, "piv": piv,
            "logdet_P": ldp}


@pytest.mark.parametrize("name,n,d,kernel,ard,rank,s2", NYS_CASES)
def test_nystrom_factor_matches_oracle(name, n, d, kernel, ard, rank, s2):
    pr, S = _nys_case(n, d, kernel, ard, rank, s2)
    out = run_nystrom(pr, "fp64", rank, S, grad=False)
    Lr, pivr, kp = go.pivoted_cholesky(pr.X, pr.theta, kernel, ard, rank, order=S)
    assert kp == rank
    np.testing.assert_array_equal(out["piv"], S)
    np.testing.assert_allclose(out["L"], Lr, rtol=1e-9, atol=1e-11)
    assert rel(out["logdet_P"], go.Preconditioner(Lr, pr.theta[-1]).logdet) < 1e-11
    assert out["stats"].rank_achieved == rank


# same-probe bars per case, about five times the measured distance (as RFF_BARS)
NYS_BARS = {
    ("rbf_ard_4d", "bf16x3"): (5e-4, 1e-2), ("rbf_ard_4d", "fp16x3"): (5e-5, 5e-3),
    ("rbf_ard_4d", "fp32"): (1e-5, 5e-4),
    ("matern32_ard_6d", "bf16x3"): (5e-7, 5e-4), ("matern32_ard_6d", "fp16x3"): (5e-7, 5e-4),
    ("matern32_ard_6d", "fp32"): (5e-9, 2e-5),
    ("matern52_iso_3d", "bf16x3"): (5e-5, 1e-3), ("matern52_iso_3d", "fp16x3"): (5e-6, 1e-3),
    ("matern52_iso_3d", "fp32"): (5e-7, 1e-4),
    ("ratquad_ard_3d", "bf16x3"): (2e-5, 5e-3), ("ratquad_ard_3d", "fp16x3"): (5e-7, 1e-3),
    ("ratquad_ard_3d", "fp32"): (5e-7, 5e-4),
}


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x3", "fp32"])
@pytest.mark.parametrize("name,n,d,kernel,ard,rank,s2", NYS_CASES)
def test_nystrom_estimator_matches_oracle(name, n, d, kernel, ard, rank, s2, precision):
    lp_tol, g_tol = (1e-7, 1e-5) if precision == "fp64" else NYS_BARS[(name, precision)]
    pr, S = _nys_case(n, d, kernel, ard, rank, s2)
    out = run_nystrom(pr, precision, rank, S)
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, kernel, ard, rank, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed, grad=True, precond="nystrom", landmarks=S)
    say(f"    logp {out['logp']:.12e} oracle {ref['logp']:.12e} rel {rel(out['logp'], ref['logp']):.2e}; "
        f"grad rel {relvec(out['grad'], ref['grad']):.2e}")
    assert rel(out["logp"], ref["logp"]) < lp_tol
    assert relvec(out["grad"], ref["grad"]) < g_tol
    assert out["stats"].flags & B.FLAG_NOT_CONVERGED == 0
    if precision == "fp64":
        assert abs(out["stats"].iters_max - int(ref["iters"].max())) <= 1 + 0.05 * int(ref["iters"].max())


@pytest.mark.parametrize("mode", [0, 1])
def test_nystrom_precond_grad_modes_match_oracle(mode):
    pr, S = _nys_case(1100, 6, "matern32", True, 24, 0.1, seed=36)
    out = run_nystrom(pr, "fp64", 24, S, precond_grad=mode)
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, "matern32", True, 24, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed, grad=True, precond_grad=mode, precond="nystrom", landmarks=S)
    assert relvec(out["grad"], ref["grad"]) < 1e-5
    assert rel(out["logp"], ref["logp"]) < 1e-7


def test_nystrom_stops_on_a_duplicate_landmark_point():
    pr, _ = _nys_case(600, 2, "rbf", True, 4, 0.1, seed=37)
    pr.X[5] = pr.X[2]
    S = np.array([2, 5, 7, 9], dtype=np.int32)
    out = run_nystrom(pr, "fp64", 4, S)
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, "rbf", True, 4, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed, grad=True, precond="nystrom", landmarks=S)
    assert ref["rank"] == 1
    assert out["stats"].rank_achieved == 1
    assert out["stats"].flags & B.FLAG_RANK_DEFICIENT
    np.testing.assert_array_equal(out["piv"], [2, -1, -1, -1])
    assert rel(out["logp"], ref["logp"]) < 1e-7
    assert relvec(out["grad"], ref["grad"]) < 1e-5


def test_nystrom_rejects_bad_landmarks():
    pr, _ = _nys_case(200, 2, "rbf", True, 4, 0.1, seed=38)
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, "rbf", True)
    opt = B.make_options("fp64", 4, 50)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, 4))
    for S in ([1, 2, 2, 3], [1, 2, 3, 200], [-1, 2, 3, 4]):
        with pytest.raises(B.GPError):
            B.gp_precond_build_nystrom(prob, pr.theta, 4, S, ws)


# ---------------------------------------------------------------- quadrature Fourier features

# A q-point rule resolves cos(w . delta) only for |delta| up to about sqrt(q), so
# the cases keep the scaled inputs compact (longer lengthscales in 2-D and 3-D).
# Noise levels keep K_hat's condition number within what BF16x3 tiles resolve
# (their relative product error ~1e-5 times the condition number bounds the
# solves; a 1-D set of 1500 points at sigma^2 = 0.01 exceeds the gradient bar).
QFF_CASES = [
    # name, n, d, ard, q (rank q^d), sigma^2, lengthscale range; CG iterations of the oracle
    ("rbf_1d", 1500, 1, False, 8, 0.05, (0.4, 1.5)),      # 27
    ("rbf_ard_2d", 1200, 2, True, 6, 0.05, (1.0, 2.0)),   # 25
    ("rbf_ard_3d", 900, 3, True, 4, 0.1, (1.0, 2.0)),     # 77
]


def run_qff(pr, precision, q, precond_grad=0, grad=True):
    rank = q ** pr.d
    say(f"[gpu] qff estimator {pr.name} n={pr.n} d={pr.d} ard={pr.ard} prec={precision} q={q} rank={rank}")
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    prob = B.make_problem(X, y, "rbf", pr.ard)
    opt = B.make_options(precision, pr.num_probes, pr.max_iters, pr.tol, pr.probe_seed, precond_grad, 1)
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank))
    h = B.gp_precond_build_qff(prob, pr.theta, q, ws)
    logp = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(len(pr.theta), dtype=torch.float64, device=dev)
    st = B.Stats(pr.num_probes, rank)
    try:
        if grad:
            B.gp_mll_grad(prob, pr.theta, opt, rank, h, ws, logp, g, st)
        else:
            B.gp_mll_eval(prob, pr.theta, opt, rank, h, ws, logp, st)
        torch.cuda.synchronize()
        v = B.gp_precond_view_of(h)
        n = pr.n
        Wg = np.frombuffer(ws.cpu().numpy().tobytes(), dtype=np.uint8)
        base = ws.data_ptr()
        Z = Wg[v.L_dev - base: v.L_dev - base + n * rank * 8].view(np.float64).reshape(rank, n).T
        ldp = float(Wg[v.logdet_dev - base: v.logdet_dev - base + 8].view(np.float64)[0])
    finally:
        B.gp_precond_free(h)
    return {"logp": float(logp.cpu()[0]), "grad": g.cpu().numpy(), "stats": st, "Z": Z, "logdet_P": ldp}


def _qff_case(n, d, ard, q, s2, ls, seed=39):
    return synthgp.random_problem(n, d, "rbf", ard=ard, rank=q ** d, num_probes=8, seed=seed,
                                  ls_range=ls, sigma2=s2, dist="normal", tol=1e-8, max_iters=400)


@pytest.mark.parametrize("name,n,d,ard,q,s2,ls", QFF_CASES)
def test_qff_features_match_oracle(name, n, d, ard, q, s2, ls):
    pr = _qff_case(n, d, ard, q, s2, ls)
    out = run_qff(pr, "fp64", q, grad=False)
    f, w = go.qff_frequencies(d, q)
    Zr = go.rff_features(pr.X, pr.theta, ard, f, w)
    np.testing.assert_allclose(out["Z"], Zr, rtol=0, atol=1e-12)
    assert rel(out["logdet_P"], go.Preconditioner(Zr, pr.theta[-1]).logdet) < 1e-11


# same-probe bars per case, about five times the measured distance (as RFF_BARS)
QFF_BARS = {
    ("rbf_1d", "bf16x3"): (5e-4, 1e-2), ("rbf_1d", "fp16x3"): (5e-5, 5e-3),
    ("rbf_ard_2d", "bf16x3"): (5e-4, 5e-4), ("rbf_ard_2d", "fp16x3"): (5e-4, 1e-3),
    ("rbf_ard_3d", "bf16x3"): (1e-5, 2e-4), ("rbf_ard_3d", "fp16x3"): (2e-6, 5e-4),
}


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("name,n,d,ard,q,s2,ls", QFF_CASES)
def test_qff_estimator_matches_oracle(name, n, d, ard, q, s2, ls, precision):
    lp_tol, g_tol = (1e-7, 1e-5) if precision == "fp64" else QFF_BARS[(name, precision)]
    pr = _qff_case(n, d, ard, q, s2, ls)
    out = run_qff(pr, precision, q)
    ref = go.estimate_mll(pr.X, pr.y, pr.theta, "rbf", ard, q ** d, pr.num_probes, pr.tol, pr.max_iters,
                          pr.probe_seed, grad=True, precond="qff", qff_nodes=q)
    say(f"    logp {out['logp']:.12e} oracle {ref['logp']:.12e} rel {rel(out['logp'], ref['logp']):.2e}; "
        f"grad rel {relvec(out['grad'], ref['grad']):.2e}; iters {out['stats'].iters_max} / {ref['iters'].max()}")
    assert rel(out["logp"], ref["logp"]) < lp_tol
    assert relvec(out["grad"], ref["grad"]) < g_tol
    assert out["stats"].flags & B.FLAG_NOT_CONVERGED == 0


def test_qff_rejects_bad_arguments():
    pr = _qff_case(300, 2, True, 4, 0.1, (1.0, 2.0))
    dev = torch.device("cuda:0")
    X = torch.tensor(pr.X, device=dev)
    y = torch.tensor(pr.y, device=dev)
    ws = B.alloc_workspace(B.gp_workspace_size(B.make_problem(X, y, "rbf", True), B.make_options("fp64", 4, 50), 64))
    for q in (3, 0, 66):
        with pytest.raises(B.GPError):
            B.gp_precond_build_qff(B.make_problem(X, y, "rbf", True), pr.theta, q, ws)
    with pytest.raises(B.GPError):
        B.gp_precond_build_qff(B.make_problem(X, y, "matern32", True), pr.theta, 4, ws)
