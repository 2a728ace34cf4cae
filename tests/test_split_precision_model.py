"""A CPU model of the split-precision K_hat V products inside the estimator's
preconditioned CG (the oracle's pcg_block with a product that rounds like the
BF16x3 tiles), on the n = 100,000 RBF recipe cut to 2,500 points.  It checks the
reason for the design of the BF16x3 tiles: rounding the kernel values to hi + lo
bfloat16 halves leaves the CG iteration count alone, rounding the search
directions to hi + lo delays CG, and a third bfloat16 piece of the directions in
the first iterations restores the FP64 count.  (The HIP tiles accumulate in FP32
in a different order; the model keeps FP64 sums to isolate the roundings.)"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import synthgp
from oracle import gp_oracle as go


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as FP64."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def pieces(x, k):
    out, r = [], np.asarray(x, dtype=np.float64)
    for _ in range(k):
        p = bf16(r)
        out.append(p)
        r = r - p
    return sum(out)


@pytest.fixture(scope="module")
def setup():
    pr = synthgp.rbf_ard_100k(n=2500)
    n, d = pr.n, pr.d
    Xs = pr.X / pr.theta[:d]
    K = np.exp(-0.5 * cdist(Xs, Xs, "sqeuclidean"))
    s2 = pr.theta[-1]
    L, piv, kp = go.pivoted_cholesky(pr.X, pr.theta, pr.kernel, pr.ard, 20)
    P = go.Preconditioner(L[:, :kp], s2)
    E, H = go.probe_signs(pr.probe_seed, n, 20, 16)
    B = math.sqrt(s2) * E + L @ H[:20]
    rhs = np.concatenate([pr.y[:, None], B], axis=1)
    return K, s2, P, rhs


def iterations(setup, k_pieces, v_pieces, v3_iters=0):
    K, s2, P, rhs = setup
    Kr = K if k_pieces is None else pieces(np.asarray(K, dtype=np.float32), k_pieces)
    calls = [0]

    def matvec(V):
        calls[0] += 1
        vp = 3 if calls[0] <= v3_iters else v_pieces
        Vr = V if vp is None else pieces(V, vp)
        return Kr @ Vr + s2 * V

    _, coeffs, _, _ = go.pcg_block(matvec, rhs, P.solve, 1e-6, 200)
    return max(len(a) for a, _ in coeffs)


def test_direction_rounding_delays_cg_and_a_third_piece_restores_it(setup):
    exact = iterations(setup, None, None)
    k_only = iterations(setup, 2, None)        # kernel values hi + lo, exact directions
    v_only = iterations(setup, None, 2)        # exact kernel values, directions hi + lo
    both = iterations(setup, 2, 2)             # BF16x3 with two-piece directions
    v3 = iterations(setup, 2, 3)               # three-piece directions throughout
    early = iterations(setup, 2, 2, v3_iters=8)  # three pieces in the first iterations only
    assert k_only == exact
    assert v_only > exact and both > exact
    assert v3 == exact and early == exact
