"""Write the full-size oracle references of the GPU parity tests.

    python tests/golden/make_full_size.py matern52_ard_20k   # dense, about 10 minutes
    python tests/golden/make_full_size.py rbf_ard_100k       # matrix-free, about an hour
    python tests/golden/make_full_size.py batched_rbf_64     # 64 dense problems

Calls only the CPU oracle (oracle/gp_oracle.py) on the seeded inputs of synthgp;
nothing here touches the GPU library.  Each run writes one JSON file next to this
script with the same-probe stochastic estimate of Algorithms 1 and 2 (the
preconditioned log p and gradient estimator of Section 4.4, readings as in the
oracle's header) and, where a dense Cholesky factor fits in memory, the exact
Eq. (1) and Eq. (2) targets.  Wall time and thread count of the oracle run are
recorded beside the numbers.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthgp  # noqa: E402
from oracle import gp_oracle as go  # noqa: E402


def _estimate(pr, dense, workers):
    t0 = time.time()
    est = go.estimate_mll(pr.X, pr.y, pr.theta, pr.kernel, pr.ard, pr.rank, pr.num_probes, pr.tol,
                          pr.max_iters, pr.probe_seed, grad=True, dense=dense, workers=workers,
                          native=not dense)
    dt = time.time() - t0
    return {
        "logp": est["logp"], "grad": est["grad"].tolist(), "datafit": est["datafit"],
        "logdet_estimate": est["logdet_est"], "logdet_precond": est["logdet_P"],
        "gammas": est["gammas"].tolist(), "col_iters": est["iters"].tolist(),
        "pivots": est["piv"][:est["rank"]].tolist(), "rank_achieved": int(est["rank"]),
        "rel_residual": est["rel_resid"].tolist(), "seconds": dt,
    }


def _exact(pr):
    t0 = time.time()
    ex = go.exact_mll(pr.X, pr.y, pr.theta, pr.kernel, pr.ard, grad=True)
    return {"logp": ex["logp"], "grad": ex["grad"].tolist(), "datafit": ex["datafit"], "logdet": ex["logdet"],
            "seconds": time.time() - t0}


def batch_main(name, workers):
    """The ragged batch: problem b of the batch with probe seed probe_seed + b and
    rank min(rank, n_b), as the batched entry points evaluate it."""
    probs = getattr(synthgp, name)()
    rec = {"workload": name, "source": "oracle/gp_oracle.py estimate_mll and exact_mll, FP64, dense",
           "host": {"cpu": platform.processor() or platform.machine(), "threads": workers,
                    "numpy": np.__version__}, "problems": []}
    for b, pr in enumerate(probs):
        t0 = time.time()
        est = go.estimate_mll(pr.X, pr.y, pr.theta, pr.kernel, pr.ard, min(pr.rank, pr.n), pr.num_probes, pr.tol,
                              pr.max_iters, pr.probe_seed + b, grad=True, dense=True)
        ex = go.exact_mll(pr.X, pr.y, pr.theta, pr.kernel, pr.ard, grad=True)
        rec["problems"].append({
            "n": pr.n, "theta": pr.theta.tolist(), "rank": min(pr.rank, pr.n), "num_probes": pr.num_probes,
            "tol": pr.tol, "max_iters": pr.max_iters, "probe_seed": pr.probe_seed + b,
            "estimate": {"logp": est["logp"], "grad": est["grad"].tolist(), "col_iters": est["iters"].tolist()},
            "exact": {"logp": ex["logp"], "grad": ex["grad"].tolist(), "datafit": ex["datafit"],
                      "logdet": ex["logdet"]},
            "seconds": time.time() - t0})
        print(f"[golden] {name} problem {b} n={pr.n}: log p {est['logp']:.10g} (exact {ex['logp']:.10g}), "
              f"CG {int(est['iters'].max())}, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, f"oracle_{name}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out)


def main(name):
    workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if name.startswith("batched"):
        return batch_main(name, workers)
    pr = getattr(synthgp, name)()
    rec = {
        "workload": name, "recipe": pr.recipe, "n": pr.n, "d": pr.d, "kernel": pr.kernel, "ard": pr.ard,
        "theta": pr.theta.tolist(), "rank": pr.rank, "num_probes": pr.num_probes, "tol": pr.tol,
        "max_iters": pr.max_iters, "probe_seed": pr.probe_seed,
        "source": "oracle/gp_oracle.py estimate_mll (Algorithms 1 and 2) and exact_mll (Eq. 1, Eq. 2), FP64",
        "host": {"cpu": platform.processor() or platform.machine(), "threads": workers,
                 "numpy": np.__version__},
    }
    dense = pr.n <= 20000
    print(f"[golden] {name}: n={pr.n} estimate ({'dense' if dense else 'matrix-free, plain C'}, "
          f"{workers} threads)",
          flush=True)
    rec["estimate"] = _estimate(pr, dense, workers)
    print(f"[golden] estimate logp {rec['estimate']['logp']:.12g} in {rec['estimate']['seconds']:.0f} s", flush=True)
    if dense:
        print(f"[golden] {name}: exact (dense Cholesky)", flush=True)
        rec["exact"] = _exact(pr)
        print(f"[golden] exact logp {rec['exact']['logp']:.12g} in {rec['exact']['seconds']:.0f} s", flush=True)
    out = os.path.join(HERE, f"oracle_{name}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out)


if __name__ == "__main__":
    main(sys.argv[1])
