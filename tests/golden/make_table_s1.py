"""Write the exact targets of the Table S1 experiment (supplement, synthetic data).

    python tests/golden/make_table_s1.py      # nine dense problems, n = 10,000

For each kernel (Matern-3/2, RBF, rational quadratic) and d in {1, 2, 3}, the
problem of synthgp.table_s1 and its exact log p (Eq. 1) and gradient (Eq. 2) from
the CPU oracle's dense FP64 Cholesky factorisation, into table_s1_exact.json next
to this script.  Calls only the oracle.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthgp  # noqa: E402
from oracle import gp_oracle as go  # noqa: E402


def main():
    out = {"source": "oracle/gp_oracle.py exact_mll (Eq. 1, Eq. 2), dense FP64 Cholesky", "problems": {}}
    for kernel in synthgp.TABLE_S1_KERNELS:
        for d in (1, 2, 3):
            pr = synthgp.table_s1(kernel, d)
            t0 = time.time()
            ex = go.exact_mll(pr.X, pr.y, pr.theta, pr.kernel, pr.ard, grad=True)
            out["problems"][pr.name] = {"kernel": kernel, "d": d, "n": pr.n, "theta": pr.theta.tolist(),
                                        "recipe": pr.recipe, "logp": ex["logp"], "grad": ex["grad"].tolist(),
                                        "datafit": ex["datafit"], "logdet": ex["logdet"]}
            print(f"[golden] {pr.name}: log p {ex['logp']:.12g} in {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, "table_s1_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
