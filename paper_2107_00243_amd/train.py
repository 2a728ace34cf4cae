"""Hyperparameter optimisation with Adam on log-parameters through GPMLL.

Each step evaluates the preconditioned estimate of log p and its gradient with
one gp_mll_grad call (the preconditioner is rebuilt for the new theta) and takes
one torch.optim.Adam step on log theta (the paper's Adam ablation, Sec. 5 and
Table S2, uses Adam on the same objective).  A checkpoint (theta, Adam moments,
step, history) is written after every step and can be resumed.

    python -m paper_2107_00243_amd.train --workload gmm_matern32_300k --steps 20 \
        --precision bf16x3 --lr 0.1 --checkpoint run.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from .model import GPMLL, GPMarginalLikelihood


def save_checkpoint(path, step, log_theta, opt, history):
    st = opt.state[log_theta] if log_theta in opt.state else {}
    np.savez(path + ".tmp.npz", step=step, log_theta=log_theta.detach().numpy(),
             exp_avg=st.get("exp_avg", torch.zeros_like(log_theta)).numpy(),
             exp_avg_sq=st.get("exp_avg_sq", torch.zeros_like(log_theta)).numpy(),
             adam_step=float(st.get("step", torch.tensor(0.0))), history=json.dumps(history))
    os.replace(path + ".tmp.npz", path)


def load_checkpoint(path, log_theta, opt):
    z = np.load(path, allow_pickle=False)
    with torch.no_grad():
        log_theta.copy_(torch.from_numpy(z["log_theta"]))
    if float(z["adam_step"]) > 0:
        opt.state[log_theta] = {"step": torch.tensor(float(z["adam_step"])),
                                "exp_avg": torch.from_numpy(z["exp_avg"]),
                                "exp_avg_sq": torch.from_numpy(z["exp_avg_sq"])}
    return int(z["step"]), json.loads(str(z["history"]))


def adam_fit(model: GPMarginalLikelihood, theta0, steps=20, lr=0.1, checkpoint=None, resume=False, log=print):
    """Maximise the log-likelihood estimate over log theta with Adam; returns the history."""
    log_theta = torch.tensor(np.log(np.asarray(theta0, dtype=np.float64)), requires_grad=True)
    opt = torch.optim.Adam([log_theta], lr=lr)
    history, start = [], 0
    if resume and checkpoint and os.path.exists(checkpoint):
        start, history = load_checkpoint(checkpoint, log_theta, opt)
    for step in range(start, steps):
        t0 = time.perf_counter()
        opt.zero_grad()
        logp = GPMLL.apply(model, log_theta)
        (-logp).backward()
        opt.step()
        st = model.last_stats
        rec = {"step": step, "logp": float(logp.detach()), "seconds": time.perf_counter() - t0,
               "theta": np.exp(log_theta.detach().numpy()).tolist()}
        if st is not None:
            rec["cg_iters"] = int(st.iters_max)
        history.append(rec)
        log(f"[adam] step {step}: logp {rec['logp']:.6f} ({rec['seconds']:.2f} s)")
        if checkpoint:
            save_checkpoint(checkpoint, step + 1, log_theta, opt, history)
    return history, np.exp(log_theta.detach().numpy())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="gmm_matern32_300k")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--lr", type=float, default=0.1)
    ap.add_argument("--precision", default="bf16x3")
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--resume", action="store_true")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synthgp
    gen = getattr(synthgp, args.workload)
    pr = gen(n=args.n) if args.n else gen()
    model = GPMarginalLikelihood(pr.X, pr.y, pr.kernel, pr.ard, pr.rank, pr.num_probes, pr.max_iters, pr.tol,
                                 args.precision, pr.probe_seed)
    model.want_stats = True
    print(f"[adam] {pr.name}: n={pr.n} d={pr.d} {pr.kernel} rank={pr.rank} probes={pr.num_probes} "
          f"max_iters={pr.max_iters} precision={args.precision}", flush=True)
    hist, theta = adam_fit(model, pr.theta, args.steps, args.lr, args.checkpoint, args.resume,
                           log=lambda m: print(m, flush=True))
    print(json.dumps({"workload": pr.name, "steps": len(hist), "logp_first": hist[0]["logp"],
                      "logp_last": hist[-1]["logp"], "seconds_per_step": float(np.mean([h["seconds"] for h in hist])),
                      "theta": theta.tolist()}), flush=True)


if __name__ == "__main__":
    main()
