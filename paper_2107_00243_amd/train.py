"""Hyperparameter optimisation on log-parameters through GPMLL.

Each evaluation is one gp_mll_grad call (the preconditioner is rebuilt for the
new theta) giving the preconditioned estimate of log p and its gradient.  Two
optimisers:

* Adam (the paper's ablation, Sec. 5 and Table S2): one torch.optim.Adam step on
  log theta per evaluation.  A checkpoint (theta, Adam moments, step, history)
  is written after every step and can be resumed.
* L-BFGS with a line search satisfying the strong Wolfe conditions (the
  paper's optimiser for its UCI runs, Sec. 5: at most 20 iterations).  The
  probes are fixed by the seed, so every evaluation sees the same random
  numbers and the objective is deterministic in theta, as a line search needs.
  A checkpoint keeps theta and the history after every iteration; a resumed
  run restarts the curvature memory from the saved theta.

    python -m paper_2107_00243_amd.train --workload gmm_matern32_300k --steps 20 \
        --precision bf16x3 --lr 0.1 --checkpoint run.npz
    python -m paper_2107_00243_amd.train --optimizer lbfgs --workload matern52_ard_20k --steps 20
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


def lbfgs_fit(model: GPMarginalLikelihood, theta0, steps=20, lr=1.0, history_size=10, checkpoint=None,
              resume=False, log=print, max_ls_evals=20):
    """Maximise the log-likelihood estimate over log theta with L-BFGS (strong Wolfe
    line search), at most `steps` iterations; returns the per-evaluation history and
    the final theta."""
    log_theta = torch.tensor(np.log(np.asarray(theta0, dtype=np.float64)), requires_grad=True)
    history, start = [], 0
    if resume and checkpoint and os.path.exists(checkpoint):
        z = np.load(checkpoint, allow_pickle=False)
        with torch.no_grad():
            log_theta.copy_(torch.from_numpy(z["log_theta"]))
        start, history = int(z["step"]), json.loads(str(z["history"]))
    # one optimiser iteration per step() call; max_eval bounds the evaluations of that
    # iteration, the line search's included (the default, 5/4 of max_iter, would
    # leave the line search no trial beyond the first)
    opt = torch.optim.LBFGS([log_theta], lr=lr, max_iter=1, max_eval=max_ls_evals + 1, history_size=history_size,
                            line_search_fn="strong_wolfe", tolerance_grad=1e-9, tolerance_change=1e-12)
    evals = []

    def closure():
        t0 = time.perf_counter()
        opt.zero_grad()
        logp = GPMLL.apply(model, log_theta)
        (-logp).backward()
        rec = {"logp": float(logp.detach()), "seconds": time.perf_counter() - t0,
               "theta": np.exp(log_theta.detach().numpy()).tolist()}
        st = model.last_stats
        if st is not None:
            rec["cg_iters"] = int(st.iters_max)
        evals.append(rec)
        return -logp

    for it in range(start, steps):
        evals.clear()
        opt.step(closure)
        best = max(evals, key=lambda r: r["logp"])
        rec = {"step": it, "evaluations": len(evals), "logp": best["logp"],
               "seconds": float(sum(r["seconds"] for r in evals)),
               "theta": np.exp(log_theta.detach().numpy()).tolist(), "evals": list(evals)}
        history.append(rec)
        log(f"[lbfgs] iteration {it}: logp {best['logp']:.6f} ({len(evals)} evaluations, {rec['seconds']:.2f} s)")
        if checkpoint:
            np.savez(checkpoint + ".tmp.npz", step=it + 1, log_theta=log_theta.detach().numpy(),
                     history=json.dumps(history))
            os.replace(checkpoint + ".tmp.npz", checkpoint)
        if len(evals) == 1:
            # one evaluation and no line search: the gradient is below tolerance_grad
            break
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
    ap.add_argument("--optimizer", choices=("adam", "lbfgs"), default="adam")
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
    print(f"[{args.optimizer}] {pr.name}: n={pr.n} d={pr.d} {pr.kernel} rank={pr.rank} probes={pr.num_probes} "
          f"max_iters={pr.max_iters} precision={args.precision}", flush=True)
    fit = adam_fit if args.optimizer == "adam" else lbfgs_fit
    lr = args.lr if args.optimizer == "adam" or args.lr != 0.1 else 1.0
    hist, theta = fit(model, pr.theta, args.steps, lr, checkpoint=args.checkpoint, resume=args.resume,
                      log=lambda m: print(m, flush=True))
    print(json.dumps({"workload": pr.name, "steps": len(hist), "logp_first": hist[0]["logp"],
                      "logp_last": hist[-1]["logp"], "seconds_per_step": float(np.mean([h["seconds"] for h in hist])),
                      "theta": theta.tolist()}), flush=True)


if __name__ == "__main__":
    main()
