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

Both stop early on a held-out validation set (Sec. 5) when given `validate`, a
function theta -> loss (model.validation_score builds one from gp_predict): the
loss is taken at the starting theta and after every step, the run ends once
`patience` steps in a row have not lowered the best loss so far, and the theta
returned is the one with the lowest validation loss, not the last iterate.

    python -m paper_2107_00243_amd.train --workload gmm_matern32_300k --steps 20 \
        --precision bf16x3 --lr 0.1 --checkpoint run.npz
    python -m paper_2107_00243_amd.train --optimizer lbfgs --workload matern52_ard_20k --steps 20 \
        --validation-fraction 0.1
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from .model import GPMLL, GPMarginalLikelihood, validation_score


def save_checkpoint(path, step, log_theta, opt, history, early=None):
    st = opt.state[log_theta] if log_theta in opt.state else {}
    np.savez(path + ".tmp.npz", step=step, log_theta=log_theta.detach().numpy(),
             exp_avg=st.get("exp_avg", torch.zeros_like(log_theta)).numpy(),
             exp_avg_sq=st.get("exp_avg_sq", torch.zeros_like(log_theta)).numpy(),
             adam_step=float(st.get("step", torch.tensor(0.0))), history=json.dumps(history),
             early=json.dumps(early))
    os.replace(path + ".tmp.npz", path)


def load_checkpoint(path, log_theta, opt):
    z = np.load(path, allow_pickle=False)
    with torch.no_grad():
        log_theta.copy_(torch.from_numpy(z["log_theta"]))
    if float(z["adam_step"]) > 0:
        opt.state[log_theta] = {"step": torch.tensor(float(z["adam_step"])),
                                "exp_avg": torch.from_numpy(z["exp_avg"]),
                                "exp_avg_sq": torch.from_numpy(z["exp_avg_sq"])}
    early = json.loads(str(z["early"])) if "early" in z.files else None
    return int(z["step"]), json.loads(str(z["history"])), early


class EarlyStopping:
    """Best-so-far tracking of a validation loss with a patience in steps."""

    def __init__(self, validate, patience):
        if patience < 1:
            raise ValueError("patience must be at least 1")
        self.validate, self.patience = validate, int(patience)
        self.best, self.best_theta, self.bad, self.stopped = float("inf"), None, 0, False

    def update(self, theta):
        """Record the loss at theta; returns it and whether the run should stop."""
        loss = float(self.validate(theta))
        if loss < self.best:
            self.best, self.best_theta, self.bad = loss, np.array(theta, dtype=np.float64), 0
        else:
            self.bad += 1
        self.stopped = self.bad >= self.patience
        return loss, self.stopped

    def state(self):
        return {"best": self.best, "bad": self.bad, "stopped": self.stopped,
                "best_theta": None if self.best_theta is None else self.best_theta.tolist()}

    def restore(self, st):
        if st is None:
            return
        self.best, self.bad, self.stopped = float(st["best"]), int(st["bad"]), bool(st["stopped"])
        self.best_theta = None if st["best_theta"] is None else np.array(st["best_theta"], dtype=np.float64)


def _start_early(validate, patience, theta0, saved, resumed, log, tag):
    if validate is None:
        return None
    es = EarlyStopping(validate, patience)
    if resumed:
        es.restore(saved)
    if es.best_theta is None:
        loss, _ = es.update(theta0)
        log(f"[{tag}] validation loss at the start: {loss:.6f}")
    return es


def adam_fit(model: GPMarginalLikelihood, theta0, steps=20, lr=0.1, checkpoint=None, resume=False, log=print,
             validate=None, patience=2):
    """Maximise the log-likelihood estimate over log theta with Adam; returns the
    history and the final theta (with `validate`: the theta of lowest validation
    loss, the run ending after `patience` steps without a new best)."""
    log_theta = torch.tensor(np.log(np.asarray(theta0, dtype=np.float64)), requires_grad=True)
    opt = torch.optim.Adam([log_theta], lr=lr)
    history, start, saved, resumed = [], 0, None, False
    if resume and checkpoint and os.path.exists(checkpoint):
        start, history, saved = load_checkpoint(checkpoint, log_theta, opt)
        resumed = True
    es = _start_early(validate, patience, np.exp(log_theta.detach().numpy()), saved, resumed, log, "adam")
    for step in range(start, steps):
        if es is not None and es.stopped:
            break
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
        if es is not None:
            rec["validation"], _ = es.update(np.exp(log_theta.detach().numpy()))
        history.append(rec)
        log(f"[adam] step {step}: logp {rec['logp']:.6f} ({rec['seconds']:.2f} s)"
            + (f", validation {rec['validation']:.6f}" if es is not None else ""))
        if checkpoint:
            save_checkpoint(checkpoint, step + 1, log_theta, opt, history, es.state() if es else None)
    if es is not None:
        if es.stopped:
            log(f"[adam] stopped early: {es.patience} steps without a lower validation loss")
        return history, es.best_theta
    return history, np.exp(log_theta.detach().numpy())


def lbfgs_fit(model: GPMarginalLikelihood, theta0, steps=20, lr=1.0, history_size=10, checkpoint=None,
              resume=False, log=print, max_ls_evals=20, validate=None, patience=2):
    """Maximise the log-likelihood estimate over log theta with L-BFGS (strong Wolfe
    line search), at most `steps` iterations; returns the per-iteration history and
    the final theta (with `validate`: the theta of lowest validation loss, the run
    ending after `patience` iterations without a new best)."""
    log_theta = torch.tensor(np.log(np.asarray(theta0, dtype=np.float64)), requires_grad=True)
    history, start, saved, resumed = [], 0, None, False
    if resume and checkpoint and os.path.exists(checkpoint):
        z = np.load(checkpoint, allow_pickle=False)
        with torch.no_grad():
            log_theta.copy_(torch.from_numpy(z["log_theta"]))
        start, history = int(z["step"]), json.loads(str(z["history"]))
        saved = json.loads(str(z["early"])) if "early" in z.files else None
        resumed = True
    es = _start_early(validate, patience, np.exp(log_theta.detach().numpy()), saved, resumed, log, "lbfgs")
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
        if es is not None and es.stopped:
            break
        evals.clear()
        opt.step(closure)
        best = max(evals, key=lambda r: r["logp"])
        rec = {"step": it, "evaluations": len(evals), "logp": best["logp"],
               "seconds": float(sum(r["seconds"] for r in evals)),
               "theta": np.exp(log_theta.detach().numpy()).tolist(), "evals": list(evals)}
        if es is not None:
            rec["validation"], _ = es.update(np.exp(log_theta.detach().numpy()))
        history.append(rec)
        log(f"[lbfgs] iteration {it}: logp {best['logp']:.6f} ({len(evals)} evaluations, {rec['seconds']:.2f} s)"
            + (f", validation {rec['validation']:.6f}" if es is not None else ""))
        if checkpoint:
            np.savez(checkpoint + ".tmp.npz", step=it + 1, log_theta=log_theta.detach().numpy(),
                     history=json.dumps(history), early=json.dumps(es.state() if es else None))
            os.replace(checkpoint + ".tmp.npz", checkpoint)
        if len(evals) == 1:
            # one evaluation and no line search: the gradient is below tolerance_grad
            break
    if es is not None:
        if es.stopped:
            log(f"[lbfgs] stopped early: {es.patience} iterations without a lower validation loss")
        return history, es.best_theta
    return history, np.exp(log_theta.detach().numpy())


def split_validation(X, y, fraction, seed):
    """A seeded random split of (X, y) into training and validation points."""
    n = len(y)
    nv = int(round(fraction * n))
    if not 0 < nv < n:
        raise ValueError(f"validation fraction {fraction} leaves no training or no validation points")
    perm = np.random.default_rng(seed).permutation(n)
    tr, va = np.sort(perm[nv:]), np.sort(perm[:nv])
    return X[tr], y[tr], X[va], y[va]


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
    ap.add_argument("--validation-fraction", type=float, default=0.0,
                    help="hold out this fraction of the points for early stopping (0: none)")
    ap.add_argument("--validation-metric", choices=("rmse", "nll"), default="rmse")
    ap.add_argument("--patience", type=int, default=2)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synthgp
    gen = getattr(synthgp, args.workload)
    pr = gen(n=args.n) if args.n else gen()
    X, y, validate = pr.X, pr.y, None
    if args.validation_fraction > 0:
        X, y, Xv, yv = split_validation(pr.X, pr.y, args.validation_fraction, pr.probe_seed)
    model = GPMarginalLikelihood(X, y, pr.kernel, pr.ard, pr.rank, pr.num_probes, pr.max_iters, pr.tol,
                                 args.precision, pr.probe_seed)
    model.want_stats = True
    if args.validation_fraction > 0:
        validate = validation_score(model, Xv, yv, args.validation_metric)
        print(f"[{args.optimizer}] {len(yv)} validation points ({args.validation_metric}), patience "
              f"{args.patience}", flush=True)
    print(f"[{args.optimizer}] {pr.name}: n={len(y)} training points of {pr.n}, d={pr.d} {pr.kernel} rank={pr.rank} "
          f"probes={pr.num_probes} "
          f"max_iters={pr.max_iters} precision={args.precision}", flush=True)
    fit = adam_fit if args.optimizer == "adam" else lbfgs_fit
    lr = args.lr if args.optimizer == "adam" or args.lr != 0.1 else 1.0
    hist, theta = fit(model, pr.theta, args.steps, lr, checkpoint=args.checkpoint, resume=args.resume,
                      log=lambda m: print(m, flush=True), validate=validate, patience=args.patience)
    print(json.dumps({"workload": pr.name, "steps": len(hist), "logp_first": hist[0]["logp"],
                      "logp_last": hist[-1]["logp"], "seconds_per_step": float(np.mean([h["seconds"] for h in hist])),
                      "theta": theta.tolist()}), flush=True)


if __name__ == "__main__":
    main()
