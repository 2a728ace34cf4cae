"""Exact-GP marginal likelihood on the HIP library, as a torch.autograd.Function.

GPMarginalLikelihood holds the device copies of X and y, one workspace and the
estimator options; GPMLL.apply(model, log_theta) returns the estimate of
log p(y | theta) with theta = exp(log_theta), and its backward returns
grad_log_theta = theta * d log p / d theta from the same library call (the
forward solves are reused; the derivative sweep runs once per evaluation).
When log_theta does not require a gradient, only the estimate is computed.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class GPMarginalLikelihood:
    def __init__(self, X, y, kernel="rbf", ard=True, rank=100, num_probes=64, max_iters=200, cg_tol=1e-6,
                 precision="bf16x3", seed=1, precond_grad=0, sync_every=1, device="cuda"):
        self.X = torch.as_tensor(X, dtype=torch.float64).to(device).contiguous()
        self.y = torch.as_tensor(y, dtype=torch.float64).to(device).contiguous()
        self.kernel, self.ard, self.rank = kernel, bool(ard), int(rank)
        self.prob = B.make_problem(self.X, self.y, kernel, ard)
        self.opt = B.make_options(precision, num_probes, max_iters, cg_tol, seed, precond_grad, sync_every)
        self.ws = B.alloc_workspace(B.gp_workspace_size(self.prob, self.opt, self.rank), device)
        self.num_params = (self.X.shape[1] if ard else 1) + 2
        self.logp = torch.zeros(1, dtype=torch.float64, device=device)
        self.grad = torch.zeros(self.num_params, dtype=torch.float64, device=device)
        self.last_stats = None
        self.want_stats = False

    def evaluate(self, theta, with_grad=True, stats=False):
        """log p (and the gradient w.r.t. natural theta) as device tensors."""
        theta = np.asarray(theta, dtype=np.float64)
        st = B.Stats(self.opt.num_probes, self.rank) if stats else None
        if with_grad:
            B.gp_mll_grad(self.prob, theta, self.opt, self.rank, None, self.ws, self.logp, self.grad, st)
        else:
            B.gp_mll_eval(self.prob, theta, self.opt, self.rank, None, self.ws, self.logp, st)
        self.last_stats = st
        return self.logp, (self.grad if with_grad else None)

    def predict(self, theta, Xstar, with_var=False):
        """Posterior mean (and latent variance) at the rows of Xstar (nstar x d),
        as FP64 NumPy arrays, from gp_predict with this model's options."""
        theta = np.asarray(theta, dtype=np.float64)
        Xs = torch.as_tensor(Xstar, dtype=torch.float64).to(self.X.device).contiguous()
        mean = torch.zeros(Xs.shape[0], dtype=torch.float64, device=self.X.device)
        var = torch.zeros_like(mean) if with_var else None
        B.gp_predict(self.prob, theta, self.opt, self.rank, None, Xs, self.ws, mean, var)
        return mean.cpu().numpy(), (var.cpu().numpy() if with_var else None)


def validation_score(model, Xv, yv, metric="rmse"):
    """A function theta -> loss on a held-out set (lower is better), for early
    stopping: "rmse" is the root mean squared error of the posterior mean;
    "nll" the mean negative log density of yv under N(mean, var + sigma^2),
    which needs the predictive variance (one CG solve per chunk of
    num_probes validation points instead of one in all)."""
    yv = np.asarray(yv, dtype=np.float64)
    if metric not in ("rmse", "nll"):
        raise ValueError(f"unknown validation metric {metric!r}")

    def score(theta):
        mean, var = model.predict(theta, Xv, with_var=(metric == "nll"))
        if metric == "rmse":
            return float(np.sqrt(np.mean((mean - yv) ** 2)))
        v = np.maximum(var, 0.0) + float(theta[-1])
        return float(np.mean(0.5 * np.log(2.0 * np.pi * v) + 0.5 * (yv - mean) ** 2 / v))
    return score


class GPMLL(torch.autograd.Function):
    """log p(y | exp(log_theta)); log_theta is a CPU FP64 tensor of length p + 2."""

    @staticmethod
    def forward(ctx, model: GPMarginalLikelihood, log_theta: torch.Tensor):
        theta = torch.exp(log_theta.detach().to(torch.float64).cpu())
        if ctx.needs_input_grad[1]:
            # log p and its gradient from one library call (the derivative sweep
            # reuses the forward solves)
            logp, grad = model.evaluate(theta.numpy(), with_grad=True, stats=model.want_stats)
            ctx.save_for_backward(theta * grad.detach().cpu())
        else:
            logp, _ = model.evaluate(theta.numpy(), with_grad=False, stats=model.want_stats)
        return logp.detach().cpu().reshape(())

    @staticmethod
    def backward(ctx, gout):
        (glog,) = ctx.saved_tensors
        return None, gout * glog
