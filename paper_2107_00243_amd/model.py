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
