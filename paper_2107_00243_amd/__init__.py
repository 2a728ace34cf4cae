"""Preconditioned GP log-marginal-likelihood estimator on AMD MI355X (gfx950).

The compute path is the HIP library libgpmll.so (C-ABI in include/gpmll.h);
`binding` marshals arguments to it, `model` wraps it as a torch.autograd.Function
and `train` drives Adam or L-BFGS through it.  Build the library with
`python -m paper_2107_00243_amd.build`.

Typical use (device tensors X (n x d, FP64) and y (n,)):

    from paper_2107_00243_amd import binding as B
    prob = B.make_problem(X, y, "rbf", ard=True)          # or "matern32", "matern52", "ratquad:<alpha>"
    opt = B.make_options("bf16x3", num_probes=64, max_iters=200, cg_tol=1e-6)  # or "fp16x3", "fp32", "fp64"
    ws = B.alloc_workspace(B.gp_workspace_size(prob, opt, rank=100))
    logp = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(len(theta), dtype=torch.float64, device="cuda")
    B.gp_mll_grad(prob, theta, opt, 100, None, ws, logp, grad)   # theta = [ls | s | sigma^2]

    # other preconditioners of Table 1: build a handle first and pass it instead of None
    h = B.gp_precond_build_nystrom(prob, theta, 100, landmarks, ws)
    # posterior mean and latent variance at test points Xs (m x d)
    B.gp_predict(prob, theta, opt, 100, None, Xs, ws, mean, var)
"""
from . import binding  # noqa: F401  (loading the library itself is lazy)

__all__ = ["binding"]
