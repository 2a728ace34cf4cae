"""Preconditioned GP log-marginal-likelihood estimator on AMD MI355X (gfx950).

The compute path is the HIP library libgpmll.so (C-ABI in include/gpmll.h);
`binding` marshals arguments to it and `model` wraps it as a
torch.autograd.Function.  Build the library with
`python -m paper_2107_00243_amd.build`.
"""
from . import binding  # noqa: F401  (loading the library itself is lazy)

__all__ = ["binding"]
