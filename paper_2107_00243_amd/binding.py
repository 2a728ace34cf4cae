"""ctypes binding of libgpmll.so (declarations in include/gpmll.h).

Argument marshalling only: every step of the estimator runs in the HIP library.
Functions keep the C names; device buffers are torch CUDA tensors, the stream is
torch's current stream unless one is given.  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GPMLL_LIB selects another build of the library (the host-sanitizer build, say)
LIB_PATH = os.environ.get("GPMLL_LIB") or os.path.join(HERE, "libgpmll.so")

GP_OK, GP_EINVAL, GP_EWORKSPACE, GP_ENOTSPD, GP_EHIP, GP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
KERNELS = {"rbf": 0, "matern32": 1, "matern52": 2, "ratquad": 3}


def kernel_id(kernel: str):
    """gp_kernel id and shape of a kernel name ("ratquad:<alpha>" carries the shape)."""
    name, _, shape = kernel.partition(":")
    if name not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}")
    return KERNELS[name], (float(shape) if shape else 1.0)
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
FLAG_NOT_CONVERGED, FLAG_RANK_DEFICIENT, FLAG_RITZ_CLAMPED = 1, 2, 4
MAX_D, MAX_PROBES, MAX_RANK = 32, 255, 1024

BATCH_MAX_RANK, BATCH_MAX_PROBES = 256, 64

EXPORTS = ("gp_workspace_size", "gp_precond_build", "gp_precond_build_nystrom", "gp_precond_build_rff",
           "gp_precond_build_qff", "gp_precond_view_of", "gp_predict",
           "gp_precond_free",
           "gp_mll_eval", "gp_mll_grad", "gp_khat_matvec", "gp_khat_matvec_noalloc", "gp_khat_profile",
           "gp_batch_workspace_size",
           "gp_batch_mll_eval", "gp_batch_mll_grad", "gp_strerror", "gp_last_hip_error")


class gp_problem(ctypes.Structure):
    _fields_ = [("X_dev", ctypes.c_void_p), ("y_dev", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("d", ctypes.c_int32), ("kernel", ctypes.c_int32), ("ard", ctypes.c_int32),
                ("kernel_shape", ctypes.c_double)]


class gp_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("num_probes", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("cg_tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("precond_grad", ctypes.c_int32),
                ("sync_every", ctypes.c_int32), ("probe_mode", ctypes.c_int32)]


class gp_stats(ctypes.Structure):
    _fields_ = [("num_columns", ctypes.c_int32), ("iters_max", ctypes.c_int32), ("rank_achieved", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("ritz_clamped", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("logdet_precond", ctypes.c_double), ("datafit", ctypes.c_double),
                ("logdet_estimate", ctypes.c_double), ("col_iters_host", ctypes.POINTER(ctypes.c_int32)),
                ("gammas_host", ctypes.POINTER(ctypes.c_double)),
                ("rel_residual_host", ctypes.POINTER(ctypes.c_double)),
                ("pivots_host", ctypes.POINTER(ctypes.c_int32))]


class gp_precond_view(ctypes.Structure):
    _fields_ = [("L_dev", ctypes.c_void_p), ("pivots_dev", ctypes.c_void_p), ("logdet_dev", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("rank", ctypes.c_int32)]


class gp_batch(ctypes.Structure):
    _fields_ = [("X_dev", ctypes.c_void_p), ("y_dev", ctypes.c_void_p),
                ("offsets_host", ctypes.POINTER(ctypes.c_int64)), ("batch", ctypes.c_int32), ("d", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("ard", ctypes.c_int32)]


class gp_batch_stats(ctypes.Structure):
    _fields_ = [("iters_max", ctypes.c_int32), ("flags_any", ctypes.c_int32),
                ("iters_host", ctypes.POINTER(ctypes.c_int32)), ("flags_host", ctypes.POINTER(ctypes.c_int32)),
                ("rank_host", ctypes.POINTER(ctypes.c_int32))]


class GPError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {gp_strerror(code)} (status {code}"
                         + (f", hipError {_lib.gp_last_hip_error()}" if code == GP_EHIP else "") + ")")


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2107_00243_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, u64, szp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_size_t)
    P, O, S = ctypes.POINTER(gp_problem), ctypes.POINTER(gp_options), ctypes.POINTER(gp_stats)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.gp_workspace_size.argtypes = [P, O, i32, szp]
    lib.gp_precond_build.argtypes = [P, dp, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.gp_precond_build_rff.argtypes = [P, dp, i32, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.gp_precond_build_qff.argtypes = [P, dp, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.gp_precond_build_nystrom.argtypes = [P, dp, i32, ctypes.POINTER(ctypes.c_int32), vp, ctypes.c_size_t, vp,
                                             ctypes.POINTER(vp)]
    lib.gp_precond_view_of.argtypes = [vp, ctypes.POINTER(gp_precond_view)]
    lib.gp_precond_free.argtypes = [vp]
    lib.gp_precond_free.restype = None
    lib.gp_mll_eval.argtypes = [P, dp, O, i32, vp, vp, ctypes.c_size_t, vp, vp, S]
    lib.gp_mll_grad.argtypes = [P, dp, O, i32, vp, vp, ctypes.c_size_t, vp, vp, vp, S]
    lib.gp_khat_matvec.argtypes = [P, dp, i32, vp, i32, vp, vp, ctypes.c_size_t, vp]
    lib.gp_khat_matvec_noalloc.argtypes = [P, dp, i32, vp, i32, vp, vp]
    lib.gp_predict.argtypes = [P, dp, O, i32, vp, vp, ctypes.c_int64, vp, ctypes.c_size_t, vp, vp, vp]
    lib.gp_khat_profile.argtypes = [P, dp, O, i32, vp, ctypes.c_size_t, vp, dp, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64)]
    BP, BS = ctypes.POINTER(gp_batch), ctypes.POINTER(gp_batch_stats)
    lib.gp_batch_workspace_size.argtypes = [BP, O, i32, szp]
    lib.gp_batch_mll_eval.argtypes = [BP, dp, O, i32, vp, ctypes.c_size_t, vp, vp, BS]
    lib.gp_batch_mll_grad.argtypes = [BP, dp, O, i32, vp, ctypes.c_size_t, vp, vp, vp, BS]
    lib.gp_strerror.argtypes = [ctypes.c_int]
    lib.gp_strerror.restype = ctypes.c_char_p
    lib.gp_last_hip_error.argtypes = []
    for name in ("gp_workspace_size", "gp_precond_build", "gp_precond_build_nystrom", "gp_precond_build_rff",
                 "gp_precond_build_qff", "gp_precond_view_of", "gp_mll_eval", "gp_mll_grad", "gp_khat_matvec",
                 "gp_predict", "gp_khat_matvec_noalloc",
                 "gp_khat_profile",
                 "gp_batch_workspace_size", "gp_batch_mll_eval", "gp_batch_mll_grad", "gp_last_hip_error"):
        getattr(lib, name).restype = ctypes.c_int
    del u64
    _lib = lib
    return lib


def gp_strerror(code: int) -> str:
    return load().gp_strerror(int(code)).decode()


def _check(code, where):
    if code != GP_OK:
        raise GPError(code, where)


def _theta(theta):
    arr = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_problem(X, y, kernel: str, ard: bool) -> gp_problem:
    """gp_problem over device tensors X (n x d, FP64, contiguous) and y (n, FP64)."""
    import torch
    if X.dtype != torch.float64 or y.dtype != torch.float64 or not X.is_cuda or not y.is_cuda:
        raise ValueError("X and y must be FP64 CUDA tensors")
    if not X.is_contiguous() or not y.is_contiguous() or X.dim() != 2 or y.shape != (X.shape[0],):
        raise ValueError("X must be a contiguous (n, d) tensor and y a contiguous (n,) tensor")
    kid, shape = kernel_id(kernel)
    return gp_problem(X.data_ptr(), y.data_ptr(), X.shape[0], X.shape[1], kid, 1 if ard else 0, shape)


def make_options(precision="fp64", num_probes=16, max_iters=200, cg_tol=1e-6, seed=1, precond_grad=0,
                 sync_every=1, probe_mode=0) -> gp_options:
    return gp_options(PRECISIONS[precision] if isinstance(precision, str) else int(precision), num_probes,
                      max_iters, cg_tol, seed, precond_grad, sync_every, probe_mode)


def gp_workspace_size(prob: gp_problem, opt: gp_options, rank: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().gp_workspace_size(ctypes.byref(prob), ctypes.byref(opt), rank, ctypes.byref(out)),
           "gp_workspace_size")
    return int(out.value)


def alloc_workspace(nbytes: int, device="cuda"):
    """A device byte buffer whose data pointer is 256-byte aligned."""
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


class Stats:
    """Host copy of gp_stats with its optional arrays."""

    def __init__(self, num_probes: int, rank: int):
        t = 1 + num_probes
        self.col_iters = np.zeros(t, dtype=np.int32)
        self.gammas = np.zeros(num_probes, dtype=np.float64)
        self.rel_residual = np.zeros(t, dtype=np.float64)
        self.pivots = np.zeros(max(1, rank), dtype=np.int32)
        self.raw = gp_stats()
        self.raw.col_iters_host = self.col_iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.raw.gammas_host = self.gammas.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.raw.rel_residual_host = self.rel_residual.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.raw.pivots_host = self.pivots.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))

    def __getattr__(self, name):
        return getattr(self.__dict__["raw"], name)


def gp_precond_build(prob, theta, rank, ws, stream=None):
    arr, tp = _theta(theta)
    h = ctypes.c_void_p()
    _check(load().gp_precond_build(ctypes.byref(prob), tp, rank, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream(stream), ctypes.byref(h)), "gp_precond_build")
    return h


def gp_precond_build_nystrom(prob, theta, rank, landmarks, ws, stream=None):
    """landmarks: host sequence of rank distinct row indices."""
    arr, tp = _theta(theta)
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(load().gp_precond_build_nystrom(ctypes.byref(prob), tp, rank,
                                           lm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                           ctypes.byref(h)), "gp_precond_build_nystrom")
    return h


def gp_precond_build_qff(prob, theta, nodes_per_dim, ws, stream=None):
    """RBF kernel only; the preconditioner rank is nodes_per_dim ** d."""
    arr, tp = _theta(theta)
    h = ctypes.c_void_p()
    _check(load().gp_precond_build_qff(ctypes.byref(prob), tp, nodes_per_dim, ctypes.c_void_p(ws.data_ptr()),
                                       ws.numel(), _stream(stream), ctypes.byref(h)), "gp_precond_build_qff")
    return h


def gp_precond_build_rff(prob, theta, rank, freqs, ws, stream=None):
    """freqs: device FP64 tensor (rank / 2, d), spectral samples at unit lengthscale."""
    arr, tp = _theta(theta)
    h = ctypes.c_void_p()
    _check(load().gp_precond_build_rff(ctypes.byref(prob), tp, rank, ctypes.c_void_p(freqs.data_ptr()),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                       ctypes.byref(h)), "gp_precond_build_rff")
    return h


def gp_precond_view_of(handle) -> gp_precond_view:
    v = gp_precond_view()
    _check(load().gp_precond_view_of(handle, ctypes.byref(v)), "gp_precond_view_of")
    return v


def gp_precond_free(handle):
    load().gp_precond_free(handle)


def gp_mll_eval(prob, theta, opt, rank, precond, ws, logp, stats: Stats | None = None, stream=None):
    arr, tp = _theta(theta)
    _check(load().gp_mll_eval(ctypes.byref(prob), tp, ctypes.byref(opt), rank, precond,
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                              ctypes.c_void_p(logp.data_ptr()),
                              ctypes.byref(stats.raw) if stats is not None else None), "gp_mll_eval")


def gp_mll_grad(prob, theta, opt, rank, precond, ws, logp, grad, stats: Stats | None = None, stream=None):
    arr, tp = _theta(theta)
    _check(load().gp_mll_grad(ctypes.byref(prob), tp, ctypes.byref(opt), rank, precond,
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                              ctypes.c_void_p(logp.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                              ctypes.byref(stats.raw) if stats is not None else None), "gp_mll_grad")


def gp_predict(prob, theta, opt, rank, precond, Xstar, ws, mean, var=None, stream=None):
    """Posterior mean (and latent variance if var is given) at the rows of the
    device tensor Xstar (nstar x d FP64)."""
    arr, tp = _theta(theta)
    _check(load().gp_predict(ctypes.byref(prob), tp, ctypes.byref(opt), rank, precond,
                             ctypes.c_void_p(Xstar.data_ptr()), Xstar.shape[0], ctypes.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream(stream), ctypes.c_void_p(mean.data_ptr()),
                             ctypes.c_void_p(var.data_ptr()) if var is not None else None), "gp_predict")


def gp_khat_matvec(prob, theta, precision, V, W, ws, stream=None):
    arr, tp = _theta(theta)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(load().gp_khat_matvec(ctypes.byref(prob), tp, prec, ctypes.c_void_p(V.data_ptr()), V.shape[1],
                                 ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream(stream)), "gp_khat_matvec")


def gp_khat_matvec_noalloc(prob, theta, precision, V, W, stream=None):
    arr, tp = _theta(theta)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(load().gp_khat_matvec_noalloc(ctypes.byref(prob), tp, prec, ctypes.c_void_p(V.data_ptr()), V.shape[1],
                                         ctypes.c_void_p(W.data_ptr()), _stream(stream)), "gp_khat_matvec_noalloc")


def gp_khat_profile(prob, theta, opt, reps, ws, stream=None):
    """Mean milliseconds per launch of the tile kernel and its grid (measurement only)."""
    arr, tp = _theta(theta)
    ms = ctypes.c_double(0.0)
    gx, gy = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load().gp_khat_profile(ctypes.byref(prob), tp, ctypes.byref(opt), reps, ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream(stream), ctypes.byref(ms), ctypes.byref(gx), ctypes.byref(gy)),
           "gp_khat_profile")
    return ms.value, (gx.value, gy.value)


class Batch:
    """A ragged batch: device X (sum n_b x d) and y, host offsets, and the C struct
    that points at them (the object keeps the offsets array alive)."""

    def __init__(self, X, y, sizes, kernel: str, ard: bool):
        import torch
        if X.dtype != torch.float64 or y.dtype != torch.float64 or not X.is_cuda or not y.is_cuda:
            raise ValueError("X and y must be FP64 CUDA tensors")
        if not X.is_contiguous() or not y.is_contiguous() or X.dim() != 2 or y.shape != (X.shape[0],):
            raise ValueError("X must be a contiguous (N, d) tensor and y a contiguous (N,) tensor")
        self.offsets = np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))]).astype(np.int64)
        if self.offsets[-1] != X.shape[0]:
            raise ValueError("the sizes must add up to the rows of X")
        self.X, self.y = X, y
        self.raw = gp_batch(X.data_ptr(), y.data_ptr(), self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            len(sizes), X.shape[1], kernel_id(kernel)[0], 1 if ard else 0)

    @property
    def batch(self) -> int:
        return int(self.raw.batch)


class BatchStats:
    """Host copy of gp_batch_stats with its per-problem arrays."""

    def __init__(self, batch: int):
        self.iters = np.zeros(batch, dtype=np.int32)
        self.flags = np.zeros(batch, dtype=np.int32)
        self.rank = np.zeros(batch, dtype=np.int32)
        self.raw = gp_batch_stats()
        self.raw.iters_host = self.iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.raw.flags_host = self.flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.raw.rank_host = self.rank.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))

    def __getattr__(self, name):
        return getattr(self.__dict__["raw"], name)


def gp_batch_workspace_size(batch: Batch, opt: gp_options, rank: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().gp_batch_workspace_size(ctypes.byref(batch.raw), ctypes.byref(opt), rank, ctypes.byref(out)),
           "gp_batch_workspace_size")
    return int(out.value)


def gp_batch_mll_eval(batch: Batch, theta, opt, rank, ws, logp, stats: BatchStats | None = None, stream=None):
    """theta: (batch, p + 2) natural hyperparameters; logp: device FP64[batch]."""
    arr, tp = _theta(np.asarray(theta, dtype=np.float64).reshape(-1))
    _check(load().gp_batch_mll_eval(ctypes.byref(batch.raw), tp, ctypes.byref(opt), rank,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                    ctypes.c_void_p(logp.data_ptr()),
                                    ctypes.byref(stats.raw) if stats is not None else None), "gp_batch_mll_eval")


def gp_batch_mll_grad(batch: Batch, theta, opt, rank, ws, logp, grad, stats: BatchStats | None = None, stream=None):
    """As gp_batch_mll_eval, plus grad: device FP64[batch x (p + 2)]."""
    arr, tp = _theta(np.asarray(theta, dtype=np.float64).reshape(-1))
    _check(load().gp_batch_mll_grad(ctypes.byref(batch.raw), tp, ctypes.byref(opt), rank,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                    ctypes.c_void_p(logp.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                    ctypes.byref(stats.raw) if stats is not None else None), "gp_batch_mll_grad")
