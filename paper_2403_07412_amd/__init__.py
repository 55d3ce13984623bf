"""MI355X-native Vecchia Gaussian-process log-likelihood (FP64) — Python binding.

The compute lives in ``libvecchia.so`` (hand-written HIP for gfx950, C ABI
declared in ``include/vecchia.h``).  This module only marshals torch tensors
(device memory and the current HIP stream) into that ABI; it has no numerical
fallback.  Importing works without a GPU; calling needs the built library and
a GPU, and fails loudly otherwise.

Functions carry the C names:

    vecchia_workspace_size(n, m)
    vecchia_loglik(locs, z, nbr, m, nu, theta, ...)          -> (out[1], status[1])
    vecchia_loglik_grad(locs, z, nbr, m, nu, theta, ...)     -> (out[1], grad[3], status[1])
    vecchia_loglik_terms(locs, z, nbr, m, nu, theta, idx...) -> (terms, gterms, status)

and ``loglik(locs, z, nbr, theta, nu, m)`` is the differentiable form
(a ``torch.autograd.Function``): its backward returns grad_out * dl/dtheta,
computed by the fused adjoint kernel in the forward pass.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; VECCHIA_LIB may name another build of the same sources
LIB_PATH = os.environ.get("VECCHIA_LIB") or os.path.join(_HERE, "libvecchia.so")

VECCHIA_MAX_M = 160
VECCHIA_STATUS_THETA = -1
VARIANTS = {"auto": 0, "unblocked": 1, "tile_w1": 2, "tile_w2": 3, "tile_w4": 4, "tile_w8": 5}
_ERRORS = {1: "VECCHIA_EINVAL", 2: "VECCHIA_EUNSUPPORTED", 3: "VECCHIA_EHIP", 4: "VECCHIA_EWORKSPACE"}

_lib = None


class _Field(ctypes.Structure):
    """Mirror of struct vecchia_field."""
    _fields_ = [("locs", ctypes.c_void_p), ("z", ctypes.c_void_p), ("nbr", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("m", ctypes.c_int32)]


class MleOptions(ctypes.Structure):
    """vecchia_mle_options."""
    _fields_ = [("max_iter", ctypes.c_int32), ("history", ctypes.c_int32), ("gtol", ctypes.c_double),
                ("ftol", ctypes.c_double), ("lower", ctypes.c_double * 3), ("upper", ctypes.c_double * 3),
                ("trial_steps", ctypes.c_int32)]


class VecchiaError(RuntimeError):
    """A synchronous error code returned by the C ABI."""

    def __init__(self, code: int, what: str = ""):
        self.code = int(code)
        msg = _load().vecchia_strerror(self.code).decode() if _lib is not None else _ERRORS.get(code, "")
        super().__init__(f"{what}: {_ERRORS.get(self.code, self.code)} ({msg})")


class VecchiaNumericalError(RuntimeError):
    """Device status: a conditional failed (status = i+1) or theta was invalid (status = -1)."""

    def __init__(self, status: int):
        self.status = int(status)
        if status == VECCHIA_STATUS_THETA:
            msg = "invalid covariance parameters"
        else:
            msg = f"point {status - 1}: block not positive definite, non-finite input or bad neighbour index"
        super().__init__(msg)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_07412_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        lib.vecchia_strerror.restype = ctypes.c_char_p
        lib.vecchia_strerror.argtypes = [ctypes.c_int]
        lib.vecchia_version.restype = ctypes.c_char_p
        lib.vecchia_version.argtypes = []
        lib.vecchia_workspace_size.restype = SZ
        lib.vecchia_workspace_size.argtypes = [I64, I32]
        lib.vecchia_loglik.restype = ctypes.c_int
        lib.vecchia_loglik.argtypes = [P, P, P, I64, I32, D, P, P, P, P, SZ, P]
        lib.vecchia_loglik_grad.restype = ctypes.c_int
        lib.vecchia_loglik_grad.argtypes = [P, P, P, I64, I32, D, P, P, P, P, P, SZ, P]
        lib.vecchia_loglik_grad_noalloc.restype = ctypes.c_int
        lib.vecchia_loglik_grad_noalloc.argtypes = [P, P, P, I64, I32, D, P, P, P, P, P]
        lib.vecchia_loglik_terms.restype = ctypes.c_int
        lib.vecchia_loglik_terms.argtypes = [P, P, P, I64, I32, D, P, P, I64, P, P, P, P]
        lib.vecchia_variant_feasible.restype = ctypes.c_int
        lib.vecchia_variant_feasible.argtypes = [I32, I32]
        lib.vecchia_set_variant.restype = ctypes.c_int
        lib.vecchia_set_variant.argtypes = [I32, I32, I32]
        lib.vecchia_get_variant.restype = ctypes.c_int
        lib.vecchia_get_variant.argtypes = [I32, I32]
        lib.vecchia_loglik_variant.restype = ctypes.c_int
        lib.vecchia_loglik_variant.argtypes = [P, P, P, I64, I32, D, P, I32, P, P, P, P, SZ, P]
        lib.vecchia_loglik_terms_variant.restype = ctypes.c_int
        lib.vecchia_loglik_terms_variant.argtypes = [P, P, P, I64, I32, D, P, I32, P, I64, P, P, P, P]
        PP = ctypes.POINTER(ctypes.c_void_p)
        lib.vecchia_plan_create.restype = ctypes.c_int
        lib.vecchia_plan_create.argtypes = [ctypes.POINTER(_Field), I32, I32, D, I32, PP]
        lib.vecchia_plan_create_cov.restype = ctypes.c_int
        lib.vecchia_plan_create_cov.argtypes = [ctypes.POINTER(_Field), I32, I32, ctypes.POINTER(Cov), I32, PP]
        lib.vecchia_plan_workspace_size.restype = SZ
        lib.vecchia_plan_workspace_size.argtypes = [P]
        lib.vecchia_plan_num_classes.restype = ctypes.c_int
        lib.vecchia_plan_num_classes.argtypes = [P]
        lib.vecchia_plan_class_info.restype = ctypes.c_int
        lib.vecchia_plan_class_info.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                                ctypes.POINTER(I32), ctypes.POINTER(I64)]
        lib.vecchia_plan_class_group.restype = ctypes.c_int
        lib.vecchia_plan_class_group.argtypes = [P, I32]
        lib.vecchia_set_lockstep.restype = ctypes.c_int
        lib.vecchia_set_lockstep.argtypes = [I32]
        lib.vecchia_plan_destroy.restype = ctypes.c_int
        lib.vecchia_plan_destroy.argtypes = [P]
        lib.vecchia_plan_loglik.restype = ctypes.c_int
        lib.vecchia_plan_loglik.argtypes = [P, P, P, P, P, P, SZ, P]
        lib.vecchia_batched_workspace.restype = SZ
        lib.vecchia_batched_workspace.argtypes = [ctypes.POINTER(_Field), I32, I32]
        lib.vecchia_loglik_batched.restype = ctypes.c_int
        lib.vecchia_loglik_batched.argtypes = [ctypes.POINTER(_Field), I32, P, I32, D, I32, P, P, P, P, SZ, P]
        lib.vecchia_batched_graph_create.restype = ctypes.c_int
        lib.vecchia_batched_graph_create.argtypes = [P, P, P, P, P, P, SZ, P, PP]
        lib.vecchia_batched_graph_launch.restype = ctypes.c_int
        lib.vecchia_batched_graph_launch.argtypes = [P, P]
        lib.vecchia_batched_graph_destroy.restype = ctypes.c_int
        lib.vecchia_batched_graph_destroy.argtypes = [P]
        lib.vecchia_autotune.restype = ctypes.c_int
        lib.vecchia_autotune.argtypes = [ctypes.POINTER(_Field), D, I32, P, I64, I32, P, SZ, P,
                                         ctypes.POINTER(I32), ctypes.POINTER(D)]
        lib.vecchia_knn_workspace_size.restype = SZ
        lib.vecchia_knn_workspace_size.argtypes = [I64]
        lib.vecchia_knn.restype = ctypes.c_int
        lib.vecchia_knn.argtypes = [P, I64, I32, P, P, SZ, P]
        lib.vecchia_random_order_workspace_size.restype = SZ
        lib.vecchia_random_order_workspace_size.argtypes = [I64]
        lib.vecchia_random_order.restype = ctypes.c_int
        lib.vecchia_random_order.argtypes = [I64, ctypes.c_uint64, P, P, SZ, P]
        lib.vecchia_maxmin_workspace_size.restype = SZ
        lib.vecchia_maxmin_workspace_size.argtypes = [I64]
        lib.vecchia_maxmin_order.restype = ctypes.c_int
        lib.vecchia_maxmin_order.argtypes = [P, I64, ctypes.c_uint64, P, P, SZ, P]
        lib.vecchia_knn_metric.restype = ctypes.c_int
        lib.vecchia_knn_metric.argtypes = [P, I64, I32, I32, P, P, SZ, P]
        lib.vecchia_knn_query.restype = ctypes.c_int
        lib.vecchia_knn_query.argtypes = [P, I64, P, I64, I32, I32, P, P, SZ, P]
        lib.vecchia_morton_workspace_size.restype = SZ
        lib.vecchia_morton_workspace_size.argtypes = [I64]
        lib.vecchia_morton_order.restype = ctypes.c_int
        lib.vecchia_morton_order.argtypes = [P, I64, P, P, SZ, P]
        lib.vecchia_mle_default_options.restype = None
        lib.vecchia_mle_default_options.argtypes = [ctypes.POINTER(MleOptions)]
        lib.vecchia_mle_workspace_size.restype = SZ
        lib.vecchia_mle_workspace_size.argtypes = [I64, I32]
        lib.vecchia_exact_workspace_size.restype = SZ
        lib.vecchia_exact_workspace_size.argtypes = [I64]
        lib.vecchia_exact_loglik.restype = ctypes.c_int
        lib.vecchia_exact_loglik.argtypes = [P, P, I64, D, P, P, P, P, SZ, P]
        lib.vecchia_dense_logdet_workspace_size.restype = SZ
        lib.vecchia_dense_logdet_workspace_size.argtypes = [I64]
        lib.vecchia_dense_logdet.restype = ctypes.c_int
        lib.vecchia_dense_logdet.argtypes = [P, I64, I64, P, P, P, P, P, SZ, P]
        CP = ctypes.POINTER(Cov)
        lib.vecchia_mle_cov.restype = ctypes.c_int
        lib.vecchia_mle_cov.argtypes = [P, P, P, I64, I32, CP, ctypes.POINTER(D), ctypes.POINTER(MleOptions),
                                        ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I32),
                                        ctypes.POINTER(I32), ctypes.POINTER(I32), P, SZ, P]
        lib.vecchia_loglik_cov.restype = ctypes.c_int
        lib.vecchia_loglik_cov.argtypes = [P, P, P, I64, I32, CP, P, P, P, P, P, SZ, P]
        lib.vecchia_loglik_terms_cov.restype = ctypes.c_int
        lib.vecchia_loglik_terms_cov.argtypes = [P, P, P, I64, I32, CP, P, P, I64, P, P, P, P]
        lib.vecchia_predict.restype = ctypes.c_int
        lib.vecchia_predict.argtypes = [P, P, I64, P, I64, P, I32, CP, P, P, P, P, P]
        lib.vecchia_mle.restype = ctypes.c_int
        lib.vecchia_mle.argtypes = [P, P, P, I64, I32, D, ctypes.POINTER(D), ctypes.POINTER(MleOptions),
                                    ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I32),
                                    ctypes.POINTER(I32), ctypes.POINTER(I32), P, SZ, P]
        _lib = lib
    return _lib


# covariance models (vecchia_cov in the C header)
MATERN, POWEXP = 0, 1
EUCLIDEAN, GREAT_CIRCLE = 0, 1


class Cov(ctypes.Structure):
    """Covariance model: family (MATERN, POWEXP), metric (EUCLIDEAN, GREAT_CIRCLE) and smoothness
    (nu for Matern, alpha for the power exponential)."""
    _fields_ = [("family", ctypes.c_int32), ("metric", ctypes.c_int32), ("smoothness", ctypes.c_double)]


def _cov(cov) -> Cov:
    if isinstance(cov, Cov):
        return cov
    family, metric, smoothness = cov
    return Cov(int(family), int(metric), float(smoothness))


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _load()


def version() -> str:
    return _load().vecchia_version().decode()


# ------------------------------------------------------------------ marshalling
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_check(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("inputs must be contiguous device tensors")


def _tensor_check(t, name: str, dtype, numel: int, device=None):
    """Raises unless t is a contiguous device tensor of `dtype` with at least `numel` elements (on
    `device` when given): the C ABI reads and writes that many elements through the raw pointer."""
    if t is None:
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the inputs on {device}")
    if t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")


def _theta_check(theta, device, count: int = 1):
    """theta: float64, exactly 3 * count elements, on the inputs' device."""
    _tensor_check(theta, "theta", torch.float64, 3 * count, device)
    if theta.numel() != 3 * count:
        raise ValueError(f"theta must hold exactly {3 * count} float64 values, has {theta.numel()}")


def _outputs_check(device, out=None, grad=None, status=None, n_out: int = 1):
    if out is not None:
        _tensor_check(out, "out", torch.float64, n_out, device)
    if grad is not None:
        _tensor_check(grad, "grad", torch.float64, 3 * n_out, device)
    if status is not None:
        _tensor_check(status, "status", torch.int64, n_out, device)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_inputs(locs, z, nbr, m):
    if locs.dtype != torch.float64 or z.dtype != torch.float64:
        raise TypeError("locs and z must be float64")
    n = z.shape[0]
    if tuple(locs.shape) != (n, 2):
        raise ValueError("locs must be [n][2]")
    if m > 0:
        if nbr is None or nbr.dtype != torch.int32 or tuple(nbr.shape) != (n, m):
            raise ValueError("nbr must be int32 [n][m]")
    _dev_check(locs, z, nbr if m > 0 else None)
    return n


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


def _check(rc, what):
    if rc != 0:
        raise VecchiaError(rc, what)


def vecchia_workspace_size(n: int, m: int) -> int:
    return int(_load().vecchia_workspace_size(int(n), int(m)))


def _workspace(n, m, device, ws):
    need = vecchia_workspace_size(n, m)
    if ws is not None:
        _dev_check(ws)
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    return ws


def vecchia_loglik(locs, z, nbr, m: int, nu: float, theta, out=None, status=None, ws=None, stream=None):
    """l = sum_i log p(z_i | z_{J_i}) on the device; returns (out[1], status[1]) without synchronising."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    status = torch.empty(1, dtype=torch.int64, device=dev) if status is None else status
    _theta_check(theta, dev)
    _outputs_check(dev, out=out, status=status)
    ws = _workspace(n, m, dev, ws)
    rc = _load().vecchia_loglik(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, float(nu), _ptr(theta),
                                _ptr(out), _ptr(status), _ptr(ws), _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_loglik")
    return out, status


def vecchia_loglik_grad(locs, z, nbr, m: int, nu: float, theta, out=None, grad=None, status=None, ws=None,
                        stream=None):
    """l and dl/d(sigma2, beta, tau2) on the device; returns (out[1], grad[3], status[1])."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    grad = torch.empty(3, dtype=torch.float64, device=dev) if grad is None else grad
    status = torch.empty(1, dtype=torch.int64, device=dev) if status is None else status
    _theta_check(theta, dev)
    _outputs_check(dev, out=out, grad=grad, status=status)
    ws = _workspace(n, m, dev, ws)
    rc = _load().vecchia_loglik_grad(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, float(nu),
                                     _ptr(theta), _ptr(out), _ptr(grad), _ptr(status), _ptr(ws), _nbytes(ws),
                                     _stream(stream))
    _check(rc, "vecchia_loglik_grad")
    return out, grad, status


VECCHIA_NOALLOC_MAX_N = 1 << 26


def vecchia_loglik_grad_noalloc(locs, z, nbr, m: int, nu: float, theta, out, grad, status, stream=None):
    """vecchia_loglik_grad without a workspace (the library's static scratch): for callers that cannot
    allocate, so the outputs are required; calls that overlap on one GPU race."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    _theta_check(theta, dev)
    _outputs_check(dev, out=out, grad=grad, status=status)
    rc = _load().vecchia_loglik_grad_noalloc(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, float(nu),
                                             _ptr(theta), _ptr(out), _ptr(grad), _ptr(status), _stream(stream))
    _check(rc, "vecchia_loglik_grad_noalloc")
    return out, grad, status


def vecchia_loglik_terms(locs, z, nbr, m: int, nu: float, theta, idx=None, with_grad: bool = False, stream=None):
    """Per-point l_i (and dl_i/dtheta) for the points idx (default all); returns (terms, gterms|None, status)."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    if idx is not None:
        if idx.dtype != torch.int64:
            raise TypeError("idx must be int64")
        _dev_check(idx)
        nidx = idx.shape[0]
    else:
        nidx = n
    terms = torch.empty(max(nidx, 1), dtype=torch.float64, device=dev)
    gterms = torch.empty((max(nidx, 1), 3), dtype=torch.float64, device=dev) if with_grad else None
    status = torch.empty(1, dtype=torch.int64, device=dev)
    _theta_check(theta, dev)
    rc = _load().vecchia_loglik_terms(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, float(nu),
                                      _ptr(theta), _ptr(idx), nidx, _ptr(terms), _ptr(gterms), _ptr(status),
                                      _stream(stream))
    _check(rc, "vecchia_loglik_terms")
    return terms[:nidx], (gterms[:nidx] if gterms is not None else None), status


def vecchia_loglik_cov(locs, z, nbr, m: int, cov, theta, with_grad: bool = False, out=None, grad=None,
                       status=None, ws=None, stream=None):
    """Log-likelihood (and gradient) under a covariance model cov = (family, metric, smoothness);
    returns (out[1], grad[3]|None, status[1]) without synchronising."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    if with_grad and grad is None:
        grad = torch.empty(3, dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int64, device=dev) if status is None else status
    _theta_check(theta, dev)
    _outputs_check(dev, out=out, grad=grad if with_grad else None, status=status)
    ws = _workspace(n, m, dev, ws)
    c = _cov(cov)
    rc = _load().vecchia_loglik_cov(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, ctypes.byref(c),
                                    _ptr(theta), _ptr(out), _ptr(grad) if with_grad else None, _ptr(status),
                                    _ptr(ws), _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_loglik_cov")
    return out, (grad if with_grad else None), status


def vecchia_loglik_terms_cov(locs, z, nbr, m: int, cov, theta, idx=None, with_grad: bool = False, stream=None):
    """Per-point l_i (and gradient) under a covariance model; returns (terms, gterms|None, status)."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    if idx is not None:
        if idx.dtype != torch.int64:
            raise TypeError("idx must be int64")
        _dev_check(idx)
        nidx = idx.shape[0]
    else:
        nidx = n
    terms = torch.empty(max(nidx, 1), dtype=torch.float64, device=dev)
    gterms = torch.empty((max(nidx, 1), 3), dtype=torch.float64, device=dev) if with_grad else None
    status = torch.empty(1, dtype=torch.int64, device=dev)
    _theta_check(theta, dev)
    c = _cov(cov)
    rc = _load().vecchia_loglik_terms_cov(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, ctypes.byref(c),
                                          _ptr(theta), _ptr(idx), nidx, _ptr(terms), _ptr(gterms), _ptr(status),
                                          _stream(stream))
    _check(rc, "vecchia_loglik_terms_cov")
    return terms[:nidx], (gterms[:nidx] if gterms is not None else None), status


def vecchia_predict(locs, z, qlocs, nbr, m: int, cov, theta, mean=None, var=None, status=None, stream=None):
    """Vecchia kriging: conditional mean and variance (of a new observation) at each prediction point
    given the observations at its neighbours (row t of nbr, [nq][m] int32 indices into locs);
    returns (mean[nq], var[nq], status[1]) without synchronising."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be float64 [n][2]")
    if qlocs.dtype != torch.float64 or qlocs.dim() != 2 or qlocs.shape[1] != 2:
        raise ValueError("qlocs must be float64 [nq][2]")
    n, nq = locs.shape[0], qlocs.shape[0]
    if z.dtype != torch.float64 or tuple(z.shape) != (n,):
        raise ValueError("z must be float64 [n]")
    if m > 0 and (nbr.dtype != torch.int32 or tuple(nbr.shape) != (nq, m)):
        raise ValueError("nbr must be int32 [nq][m]")
    dev = qlocs.device
    mean = torch.empty(max(nq, 1), dtype=torch.float64, device=dev) if mean is None else mean
    var = torch.empty(max(nq, 1), dtype=torch.float64, device=dev) if var is None else var
    status = torch.empty(1, dtype=torch.int64, device=dev) if status is None else status
    _dev_check(locs, z, qlocs, nbr if m > 0 else None)
    _theta_check(theta, dev)
    _tensor_check(mean, "mean", torch.float64, nq, dev)
    _tensor_check(var, "var", torch.float64, nq, dev)
    _tensor_check(status, "status", torch.int64, 1, dev)
    c = _cov(cov)
    rc = _load().vecchia_predict(_ptr(locs), _ptr(z), n, _ptr(qlocs), nq, _ptr(nbr) if m > 0 else None, m,
                                 ctypes.byref(c), _ptr(theta), _ptr(mean), _ptr(var), _ptr(status), _stream(stream))
    _check(rc, "vecchia_predict")
    return mean[:nq], var[:nq], status


def _variant_id(variant) -> int:
    return VARIANTS[variant] if isinstance(variant, str) else int(variant)


def vecchia_variant_feasible(m: int, variant) -> bool:
    return bool(_load().vecchia_variant_feasible(int(m), _variant_id(variant)))


def vecchia_set_variant(m: int, with_grad: bool, variant) -> None:
    _check(_load().vecchia_set_variant(int(m), int(bool(with_grad)), _variant_id(variant)), "vecchia_set_variant")


def vecchia_get_variant(m: int, with_grad: bool) -> int:
    return int(_load().vecchia_get_variant(int(m), int(bool(with_grad))))


def vecchia_loglik_variant(locs, z, nbr, m: int, nu: float, theta, variant, with_grad: bool = False, out=None,
                           grad=None, status=None, ws=None, stream=None):
    """vecchia_loglik / vecchia_loglik_grad with an explicit kernel variant; returns (out, grad|None, status)."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    if with_grad and grad is None:
        grad = torch.empty(3, dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int64, device=dev) if status is None else status
    _theta_check(theta, dev)
    _outputs_check(dev, out=out, grad=grad if with_grad else None, status=status)
    ws = _workspace(n, m, dev, ws)
    rc = _load().vecchia_loglik_variant(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, float(nu),
                                        _ptr(theta), _variant_id(variant), _ptr(out),
                                        _ptr(grad) if with_grad else None, _ptr(status), _ptr(ws), _nbytes(ws),
                                        _stream(stream))
    _check(rc, "vecchia_loglik_variant")
    return out, (grad if with_grad else None), status


def vecchia_loglik_terms_variant(locs, z, nbr, m: int, nu: float, theta, variant, idx=None, with_grad=False,
                                 stream=None):
    """vecchia_loglik_terms with an explicit kernel variant."""
    n = _as_inputs(locs, z, nbr, m)
    dev = z.device
    if idx is not None:
        if idx.dtype != torch.int64:
            raise TypeError("idx must be int64")
        _dev_check(idx)
        nidx = idx.shape[0]
    else:
        nidx = n
    terms = torch.empty(max(nidx, 1), dtype=torch.float64, device=dev)
    gterms = torch.empty((max(nidx, 1), 3), dtype=torch.float64, device=dev) if with_grad else None
    status = torch.empty(1, dtype=torch.int64, device=dev)
    _theta_check(theta, dev)
    rc = _load().vecchia_loglik_terms_variant(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, m, float(nu),
                                              _ptr(theta), _variant_id(variant), _ptr(idx), nidx, _ptr(terms),
                                              _ptr(gterms), _ptr(status), _stream(stream))
    _check(rc, "vecchia_loglik_terms_variant")
    return terms[:nidx], (gterms[:nidx] if gterms is not None else None), status


def raise_on_status(status) -> None:
    """Synchronises and raises VecchiaNumericalError when a device status word is non-zero."""
    s = int(status.reshape(-1)[0].item())
    if s != 0:
        raise VecchiaNumericalError(s)


# ------------------------------------------------------------------ autograd
class VecchiaLogLik(torch.autograd.Function):
    """l(theta) with the analytic adjoint; theta = (sigma2, beta, tau2) as a float64 device tensor [3].
    `model` is the Matern smoothness nu (a float) or a covariance model (family, metric, smoothness)."""

    @staticmethod
    def forward(ctx, theta, locs, z, nbr, model, m, check):
        _theta_check(theta, z.device)
        theta_c = theta.detach()
        cov = model if isinstance(model, (tuple, list, Cov)) else (MATERN, EUCLIDEAN, float(model))
        out, grad, status = vecchia_loglik_cov(locs, z, nbr, m, cov, theta_c, with_grad=ctx.needs_input_grad[0])
        if ctx.needs_input_grad[0]:
            ctx.save_for_backward(grad)
        if check:
            raise_on_status(status)
        return out.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None, None, None, None, None, None


def loglik(locs, z, nbr, theta, nu: float, m: int, check: bool = True, cov=None):
    """Differentiable Vecchia log-likelihood (0-d float64 tensor on the device), Matern with smoothness
    nu on Euclidean distances, or the covariance model cov = (family, metric, smoothness) when given.

    check=True synchronises once to raise VecchiaNumericalError on a failed
    conditional; pass False inside captured graphs or tight loops and read the
    status yourself."""
    model = tuple(cov) if cov is not None else float(nu)
    return VecchiaLogLik.apply(theta, locs, z, nbr, model, int(m), check)


# ------------------------------------------------------------------ batched
def _field_struct(locs, z, nbr, m):
    n = _as_inputs(locs, z, nbr, m)
    return _Field(locs.data_ptr() if n else None, z.data_ptr() if n else None,
                  nbr.data_ptr() if (m > 0 and n) else None, n, m)


class BatchedPlan:
    """vecchia_plan_* over a list of fields (each (locs, z, nbr, m) of device tensors), ntheta parameter
    vectors per field, Matern nu on Euclidean distances or the covariance model cov = (family, metric,
    smoothness) when given.  Keeps references to the field tensors for the plan's lifetime."""

    def __init__(self, fields, ntheta: int, nu: float, with_grad: bool, cov=None):
        self._fields = [tuple(f) for f in fields]
        arr = (_Field * len(self._fields))(*[_field_struct(*f) for f in self._fields])
        handle = ctypes.c_void_p()
        c = _cov(cov if cov is not None else (MATERN, EUCLIDEAN, nu))
        _check(_load().vecchia_plan_create_cov(arr, len(self._fields), int(ntheta), ctypes.byref(c),
                                               int(bool(with_grad)), ctypes.byref(handle)), "vecchia_plan_create")
        self.handle = handle
        self.nf, self.ntheta, self.nu, self.with_grad = len(self._fields), int(ntheta), float(nu), bool(with_grad)
        self.device = self._fields[0][1].device
        self.ws = torch.empty(max(1, int(_load().vecchia_plan_workspace_size(handle))), dtype=torch.uint8,
                              device=self.device)

    def classes(self):
        """[(tile_rows, variant, nfields, items)] per tile class."""
        out = []
        for c in range(_load().vecchia_plan_num_classes(self.handle)):
            T, var, nfc, items = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
            _check(_load().vecchia_plan_class_info(self.handle, c, ctypes.byref(T), ctypes.byref(var),
                                                   ctypes.byref(nfc), ctypes.byref(items)), "class_info")
            out.append((T.value, var.value, nfc.value, items.value))
        return out

    def groups(self):
        """Parameter vectors per workgroup (lockstep group size) of each tile class."""
        lib = _load()
        out = []
        for c in range(lib.vecchia_plan_num_classes(self.handle)):
            g = lib.vecchia_plan_class_group(self.handle, c)
            if g < 0:
                _check(-g, "vecchia_plan_class_group")
            out.append(g)
        return out

    def _check_arrays(self, thetas, out, grad, status):
        ne = self.nf * self.ntheta
        _theta_check(thetas, self.device, ne)
        _outputs_check(self.device, out=out, grad=grad, status=status, n_out=ne)
        if self.with_grad and grad is None:
            raise ValueError("the plan evaluates gradients: grad is required")

    def outputs(self):
        dev = self.device
        out = torch.empty((self.nf, self.ntheta), dtype=torch.float64, device=dev)
        grad = torch.empty((self.nf, self.ntheta, 3), dtype=torch.float64, device=dev) if self.with_grad else None
        status = torch.empty((self.nf, self.ntheta), dtype=torch.int64, device=dev)
        return out, grad, status

    def __call__(self, thetas, out=None, grad=None, status=None, stream=None):
        """vecchia_plan_loglik: thetas [nf][ntheta][3] float64 device tensor -> (out, grad|None, status)."""
        if tuple(thetas.shape) != (self.nf, self.ntheta, 3) or thetas.dtype != torch.float64:
            raise ValueError("thetas must be float64 [nf][ntheta][3]")
        o, g, st = self.outputs()
        out = o if out is None else out
        grad = (g if grad is None else grad) if self.with_grad else None
        status = st if status is None else status
        self._check_arrays(thetas, out, grad, status)
        rc = _load().vecchia_plan_loglik(self.handle, _ptr(thetas), _ptr(out), _ptr(grad), _ptr(status),
                                            _ptr(self.ws), _nbytes(self.ws), _stream(stream))
        _check(rc, "vecchia_plan_loglik")
        return out, grad, status

    def capture(self, thetas, out, grad, status, stream=None):
        """vecchia_batched_graph_create on a side stream; returns a BatchedGraph bound to these arrays."""
        self._check_arrays(thetas, out, grad, status)
        s = stream if stream is not None else torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        handle = ctypes.c_void_p()
        rc = _load().vecchia_batched_graph_create(self.handle, _ptr(thetas), _ptr(out), _ptr(grad), _ptr(status),
                                                  _ptr(self.ws), _nbytes(self.ws), ctypes.c_void_p(s.cuda_stream),
                                                  ctypes.byref(handle))
        _check(rc, "vecchia_batched_graph_create")
        return BatchedGraph(handle, self, (thetas, out, grad, status))

    def close(self):
        if getattr(self, "handle", None):
            _load().vecchia_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vecchia_batched_workspace(fields, ntheta: int) -> int:
    """Workspace bytes of vecchia_loglik_batched for these fields (each (locs, z, nbr, m))."""
    fs = [tuple(f) for f in fields]
    arr = (_Field * len(fs))(*[_field_struct(*f) for f in fs])
    return int(_load().vecchia_batched_workspace(arr, len(fs), int(ntheta)))


def vecchia_loglik_batched(fields, thetas, nu: float, with_grad: bool, out=None, grad=None, status=None, ws=None,
                           stream=None):
    """The one-call batched form: fields = [(locs, z, nbr, m)], thetas float64 [nf][ntheta][3] on the
    device; returns (out [nf][ntheta], grad [nf][ntheta][3] | None, status [nf][ntheta])."""
    fs = [tuple(f) for f in fields]
    nf = len(fs)
    if nf < 1:
        raise ValueError("at least one field")
    if thetas.dim() != 3 or thetas.shape[0] != nf or thetas.shape[2] != 3:
        raise ValueError("thetas must be float64 [nf][ntheta][3]")
    ntheta = int(thetas.shape[1])
    dev = fs[0][1].device
    arr = (_Field * nf)(*[_field_struct(*f) for f in fs])
    _theta_check(thetas, dev, nf * ntheta)
    out = torch.empty((nf, ntheta), dtype=torch.float64, device=dev) if out is None else out
    if with_grad and grad is None:
        grad = torch.empty((nf, ntheta, 3), dtype=torch.float64, device=dev)
    status = torch.empty((nf, ntheta), dtype=torch.int64, device=dev) if status is None else status
    _outputs_check(dev, out=out, grad=grad if with_grad else None, status=status, n_out=nf * ntheta)
    need = int(_load().vecchia_batched_workspace(arr, nf, ntheta))
    if need == 0:
        raise ValueError("vecchia_batched_workspace rejected the fields")
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    _dev_check(ws)
    rc = _load().vecchia_loglik_batched(arr, nf, _ptr(thetas), ntheta, float(nu), int(bool(with_grad)), _ptr(out),
                                        _ptr(grad) if with_grad else None, _ptr(status), _ptr(ws), _nbytes(ws),
                                        _stream(stream))
    _check(rc, "vecchia_loglik_batched")
    return out, (grad if with_grad else None), status


class BatchedGraph:
    """A captured, instantiated batched evaluation; launch() replays it (reads thetas in place)."""

    def __init__(self, handle, plan, keep):
        self.handle, self._plan, self._keep = handle, plan, keep

    def launch(self, stream=None):
        _check(_load().vecchia_batched_graph_launch(self.handle, _stream(stream)), "vecchia_batched_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            _load().vecchia_batched_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_lockstep(enable: bool) -> bool:
    """Whether plans created from now on may evaluate several parameter vectors per workgroup (default on);
    returns the previous setting (process-wide)."""
    return bool(_load().vecchia_set_lockstep(int(bool(enable))))


def vecchia_autotune(locs, z, nbr, m: int, nu: float, theta, with_grad: bool, sample: int = 20000, reps: int = 3,
                     stream=None):
    """Times every feasible variant for (m, with_grad) on these inputs, stores the fastest in the variant
    table and returns (best_variant, {variant: microseconds per point})."""
    f = _field_struct(locs, z, nbr, m)
    ws = torch.empty(max(1, 40 * f.n), dtype=torch.uint8, device=z.device)
    best = ctypes.c_int32()
    us = (ctypes.c_double * 6)()
    _theta_check(theta, z.device)
    rc = _load().vecchia_autotune(ctypes.byref(f), float(nu), int(bool(with_grad)), _ptr(theta), int(sample),
                                  int(reps), _ptr(ws), _nbytes(ws), _stream(stream), ctypes.byref(best), us)
    _check(rc, "vecchia_autotune")
    names = {v: k for k, v in VARIANTS.items()}
    return best.value, {names[v]: us[v] for v in range(1, 6) if us[v] >= 0}


def variant_table():
    """The variant each (m, with_grad) uses now: {"grad": [...161], "value": [...161]}."""
    return {"value": [vecchia_get_variant(m, False) for m in range(VECCHIA_MAX_M + 1)],
            "grad": [vecchia_get_variant(m, True) for m in range(VECCHIA_MAX_M + 1)]}


def save_variant_table(path: str) -> None:
    """Writes the current variant table (e.g. after autotuning) as JSON."""
    import json

    with open(path, "w") as fh:
        json.dump({"format": "vecchia-variant-table-1", **variant_table()}, fh)


def load_variant_table(path: str) -> None:
    """Loads a table written by save_variant_table into the library (infeasible entries are rejected)."""
    import json

    with open(path) as fh:
        data = json.load(fh)
    if data.get("format") != "vecchia-variant-table-1":
        raise ValueError(f"{path}: not a variant table")
    for key, grad in (("value", False), ("grad", True)):
        for m, var in enumerate(data[key]):
            vecchia_set_variant(m, grad, int(var))


# ------------------------------------------------------------- preprocessing
def vecchia_knn_workspace_size(n: int) -> int:
    return int(_load().vecchia_knn_workspace_size(int(n)))


def vecchia_knn(locs, m: int, out=None, ws=None, stream=None, metric: int = EUCLIDEAN):
    """Conditioning sets on the GPU: int32 [n][m], row i = the min(i, m) nearest points j < i by
    (key, index), -1 padded; the key is the squared distance (EUCLIDEAN) or the haversine value of
    (longitude, latitude) degrees (GREAT_CIRCLE).  locs: float64 [n][2] device tensor."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be float64 [n][2]")
    _dev_check(locs)
    n = locs.shape[0]
    if out is None:
        out = torch.empty((n, max(m, 0)), dtype=torch.int32, device=locs.device)
    if tuple(out.shape) != (n, m) or out.dtype != torch.int32:
        raise ValueError("out must be int32 [n][m]")
    _dev_check(out)
    need = vecchia_knn_workspace_size(n)
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=locs.device)
    rc = _load().vecchia_knn_metric(_ptr(locs), n, int(m), int(metric), _ptr(out), _ptr(ws), _nbytes(ws),
                                    _stream(stream))
    _check(rc, "vecchia_knn")
    return out


def vecchia_knn_query(locs, qlocs, m: int, metric: int = EUCLIDEAN, out=None, ws=None, stream=None):
    """Neighbour sets of prediction points: int32 [nq][m], row t = the min(n, m) points of locs nearest
    to qlocs[t] by (key, index), -1 padded."""
    for t, name in ((locs, "locs"), (qlocs, "qlocs")):
        if t.dtype != torch.float64 or t.dim() != 2 or t.shape[1] != 2:
            raise ValueError(f"{name} must be float64 [rows][2]")
    _dev_check(locs, qlocs)
    n, nq = locs.shape[0], qlocs.shape[0]
    if out is None:
        out = torch.empty((nq, max(m, 0)), dtype=torch.int32, device=qlocs.device)
    if tuple(out.shape) != (nq, m) or out.dtype != torch.int32:
        raise ValueError("out must be int32 [nq][m]")
    _dev_check(out)
    need = vecchia_knn_workspace_size(n)
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=qlocs.device)
    rc = _load().vecchia_knn_query(_ptr(locs), n, _ptr(qlocs), nq, int(m), int(metric), _ptr(out), _ptr(ws),
                                   _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_knn_query")
    return out


def vecchia_random_order(n: int, seed: int = 0, device=None, out=None, ws=None, stream=None):
    """Random permutation of n points (int64 [n] on the device): indices by ascending splitmix64
    finaliser of seed XOR i."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    n = int(n)
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=dev)
    if tuple(out.shape) != (n,) or out.dtype != torch.int64:
        raise ValueError("out must be int64 [n]")
    _dev_check(out)
    need = int(_load().vecchia_random_order_workspace_size(n))
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=out.device)
    rc = _load().vecchia_random_order(n, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(out), _ptr(ws),
                                      _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_random_order")
    return out


def vecchia_maxmin_order(locs, seed: int = 0, out=None, ws=None, stream=None):
    """Approximate maxmin permutation (int64 [n]): rounds of per-cell elections over finer and finer
    grids, each round in hashed-index order.  Synchronises the stream once per round."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be float64 [n][2]")
    _dev_check(locs)
    n = locs.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=locs.device)
    if tuple(out.shape) != (n,) or out.dtype != torch.int64:
        raise ValueError("out must be int64 [n]")
    _dev_check(out)
    need = int(_load().vecchia_maxmin_workspace_size(n))
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=locs.device)
    rc = _load().vecchia_maxmin_order(_ptr(locs), n, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), _ptr(out),
                                      _ptr(ws), _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_maxmin_order")
    return out


def vecchia_morton_order(locs, out=None, ws=None, stream=None):
    """Morton (Z-order) permutation of the points: int64 [n], ties by index."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be float64 [n][2]")
    _dev_check(locs)
    n = locs.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=locs.device)
    if tuple(out.shape) != (n,) or out.dtype != torch.int64:
        raise ValueError("out must be int64 [n]")
    _dev_check(out)
    need = int(_load().vecchia_morton_workspace_size(n))
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=locs.device)
    rc = _load().vecchia_morton_order(_ptr(locs), n, _ptr(out), _ptr(ws), _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_morton_order")
    return out


# ------------------------------------------------------------------ estimation
def mle_default_options() -> MleOptions:
    opt = MleOptions()
    _load().vecchia_mle_default_options(ctypes.byref(opt))
    return opt


def vecchia_mle(locs, z, nbr, m: int, nu: float, theta0, options: MleOptions = None, ws=None, stream=None,
                cov=None):
    """Maximum-likelihood (sigma2, beta, tau2) at fixed nu (Matern, Euclidean), or under the covariance
    model cov = (family, metric, smoothness) when given (then nu is ignored).  Returns a dict with theta,
    loglik, grad, iterations, evaluations and round_trips (device launches with a read-back)."""
    n = _as_inputs(locs, z, nbr, m)
    c = _cov(cov if cov is not None else (MATERN, EUCLIDEAN, nu))
    need = int(_load().vecchia_mle_workspace_size(n, m))
    if ws is None or _nbytes(ws) < need:
        ws = torch.empty(need, dtype=torch.uint8, device=locs.device)
    th0 = (ctypes.c_double * 3)(*[float(x) for x in theta0])
    th = (ctypes.c_double * 3)()
    gr = (ctypes.c_double * 3)()
    ll = ctypes.c_double()
    it = ctypes.c_int32()
    ev = ctypes.c_int32()
    trips = ctypes.c_int32()
    rc = _load().vecchia_mle_cov(_ptr(locs), _ptr(z), _ptr(nbr) if m > 0 else None, n, int(m), ctypes.byref(c),
                                 th0, ctypes.byref(options) if options is not None else None, th, ctypes.byref(ll),
                                 gr, ctypes.byref(it), ctypes.byref(ev), ctypes.byref(trips), _ptr(ws), _nbytes(ws),
                                 _stream(stream))
    _check(rc, "vecchia_mle")
    return {"theta": np.array(th[:]), "loglik": ll.value, "grad": np.array(gr[:]), "iterations": it.value,
            "evaluations": ev.value, "round_trips": trips.value}


# ------------------------------------------------------------- KL harness
def vecchia_exact_loglik(locs, z, nu: float, theta, stream=None):
    """Exact log-likelihood (dense Cholesky on the GPU); z=None means y = 0.  Returns (out, status)."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be float64 [n][2]")
    _dev_check(locs, z)
    _theta_check(theta, locs.device)
    n = locs.shape[0]
    if z is not None and (z.dtype != torch.float64 or tuple(z.shape) != (n,)):
        raise ValueError("z must be float64 [n]")
    ws = torch.empty(int(_load().vecchia_exact_workspace_size(n)), dtype=torch.uint8, device=locs.device)
    out = torch.empty(1, dtype=torch.float64, device=locs.device)
    status = torch.empty(1, dtype=torch.int64, device=locs.device)
    rc = _load().vecchia_exact_loglik(_ptr(locs), _ptr(z), n, float(nu), _ptr(theta), _ptr(out), _ptr(status),
                                      _ptr(ws), _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_exact_loglik")
    return out, status


def vecchia_dense_logdet(A, z=None, stream=None):
    """log det A (and z^T A^-1 z with z) of an SPD float64 [n][n] device tensor, factored in place.

    A is read as column-major with leading dimension A.stride(0) when
    A.stride(1) == 1 (a row-major symmetric matrix is its own transpose),
    so any contiguous symmetric tensor works.  Returns (logdet, quad or None, status).
    """
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
        raise ValueError("A must be a float64 [n][n] tensor with unit column stride")
    if z is not None and (z.dtype != torch.float64 or tuple(z.shape) != (A.shape[0],) or not z.is_contiguous()):
        raise ValueError("z must be a contiguous float64 [n]")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    _dev_check(z)
    n = A.shape[0]
    ws = torch.empty(int(_load().vecchia_dense_logdet_workspace_size(n)), dtype=torch.uint8, device=A.device)
    logdet = torch.empty(1, dtype=torch.float64, device=A.device)
    quad = torch.empty(1, dtype=torch.float64, device=A.device) if z is not None else None
    status = torch.empty(1, dtype=torch.int64, device=A.device)
    rc = _load().vecchia_dense_logdet(_ptr(A), n, A.stride(0), _ptr(z), _ptr(logdet), _ptr(quad), _ptr(status),
                                      _ptr(ws), _nbytes(ws), _stream(stream))
    _check(rc, "vecchia_dense_logdet")
    return logdet, quad, status


def kl_curve(locs, ms, nu: float, theta, ordering: str = "random", seed: int = 0, stream=None) -> dict:
    """KL divergence of Eq. (9) against the conditioning size, for one ordering of the points.

    ordering: "random" (vecchia_random_order), "morton" (vecchia_morton_order),
    "maxmin" (vecchia_maxmin_order) or "given" (as passed).  The exact log-likelihood is computed once; each m
    takes GPU conditioning sets and one Vecchia evaluation at y = 0.
    Returns {"ordering", "exact", "exact_seconds", "kl": {m: KL}}.
    """
    n = locs.shape[0]
    if ordering == "random":
        locs = locs[vecchia_random_order(n, seed=seed, device=locs.device, stream=stream)].contiguous()
    elif ordering == "morton":
        locs = locs[vecchia_morton_order(locs, stream=stream)].contiguous()
    elif ordering == "maxmin":
        locs = locs[vecchia_maxmin_order(locs, seed=seed, stream=stream)].contiguous()
    elif ordering != "given":
        raise ValueError(f"unknown ordering {ordering!r}")
    t0 = time.perf_counter()
    ex, st = vecchia_exact_loglik(locs, None, nu, theta, stream=stream)
    raise_on_status(st)
    exact = float(ex.item())
    exact_seconds = time.perf_counter() - t0
    zero = torch.zeros(n, dtype=torch.float64, device=locs.device)
    kl = {}
    for m in ms:
        nbr = vecchia_knn(locs, int(m), stream=stream)
        va, st2 = vecchia_loglik(locs, zero, nbr, int(m), nu, theta, stream=stream)
        raise_on_status(st2)
        kl[int(m)] = exact - float(va.item())
        del nbr
    return {"ordering": ordering, "exact": exact, "exact_seconds": round(exact_seconds, 3), "kl": kl}


def kl_divergence(locs, nbr, m: int, nu: float, theta, stream=None) -> float:
    """Eq. (9): KL(N_0 || N_a) = l_0(theta; 0) - l_a(theta; 0), exact minus Vecchia log-likelihood at y = 0."""
    zero = torch.zeros(locs.shape[0], dtype=torch.float64, device=locs.device)
    ex, st = vecchia_exact_loglik(locs, None, nu, theta, stream=stream)
    va, st2 = vecchia_loglik(locs, zero, nbr, m, nu, theta, stream=stream)
    raise_on_status(st)
    raise_on_status(st2)
    return float(ex.item() - va.item())
