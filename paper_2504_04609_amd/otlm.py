"""Thin ctypes binding of libotlm (include/otlm.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch tensors supply device memory and the stream; nothing here computes.
Importing works without a GPU; calling anything that needs the library raises
if ``libotlm.so`` has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libotlm.so")

FIT = {"balanced": 0, "kl": 1, "tv": 2, "l2": 3, "l2tv": 4, "poisson": 5}
PEN = {"none": 0, "l1": 1, "l2sq": 2, "en": 3}
PREC = {"fp32": 0, "bf16": 1}
REFINE = {"none": 0, "fp32": 1, "fp64": 2}
WSTEP = {"mm": 0, "exact": 1}

STATUS_CONVERGED, STATUS_MAX_ITER, STATUS_NONFINITE, STATUS_STAGNATED = 1, 2, 4, 8

EXPORTED = ("otlm_default_params", "otlm_make_kernel", "otlm_free_kernel", "otlm_kernel_info",
            "otlm_solve_batch", "otlm_objective", "otlm_status_str", "otlm_profile_enable",
            "otlm_profile_read")
PROFILE_CLASSES = ("kv_product", "weight_step", "u_update", "ktu_product", "convergence_test",
                   "kv_product_f64", "weight_prox_f64", "u_update_f64", "ktu_product_f64",
                   "kv_product_bf16", "ktu_product_bf16")


class OtlmError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("lambda_", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("tol", ctypes.c_double),
                ("bulk_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32), ("fit", ctypes.c_int32),
                ("pen", ctypes.c_int32), ("prec", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("refine_sweeps", ctypes.c_int32), ("warm", ctypes.c_int32), ("wstep", ctypes.c_int32),
                ("inner_max", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libotlm.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OtlmError(f"{LIB_PATH} is not built; run `python -m paper_2504_04609_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib.otlm_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.otlm_default_params.restype = None
    lib.otlm_make_kernel.argtypes = [vp, i64, f64, vp, ctypes.POINTER(vp)]
    lib.otlm_free_kernel.argtypes = [vp]
    lib.otlm_kernel_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(f64)]
    lib.otlm_solve_batch.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(Params), vp, vp, vp, vp, vp, vp]
    lib.otlm_objective.argtypes = [vp, vp, vp, i64, vp, i64, ctypes.POINTER(Params), vp, vp, vp, vp, vp]
    lib.otlm_profile_enable.argtypes = [vp, ctypes.c_int32]
    lib.otlm_profile_read.argtypes = [vp, ctypes.POINTER(f64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.otlm_status_str.argtypes = [ctypes.c_int]
    lib.otlm_status_str.restype = ctypes.c_char_p
    for name in ("otlm_make_kernel", "otlm_free_kernel", "otlm_kernel_info", "otlm_solve_batch", "otlm_objective",
                 "otlm_profile_enable", "otlm_profile_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = load().otlm_status_str(rc).decode()
        raise OtlmError(f"{what} failed: {msg} ({rc})")


@dataclasses.dataclass
class SolveParams:
    eps: float
    fit: str = "kl"
    pen: str = "none"
    lam: float = 1.0
    lam2: float = 0.0
    alpha: float = 0.0
    beta: float = 0.0
    tol: float = 1e-6
    max_iter: int = 1000
    check_every: int = 10
    prec: str = "fp32"          # bulk-phase products: "fp32" or "bf16"
    refine: str = "none"        # refinement phase: "none", "fp32" or "fp64"
    refine_sweeps: int = 200
    bulk_tol: float = 1e-4
    warm: bool = False
    wstep: str = "mm"           # "mm" (one MM step, Algorithm 1) or "exact" (ProxP by Newton)
    inner_max: int = 5

    def c(self) -> Params:
        p = Params()
        load().otlm_default_params(ctypes.byref(p))
        p.eps, p.lambda_, p.lambda2 = self.eps, self.lam, self.lam2
        p.alpha, p.beta, p.tol, p.bulk_tol = self.alpha, self.beta, self.tol, self.bulk_tol
        p.max_iter, p.check_every = self.max_iter, self.check_every
        p.fit, p.pen, p.prec = FIT[self.fit], PEN[self.pen], PREC[self.prec]
        p.refine, p.refine_sweeps = REFINE[self.refine], self.refine_sweeps
        p.warm = int(self.warm)
        p.wstep, p.inner_max = WSTEP[self.wstep], self.inner_max
        return p


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise OtlmError(f"{name} must be a contiguous CUDA {dtype} tensor")
    if tuple(t.shape) != tuple(shape):
        raise OtlmError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class GibbsKernel:
    """Owns the device Gibbs kernel K = exp(-C / eps) (otlm_make_kernel)."""

    def __init__(self, C, eps: float, stream=None):
        import torch
        n = C.shape[0]
        _need(C, torch.float64, (n, n), "C")
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.otlm_make_kernel(_ptr(C), n, float(eps), _stream(stream), ctypes.byref(h)), "otlm_make_kernel")
        self.handle, self.n, self.eps = h, n, float(eps)

    def info(self):
        n, sym, eps = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
        _check(load().otlm_kernel_info(self.handle, ctypes.byref(n), ctypes.byref(sym), ctypes.byref(eps)),
               "otlm_kernel_info")
        return n.value, bool(sym.value), eps.value

    def profile(self, on: bool = True):
        """Enable (and reset) or disable per-kernel event timing in the solve."""
        _check(load().otlm_profile_enable(self.handle, int(on)), "otlm_profile_enable")

    def profile_read(self):
        """Mean ms per launch and launch count for each timed kernel class."""
        ms = (ctypes.c_double * len(PROFILE_CLASSES))()
        cnt = (ctypes.c_int64 * len(PROFILE_CLASSES))()
        nit = ctypes.c_int64()
        _check(load().otlm_profile_read(self.handle, ms, cnt, ctypes.byref(nit)), "otlm_profile_read")
        out = {name: (ms[i], cnt[i]) for i, name in enumerate(PROFILE_CLASSES)}
        out["newton_iters"] = nit.value
        return out

    def close(self):
        if getattr(self, "handle", None):
            load().otlm_free_kernel(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, D, Y, params: SolveParams, W=None, logV=None, want_logU=True, stream=None):
        """otlm_solve_batch.  D [n,k] f32, Y [B,n] f32 (CUDA).  Returns a dict of
        CUDA tensors W [B,k], logU [B,n] (or None), logV [B,n], iters [B], status [B]."""
        import torch
        n = self.n
        k = D.shape[1]
        B = Y.shape[0]
        _need(D, torch.float32, (n, k), "D")
        _need(Y, torch.float32, (B, n), "Y")
        dev = Y.device
        if params.warm:
            _need(W, torch.float32, (B, k), "W")
            _need(logV, torch.float32, (B, n), "logV")
        else:
            W = torch.empty((B, k), device=dev, dtype=torch.float32) if W is None else W
            logV = torch.empty((B, n), device=dev, dtype=torch.float32) if logV is None else logV
        logU = torch.empty((B, n), device=dev, dtype=torch.float32) if want_logU else None
        iters = torch.empty(B, device=dev, dtype=torch.int32)
        status = torch.empty(B, device=dev, dtype=torch.int32)
        p = params.c()
        _check(load().otlm_solve_batch(self.handle, _ptr(D), k, _ptr(Y), B, ctypes.byref(p), _ptr(W), _ptr(logU),
                                       _ptr(logV), _ptr(iters), _ptr(status), _stream(stream)),
               "otlm_solve_batch")
        return {"W": W, "logU": logU, "logV": logV, "iters": iters, "status": status}

    def objective(self, C, D, Y, params: SolveParams, W, logU, logV, stream=None):
        """otlm_objective: FP64 [B, 6] = primal, dual, <C,Q>, src_err, tgt_kkt, w_kkt."""
        import torch
        n = self.n
        k = D.shape[1]
        B = Y.shape[0]
        _need(C, torch.float64, (n, n), "C")
        _need(D, torch.float32, (n, k), "D")
        _need(Y, torch.float32, (B, n), "Y")
        _need(W, torch.float32, (B, k), "W")
        _need(logU, torch.float32, (B, n), "logU")
        _need(logV, torch.float32, (B, n), "logV")
        out = torch.empty((B, 6), device=Y.device, dtype=torch.float64)
        p = params.c()
        _check(load().otlm_objective(self.handle, _ptr(C), _ptr(D), k, _ptr(Y), B, ctypes.byref(p), _ptr(W),
                                     _ptr(logU), _ptr(logV), _ptr(out), _stream(stream)), "otlm_objective")
        return out
