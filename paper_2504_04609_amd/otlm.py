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
STATUS_FALLBACK, STATUS_ABSORBED = 16, 32

EXPORTED = ("otlm_default_params", "otlm_make_kernel", "otlm_free_kernel", "otlm_kernel_info",
            "otlm_solve_batch", "otlm_objective", "otlm_status_str", "otlm_profile_enable",
            "otlm_profile_read", "otlm_ragged_default_opts", "otlm_ragged_create", "otlm_ragged_solve",
            "otlm_ragged_info", "otlm_ragged_profile_enable", "otlm_ragged_profile_read", "otlm_ragged_free",
            "otlm_mlp_create", "otlm_mlp_info", "otlm_mlp_set_norm", "otlm_mlp_set_loss_weights",
            "otlm_mlp_set_norm_stats", "otlm_mlp_get_norm", "otlm_mlp_grad",
            "otlm_mlp_train_step", "otlm_mlp_get_params", "otlm_mlp_set_params", "otlm_mlp_infer", "otlm_mlp_free")
PROFILE_CLASSES = ("kv_product", "weight_step", "u_update", "ktu_product", "convergence_test",
                   "kv_product_f64", "weight_prox_f64", "u_update_f64", "ktu_product_f64",
                   "kv_product_bf16", "ktu_product_bf16", "weight_mm_warmup")
RAGGED_PROFILE_CLASSES = ("kv_product", "weight_step", "ktu_product", "convergence_test", "weight_prox_newton")
RAGGED_TILES = ((128, 128), (128, 64), (64, 128), (64, 64))


class OtlmError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("lambda_", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("tol", ctypes.c_double),
                ("bulk_tol", ctypes.c_double), ("warm_probe", ctypes.c_double), ("absorb_tau", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32), ("fit", ctypes.c_int32),
                ("pen", ctypes.c_int32), ("prec", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("refine_sweeps", ctypes.c_int32), ("warm", ctypes.c_int32), ("wstep", ctypes.c_int32),
                ("inner_max", ctypes.c_int32), ("refine_check_every", ctypes.c_int32)]


class AdamW(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("weight_decay", ctypes.c_double)]


class RaggedOpts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("tile", ctypes.c_int32), ("newton_after", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


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
    lib.otlm_ragged_default_opts.argtypes = [ctypes.POINTER(RaggedOpts)]
    lib.otlm_ragged_default_opts.restype = None
    lib.otlm_ragged_create.argtypes = [vp, ctypes.c_int32, vp, vp, i64, ctypes.POINTER(Params),
                                       ctypes.POINTER(RaggedOpts), vp, ctypes.POINTER(vp)]
    lib.otlm_ragged_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.otlm_ragged_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(f64), ctypes.POINTER(i64)]
    lib.otlm_ragged_profile_enable.argtypes = [vp, ctypes.c_int32]
    lib.otlm_ragged_profile_read.argtypes = [vp, ctypes.POINTER(f64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.otlm_ragged_free.argtypes = [vp]
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.otlm_mlp_create.argtypes = [i32p, vp, vp, ctypes.POINTER(vp)]
    lib.otlm_mlp_info.argtypes = [vp, i32p, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.otlm_mlp_set_norm.argtypes = [vp, vp, vp, i64, vp]
    lib.otlm_mlp_get_norm.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.otlm_mlp_set_loss_weights.argtypes = [vp, vp, vp]
    lib.otlm_mlp_set_norm_stats.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.otlm_mlp_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    lib.otlm_mlp_train_step.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(AdamW), vp, vp]
    lib.otlm_mlp_get_params.argtypes = [vp, vp, vp]
    lib.otlm_mlp_set_params.argtypes = [vp, vp, vp]
    lib.otlm_mlp_infer.argtypes = [vp, vp, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
    lib.otlm_mlp_free.argtypes = [vp]
    for name in ("otlm_mlp_create", "otlm_mlp_info", "otlm_mlp_set_norm", "otlm_mlp_set_loss_weights",
                 "otlm_mlp_set_norm_stats", "otlm_mlp_get_norm", "otlm_mlp_grad",
                 "otlm_mlp_train_step", "otlm_mlp_get_params", "otlm_mlp_set_params", "otlm_mlp_infer",
                 "otlm_mlp_free"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("otlm_make_kernel", "otlm_free_kernel", "otlm_kernel_info", "otlm_solve_batch", "otlm_objective",
                 "otlm_profile_enable", "otlm_profile_read", "otlm_ragged_create", "otlm_ragged_solve",
                 "otlm_ragged_info", "otlm_ragged_profile_enable", "otlm_ragged_profile_read",
                 "otlm_ragged_free"):
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
    warm_probe: float = 0.0     # > 0: cold restart of warm starts whose first interval moves w more
    absorb_tau: float = 30.0    # FP64 refinement: move spectra with |log u| or |log v| above it to FP64
    wstep: str = "mm"           # "mm" (one MM step, Algorithm 1) or "exact" (ProxP by Newton)
    inner_max: int = 5
    refine_check_every: int = 2  # convergence test cadence of the refinement phase (0: check_every)

    def c(self) -> Params:
        p = Params()
        load().otlm_default_params(ctypes.byref(p))
        p.eps, p.lambda_, p.lambda2 = self.eps, self.lam, self.lam2
        p.alpha, p.beta, p.tol, p.bulk_tol = self.alpha, self.beta, self.tol, self.bulk_tol
        p.max_iter, p.check_every = self.max_iter, self.check_every
        p.fit, p.pen, p.prec = FIT[self.fit], PEN[self.pen], PREC[self.prec]
        p.refine, p.refine_sweeps = REFINE[self.refine], self.refine_sweeps
        p.warm = int(self.warm)
        p.warm_probe = self.warm_probe
        p.absorb_tau = self.absorb_tau
        p.wstep, p.inner_max = WSTEP[self.wstep], self.inner_max
        p.refine_check_every = self.refine_check_every
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
        nit = (ctypes.c_int64 * 6)()
        _check(load().otlm_profile_read(self.handle, ms, cnt, nit), "otlm_profile_read")
        out = {name: (ms[i], cnt[i]) for i, name in enumerate(PROFILE_CLASSES)}
        out["newton_iters"] = nit[0] + nit[1]
        out["newton_iters_fp32"], out["newton_iters_fp64"] = nit[0], nit[1]
        out["factorisations_fp32"], out["factorisations_fp64"] = nit[2], nit[3]
        out["hessian_entries_fp32"], out["hessian_entries_fp64"] = nit[4], nit[5]
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


class RaggedPlan:
    """A planned ragged batch (otlm_ragged_create): spectrum b uses kernel
    kernels[kernel_of[b]] (so n_b = that kernel's n) and a dictionary with
    kdim[b] columns.  Packed layouts as in include/otlm.h."""

    def __init__(self, kernels, kernel_of, kdim, params: SolveParams, use_graph: bool = True, tile: int = -1,
                 newton_after: int = 15, stream=None):
        import numpy as np
        self.kernels = list(kernels)  # the plan reads their K: keep them alive
        self.kernel_of = np.ascontiguousarray(kernel_of, dtype=np.int32)
        self.kdim = np.ascontiguousarray(kdim, dtype=np.int32)
        if self.kernel_of.shape != self.kdim.shape or self.kernel_of.ndim != 1:
            raise OtlmError("kernel_of and kdim must be 1-D arrays of one length")
        self.B = int(self.kernel_of.size)
        if self.B and (self.kernel_of.min() < 0 or self.kernel_of.max() >= len(self.kernels)):
            raise OtlmError("kernel_of out of range")
        ns = np.array([kk.n for kk in self.kernels], dtype=np.int64)
        self.n = ns[self.kernel_of] if self.B else np.zeros(0, np.int64)
        self.y_off = np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)
        self.w_off = np.concatenate([[0], np.cumsum(self.kdim)]).astype(np.int64)
        self.d_off = np.concatenate([[0], np.cumsum(self.n * self.kdim)]).astype(np.int64)
        self.params = params
        lib = load()
        handles = (ctypes.c_void_p * len(self.kernels))(*[kk.handle for kk in self.kernels])
        o = RaggedOpts()
        lib.otlm_ragged_default_opts(ctypes.byref(o))
        o.use_graph, o.tile, o.newton_after = int(use_graph), int(tile), int(newton_after)
        p = params.c()
        h = ctypes.c_void_p()
        _check(lib.otlm_ragged_create(handles, len(self.kernels), self.kernel_of.ctypes.data_as(ctypes.c_void_p),
                                      self.kdim.ctypes.data_as(ctypes.c_void_p), self.B, ctypes.byref(p),
                                      ctypes.byref(o), _stream(stream), ctypes.byref(h)), "otlm_ragged_create")
        self.handle = h

    def info(self):
        bm, bn = ctypes.c_int32(), ctypes.c_int32()
        tune = (ctypes.c_double * 4)()
        sizes = (ctypes.c_int64 * 4)()
        _check(load().otlm_ragged_info(self.handle, ctypes.byref(bm), ctypes.byref(bn), tune, sizes),
               "otlm_ragged_info")
        return {"tile": (bm.value, bn.value), "tune_ms": list(tune), "bins": sizes[0], "columns": sizes[1],
                "dict_entries": sizes[2], "device_bytes": sizes[3]}

    def profile(self, on: bool = True):
        _check(load().otlm_ragged_profile_enable(self.handle, int(on)), "otlm_ragged_profile_enable")

    def profile_read(self):
        ms = (ctypes.c_double * len(RAGGED_PROFILE_CLASSES))()
        cnt = (ctypes.c_int64 * len(RAGGED_PROFILE_CLASSES))()
        work = (ctypes.c_int64 * 3)()
        _check(load().otlm_ragged_profile_read(self.handle, ms, cnt, work), "otlm_ragged_profile_read")
        out = {name: (ms[i], cnt[i]) for i, name in enumerate(RAGGED_PROFILE_CLASSES)}
        out["product_macs"], out["weight_step_bytes"], out["newton_flops"] = work[0], work[1], work[2]
        return out

    def solve(self, D, Y, W=None, logV=None, want_logU=True, stream=None):
        """otlm_ragged_solve on packed CUDA tensors D [sum n_b k_b], Y [sum n_b].
        Returns packed W [sum k_b], logU / logV [sum n_b], iters / status [B]."""
        import torch
        nb, kb, db = int(self.y_off[-1]), int(self.w_off[-1]), int(self.d_off[-1])
        _need(D, torch.float32, (db,), "D")
        _need(Y, torch.float32, (nb,), "Y")
        dev = Y.device
        if self.params.warm:
            _need(W, torch.float32, (kb,), "W")
            _need(logV, torch.float32, (nb,), "logV")
        else:
            W = torch.empty(kb, device=dev, dtype=torch.float32) if W is None else W
            logV = torch.empty(nb, device=dev, dtype=torch.float32) if logV is None else logV
        logU = torch.empty(nb, device=dev, dtype=torch.float32) if want_logU else None
        iters = torch.empty(self.B, device=dev, dtype=torch.int32)
        status = torch.empty(self.B, device=dev, dtype=torch.int32)
        _check(load().otlm_ragged_solve(self.handle, _ptr(D), _ptr(Y), _ptr(W), _ptr(logU), _ptr(logV), _ptr(iters),
                                        _ptr(status), _stream(stream)), "otlm_ragged_solve")
        return {"W": W, "logU": logU, "logV": logV, "iters": iters, "status": status}

    def unpack_w(self, W, b):
        return W[int(self.w_off[b]):int(self.w_off[b + 1])]

    def unpack_n(self, X, b):
        return X[int(self.y_off[b]):int(self.y_off[b + 1])]

    def close(self):
        if getattr(self, "handle", None):
            load().otlm_ragged_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WarmStartMLP:
    """The warm-start network (otlm_mlp_*): dims = (in, h1, h2, out), initial
    flat parameters theta (FP32, host NumPy or CUDA tensor)."""

    def __init__(self, dims, theta, stream=None):
        import numpy as np
        import torch
        self.dims = tuple(int(d) for d in dims)
        d = (ctypes.c_int32 * 4)(*self.dims)
        if isinstance(theta, torch.Tensor):
            if theta.dtype != torch.float32 or not theta.is_contiguous():
                raise OtlmError("theta must be a contiguous float32 tensor")
            tp, self._keep = ctypes.c_void_p(theta.data_ptr()), theta
        else:
            self._keep = np.ascontiguousarray(theta, dtype=np.float32)
            tp = self._keep.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(load().otlm_mlp_create(d, tp, _stream(stream), ctypes.byref(h)), "otlm_mlp_create")
        self.handle = h
        self._keep = None
        self.nparam = self.info()["nparam"]

    def info(self):
        d = (ctypes.c_int32 * 4)()
        n, st = ctypes.c_int64(), ctypes.c_int64()
        _check(load().otlm_mlp_info(self.handle, d, ctypes.byref(n), ctypes.byref(st)), "otlm_mlp_info")
        return {"dims": tuple(d), "nparam": n.value, "step": st.value}

    def set_norm(self, X, T, stream=None):
        import torch
        N = X.shape[0]
        _need(X, torch.float32, (N, self.dims[0]), "X")
        _need(T, torch.float32, (N, self.dims[3]), "T")
        _check(load().otlm_mlp_set_norm(self.handle, _ptr(X), _ptr(T), N, _stream(stream)), "otlm_mlp_set_norm")

    def set_loss_weights(self, weights, stream=None):
        import numpy as np
        w = np.ascontiguousarray(weights, dtype=np.float32)
        if w.shape != (self.dims[3],):
            raise OtlmError(f"weights must have shape ({self.dims[3]},)")
        _check(load().otlm_mlp_set_loss_weights(self.handle, w.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "otlm_mlp_set_loss_weights")

    def set_norm_stats(self, in_mu, in_sd, out_mu, out_sd, stream=None):
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (in_mu, in_sd, out_mu, out_sd)]
        if arrs[0].shape != (self.dims[0],) or arrs[1].shape != (self.dims[0],) or \
                arrs[2].shape != (self.dims[3],) or arrs[3].shape != (self.dims[3],):
            raise OtlmError("standardisation statistics have the wrong shapes")
        ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
        _check(load().otlm_mlp_set_norm_stats(self.handle, *ptrs, _stream(stream)), "otlm_mlp_set_norm_stats")

    def get_norm(self, stream=None):
        import torch
        i_mu = torch.empty(self.dims[0], device="cuda", dtype=torch.float32)
        i_sd, o_mu, o_sd = torch.empty_like(i_mu), torch.empty(self.dims[3], device="cuda"), None
        o_sd = torch.empty_like(o_mu)
        _check(load().otlm_mlp_get_norm(self.handle, _ptr(i_mu), _ptr(i_sd), _ptr(o_mu), _ptr(o_sd),
                                        _stream(stream)), "otlm_mlp_get_norm")
        return i_mu, i_sd, o_mu, o_sd

    def grad(self, X, T, idx, stream=None):
        """(flat gradient, loss) on the minibatch rows idx (CUDA int32)."""
        import torch
        g = torch.empty(self.nparam, device=X.device, dtype=torch.float32)
        loss = torch.empty(1, device=X.device, dtype=torch.float32)
        _check(load().otlm_mlp_grad(self.handle, _ptr(X), _ptr(T), _ptr(idx), idx.numel(), _ptr(g), _ptr(loss),
                                    _stream(stream)), "otlm_mlp_grad")
        return g, loss

    def train_step(self, X, T, idx, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, loss=None,
                   stream=None):
        h = AdamW(lr, beta1, beta2, eps, weight_decay)
        _check(load().otlm_mlp_train_step(self.handle, _ptr(X), _ptr(T), _ptr(idx), idx.numel(), ctypes.byref(h),
                                          _ptr(loss), _stream(stream)), "otlm_mlp_train_step")

    def params(self, stream=None):
        import torch
        t = torch.empty(self.nparam, device="cuda", dtype=torch.float32)
        _check(load().otlm_mlp_get_params(self.handle, _ptr(t), _stream(stream)), "otlm_mlp_get_params")
        return t

    def set_params(self, theta, stream=None):
        _check(load().otlm_mlp_set_params(self.handle, _ptr(theta), _stream(stream)), "otlm_mlp_set_params")

    def infer(self, Y, n_u, n_v, prec="bf16", logU=None, logV=None, W=None, stream=None):
        """Split prediction (logU or None, logV [B, n_v], W [B, out - n_u - n_v])."""
        import torch
        B = Y.shape[0]
        _need(Y, torch.float32, (B, self.dims[0]), "Y")
        k = self.dims[3] - n_u - n_v
        logV = torch.empty((B, n_v), device=Y.device, dtype=torch.float32) if logV is None else logV
        W = torch.empty((B, k), device=Y.device, dtype=torch.float32) if W is None else W
        _check(load().otlm_mlp_infer(self.handle, _ptr(Y), B, PREC[prec], n_u, n_v, _ptr(logU), _ptr(logV), _ptr(W),
                                     _stream(stream)), "otlm_mlp_infer")
        return logU, logV, W

    def close(self):
        if getattr(self, "handle", None):
            load().otlm_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
