"""Host-only checks of the C-ABI library: it loads, exports every function that
include/otlm.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2504_04609_amd import otlm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "otlm.h")

needs_lib = pytest.mark.skipif(not os.path.exists(otlm.LIB_PATH), reason="libotlm.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(otlm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("otlm_make_kernel", "otlm_solve_batch", "otlm_objective", "otlm_free_kernel"):
        assert required in names
    assert set(names) == set(otlm.EXPORTED)


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(otlm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


@needs_lib
def test_params_struct_matches_header():
    # 9 doubles + 10 int32 in include/otlm.h
    assert ctypes.sizeof(otlm.Params) == 9 * 8 + 11 * 4 + 4  # eleven int32 fields, tail padding to 8 bytes
    p = otlm.Params()
    otlm.load().otlm_default_params(ctypes.byref(p))
    assert p.fit == otlm.FIT["kl"] and p.pen == otlm.PEN["none"] and p.max_iter == 1000
    assert p.check_every == 10 and p.tol == pytest.approx(1e-6) and p.refine_check_every == 2
    assert p.wstep == 0 and p.inner_max == 5 and p.refine == 0 and p.refine_sweeps == 200
    assert p.bulk_tol == pytest.approx(1e-4) and p.absorb_tau == 30.0 and p.warm_probe == 0.0


@needs_lib
def test_argument_errors_before_any_launch():
    lib = otlm.load()
    h = ctypes.c_void_p()
    assert lib.otlm_make_kernel(None, 16, 0.1, None, ctypes.byref(h)) == -1
    assert lib.otlm_make_kernel(ctypes.c_void_p(16), 0, 0.1, None, ctypes.byref(h)) == -1
    assert lib.otlm_make_kernel(ctypes.c_void_p(16), 16, -1.0, None, ctypes.byref(h)) == -1
    p = otlm.Params()
    lib.otlm_default_params(ctypes.byref(p))
    assert lib.otlm_solve_batch(None, None, 4, None, 1, ctypes.byref(p), None, None, None, None, None, None) == -1
    assert lib.otlm_objective(None, None, None, 4, None, 1, ctypes.byref(p), None, None, None, None, None) == -1
    assert lib.otlm_free_kernel(None) == 0
    assert lib.otlm_status_str(-1) == b"invalid argument"
    assert lib.otlm_status_str(0) == b"ok"


@needs_lib
def test_ragged_opts_and_argument_errors():
    lib = otlm.load()
    assert ctypes.sizeof(otlm.RaggedOpts) == 16
    o = otlm.RaggedOpts()
    lib.otlm_ragged_default_opts(ctypes.byref(o))
    assert o.use_graph == 1 and o.tile == -1 and o.newton_after == 15
    p = otlm.Params()
    lib.otlm_default_params(ctypes.byref(p))
    h = ctypes.c_void_p()
    ko = (ctypes.c_int32 * 2)(0, 0)
    kd = (ctypes.c_int32 * 2)(4, 4)
    # no kernels / bad counts / null output: rejected before any HIP call
    assert lib.otlm_ragged_create(None, 1, ko, kd, 2, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    kernels = (ctypes.c_void_p * 1)(None)
    assert lib.otlm_ragged_create(kernels, 0, ko, kd, 2, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert lib.otlm_ragged_create(kernels, 1, ko, kd, 0, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert lib.otlm_ragged_create(kernels, 1, ko, kd, 2, ctypes.byref(p), None, None, None) == -1
    assert lib.otlm_ragged_create(kernels, 9, ko, kd, 2, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert lib.otlm_ragged_solve(None, None, None, None, None, None, None, None, None) == -1
    assert lib.otlm_ragged_info(None, None, None, None, None) == -1
    assert lib.otlm_ragged_free(None) == 0
