"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1706_06972_amd import ocsc as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "ocsc.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ocsc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_bound_calls():
    assert declared_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = B.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def init_rc(K=16, fh=11, fw=11, ph=64, pw=64, lam=1.0, rho=1.0, opts=None):
    L = B.load()
    ctx = ctypes.c_void_p()
    rc = L.ocsc_init(ctypes.byref(ctx), K, fh, fw, ph, pw, lam, rho, opts)
    return rc, ctx, B.ocsc_last_error(None)


@pytest.mark.parametrize("kw, text", [
    (dict(K=0), "K must be"),
    (dict(ph=48), "powers of two"),
    (dict(pw=2048), "powers of two"),
    (dict(fh=0), "filt"),
    (dict(fw=65), "filt"),
    (dict(lam=-1.0), "lambda"),
    (dict(rho=0.0), "rho"),
    (dict(rho=float("nan")), "rho"),
])
def test_init_rejects_bad_arguments_before_device_work(kw, text):
    rc, ctx, msg = init_rc(**kw)
    assert rc == B.OCSC_E_INVALID_ARG
    assert ctx.value is None
    assert text in msg


def test_init_rejects_bad_opts():
    o = B.ocsc_default_opts()
    assert (o.iters_code, o.iters_dict, o.max_batch, o.precision) == (10, 10, 1, B.OCSC_FP64)
    o.struct_size = 8
    assert init_rc(opts=ctypes.byref(o))[0] == B.OCSC_E_INVALID_ARG
    for field, val in (("iters_code", 0), ("iters_dict", 0), ("max_batch", 0), ("precision", 7),
                       ("flags", 64), ("flags", B.OCSC_FLAG_KEEP_HISTORY | 32)):
        o = B.ocsc_default_opts()
        setattr(o, field, val)
        assert init_rc(opts=ctypes.byref(o))[0] == B.OCSC_E_INVALID_ARG, field


def test_refinement_needs_the_cholesky_form():
    o = B.ocsc_default_opts()
    o.precision, o.flags = B.OCSC_FP32, B.OCSC_FLAG_REFINE
    rc, ctx, msg = init_rc(opts=ctypes.byref(o))
    assert rc == B.OCSC_E_UNSUPPORTED and ctx.value is None
    assert "OCSC_FLAG_REFINE" in msg


def test_cholesky_form_limits():
    for prec, K, extra in ((B.OCSC_FP64, 16, 0), (B.OCSC_FP32, 257, 0), (B.OCSC_FP32, 16, B.OCSC_FLAG_WARM_START)):
        o = B.ocsc_default_opts()
        o.precision, o.flags = prec, B.OCSC_FLAG_CHOLESKY | extra
        rc, _, msg = init_rc(K=K, opts=ctypes.byref(o))
        assert rc == B.OCSC_E_UNSUPPORTED and "Cholesky" in msg
    # K > 128 is only offered in the Cholesky form (its D-step streams C_p)
    o = B.ocsc_default_opts()
    o.precision = B.OCSC_FP32
    rc, _, msg = init_rc(K=200, opts=ctypes.byref(o))
    assert rc == B.OCSC_E_UNSUPPORTED and "Cholesky form" in msg


def test_unsupported_sizes_are_reported():
    for ph, pw in ((1024, 1024), (128, 256), (512, 64)):
        rc, _, msg = init_rc(ph=ph, pw=pw)
        assert rc == B.OCSC_E_UNSUPPORTED and "256, 512" in msg, (ph, pw)
    # the Sherman-Morrison form holds C_p in LDS: FP64 K <= 92, FP32 K <= 128
    o = B.ocsc_default_opts()
    o.precision = B.OCSC_FP64
    rc, _, msg = init_rc(K=93, opts=ctypes.byref(o))
    assert rc == B.OCSC_E_UNSUPPORTED and "LDS" in msg
    o.precision = B.OCSC_FP32
    rc, _, msg = init_rc(K=129, opts=ctypes.byref(o))
    assert rc == B.OCSC_E_UNSUPPORTED and "Cholesky form" in msg
    # the largest sizes pass the checks (without a GPU the call then fails in HIP)
    for prec, K in ((B.OCSC_FP64, 92), (B.OCSC_FP32, 128)):
        o.precision = prec
        rc, ctx, msg = init_rc(K=K, ph=32, pw=32, opts=ctypes.byref(o))
        assert rc in (B.OCSC_OK, B.OCSC_E_HIP), (K, msg)
        if rc == B.OCSC_OK:
            B.load().ocsc_destroy(ctx)


def test_null_context_calls():
    L = B.load()
    assert L.ocsc_destroy(None) == B.OCSC_OK
    for name in ("ocsc_history_accumulate", "ocsc_dict_update", "ocsc_sync"):
        assert getattr(L, name)(None) == B.OCSC_E_INVALID_ARG
    assert L.ocsc_code_update(None, None, 1, None) == B.OCSC_E_INVALID_ARG
    out = (ctypes.c_double * 4)()
    assert L.ocsc_surrogate(None, None, out) == B.OCSC_E_INVALID_ARG
    assert L.ocsc_diagnostics(None, out) == B.OCSC_E_INVALID_ARG
    assert L.ocsc_objective_terms(None, None, None, 1, out) == B.OCSC_E_INVALID_ARG
    t = B.OcscTuning()
    assert L.ocsc_get_tuning(None, ctypes.byref(t)) == B.OCSC_E_INVALID_ARG
    assert L.ocsc_set_tuning(None, ctypes.byref(t)) == B.OCSC_E_INVALID_ARG
    assert L.ocsc_autotune(None, 1, None, None) == B.OCSC_E_INVALID_ARG


def test_no_device_is_a_hip_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, ctx, msg = init_rc()
    assert rc == B.OCSC_E_HIP and ctx.value is None and msg
