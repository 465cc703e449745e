"""Python binding of libocsc (ctypes): argument marshalling only.

Every function here has the name and argument order of the C call in
include/ocsc.h; device buffers are torch tensors (their ``data_ptr()`` is
passed), the context stream is torch's current stream at ``ocsc_init`` unless
another is given.  All arithmetic runs in the library's HIP kernels: if the
built library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
# OCSC_LIBRARY selects another build of the same library (the host-sanitized
# build that the CPU ABI tests load); by default the in-tree libocsc.so.
LIB_PATH = os.environ.get("OCSC_LIBRARY") or os.path.join(HERE, "libocsc.so")

OCSC_OK = 0
OCSC_E_INVALID_ARG = -1
OCSC_E_STATE = -2
OCSC_E_OOM = -3
OCSC_E_HIP = -4
OCSC_E_NUMERIC = -5
OCSC_E_UNSUPPORTED = -6

OCSC_FP64 = 0
OCSC_FP32 = 1
OCSC_FLAG_OWN_STREAM = 1
OCSC_FLAG_KEEP_HISTORY = 2
OCSC_FLAG_WARM_START = 4
OCSC_FLAG_CHOLESKY = 8
OCSC_FLAG_REFINE = 16

STATE = {"dict_hat": 0, "G": 1, "cinv": 2, "V": 3, "theta": 4, "zhat": 5, "xhat": 6, "H": 7, "sums": 8,
         "rhs": 9}
KERNEL_CLASS = {"fft": 0, "zstep": 1, "codeplane": 2, "history": 3, "dstep": 4, "vstep": 5, "other": 6}

EXPORTS = [
    "ocsc_default_opts", "ocsc_init", "ocsc_destroy", "ocsc_set_dictionary", "ocsc_get_dictionary",
    "ocsc_code_update", "ocsc_code_append", "ocsc_code_update_group", "ocsc_history_accumulate",
    "ocsc_dict_update",
    "ocsc_dict_update_group", "ocsc_objective",
    "ocsc_objective_terms", "ocsc_objective_noalloc", "ocsc_surrogate", "ocsc_diagnostics", "ocsc_sync",
    "ocsc_graph_create", "ocsc_graph_launch", "ocsc_graph_destroy",
    "ocsc_get_tuning", "ocsc_set_tuning", "ocsc_autotune",
    "ocsc_last_error", "ocsc_state_bytes", "ocsc_get_state", "ocsc_set_state", "ocsc_get_count",
    "ocsc_set_count", "ocsc_profile_enable", "ocsc_profile_read",
]


class OcscOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("iters_code", ctypes.c_int32),
        ("iters_dict", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("rho_dict", ctypes.c_double),
        ("stream", ctypes.c_void_p),
    ]


class OcscTuning(ctypes.Structure):
    _fields_ = [
        ("plane_threads", ctypes.c_int32),
        ("zstep_freqs", ctypes.c_int32),
        ("zstep_samples", ctypes.c_int32),
        ("col_bytes", ctypes.c_int32),
        ("row_block", ctypes.c_int32),
        ("chunk_samples", ctypes.c_int32),
        ("two_pass", ctypes.c_int32),
    ]


class OcscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libocsc status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the built library (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libocsc is not built ({path} missing); run `python -m paper_1706_06972_amd.build`")
    # torch ships its own HIP runtime; importing it first makes the library's
    # HIP calls resolve to that same runtime, so torch's device pointers and
    # streams are valid handles for the library.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "ocsc_default_opts": (None, [ctypes.POINTER(OcscOpts)]),
        "ocsc_init": (i32, [ctypes.POINTER(vp), i32, i32, i32, i32, i32, dbl, dbl, ctypes.POINTER(OcscOpts)]),
        "ocsc_destroy": (i32, [vp]),
        "ocsc_set_dictionary": (i32, [vp, vp]),
        "ocsc_get_dictionary": (i32, [vp, vp]),
        "ocsc_code_update": (i32, [vp, vp, i32, vp]),
        "ocsc_code_append": (i32, [vp, vp, i32, vp]),
        "ocsc_code_update_group": (i32, [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                         ctypes.POINTER(vp), i32]),
        "ocsc_dict_update_group": (i32, [ctypes.POINTER(vp), i32]),
        "ocsc_history_accumulate": (i32, [vp]),
        "ocsc_dict_update": (i32, [vp]),
        "ocsc_objective": (i32, [vp, vp, vp, i32, ctypes.POINTER(dbl)]),
        "ocsc_objective_terms": (i32, [vp, vp, vp, i32, ctypes.POINTER(dbl)]),
        "ocsc_objective_noalloc": (i32, [vp, vp, vp, i32, vp]),
        "ocsc_surrogate": (i32, [vp, vp, ctypes.POINTER(dbl)]),
        "ocsc_diagnostics": (i32, [vp, ctypes.POINTER(dbl)]),
        "ocsc_sync": (i32, [vp]),
        "ocsc_graph_create": (i32, [vp, vp, i32, vp, ctypes.POINTER(vp)]),
        "ocsc_graph_launch": (i32, [vp]),
        "ocsc_graph_destroy": (i32, [vp]),
        "ocsc_get_tuning": (i32, [vp, ctypes.POINTER(OcscTuning)]),
        "ocsc_set_tuning": (i32, [vp, ctypes.POINTER(OcscTuning)]),
        "ocsc_autotune": (i32, [vp, i32, ctypes.POINTER(OcscTuning), ctypes.POINTER(dbl)]),
        "ocsc_last_error": (ctypes.c_char_p, [vp]),
        "ocsc_state_bytes": (i32, [vp, i32, ctypes.POINTER(i64)]),
        "ocsc_get_state": (i32, [vp, i32, vp]),
        "ocsc_set_state": (i32, [vp, i32, vp]),
        "ocsc_get_count": (i32, [vp, ctypes.POINTER(i64)]),
        "ocsc_set_count": (i32, [vp, i64]),
        "ocsc_profile_enable": (i32, [vp, ctypes.c_uint]),
        "ocsc_profile_read": (i32, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(ctx, rc: int) -> None:
    if rc != OCSC_OK:
        msg = load().ocsc_last_error(ctx)
        raise OcscError(rc, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return t.data_ptr()


# ---------------------------------------------------------------------------
# The C calls, one for one
# ---------------------------------------------------------------------------

def ocsc_default_opts() -> OcscOpts:
    o = OcscOpts()
    load().ocsc_default_opts(ctypes.byref(o))
    return o


def ocsc_init(K, filt_h, filt_w, pad_h, pad_w, lam, rho, *, iters_code=10, iters_dict=10,
              max_batch=1, precision="f64", rho_dict=0.0, flags=0, stream=None):
    """Returns an opaque context handle (c_void_p)."""
    L = load()
    o = ocsc_default_opts()
    o.iters_code, o.iters_dict, o.max_batch = iters_code, iters_dict, max_batch
    o.flags = int(flags)
    o.precision = {"f64": OCSC_FP64, "f32": OCSC_FP32}[precision]
    o.rho_dict = float(rho_dict)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    o.stream = stream
    ctx = ctypes.c_void_p()
    rc = L.ocsc_init(ctypes.byref(ctx), K, filt_h, filt_w, pad_h, pad_w, float(lam), float(rho), ctypes.byref(o))
    _check(None, rc)
    return ctx


def ocsc_destroy(ctx) -> None:
    _check(None, load().ocsc_destroy(ctx))


def ocsc_set_dictionary(ctx, D) -> None:
    _check(ctx, load().ocsc_set_dictionary(ctx, _ptr(D)))


def ocsc_get_dictionary(ctx, D_out) -> None:
    _check(ctx, load().ocsc_get_dictionary(ctx, _ptr(D_out)))


def ocsc_code_update(ctx, x, B, codes_out=None) -> None:
    _check(ctx, load().ocsc_code_update(ctx, _ptr(x), int(B), _ptr(codes_out)))


def ocsc_code_append(ctx, x, B, codes_out=None) -> None:
    _check(ctx, load().ocsc_code_append(ctx, _ptr(x), int(B), _ptr(codes_out)))


def ocsc_code_update_group(ctxs, xs, Bs, codes_out=None) -> None:
    """One persistent launch coding xs[s] (Bs[s] samples) on ctxs[s] for every s."""
    n = len(ctxs)
    if not (len(xs) == len(Bs) == n) or (codes_out is not None and len(codes_out) != n):
        raise ValueError("ctxs, xs, Bs (and codes_out) must have the same length")
    carr = (ctypes.c_void_p * n)(*[c.value for c in ctxs])
    xarr = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
    barr = (ctypes.c_int * n)(*[int(b) for b in Bs])
    oarr = None if codes_out is None else (ctypes.c_void_p * n)(*[_ptr(c) for c in codes_out])
    _check(ctxs[0], load().ocsc_code_update_group(carr, xarr, barr, oarr, n))


def ocsc_dict_update_group(ctxs) -> None:
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    _check(ctxs[0], load().ocsc_dict_update_group(arr, len(ctxs)))


def ocsc_history_accumulate(ctx) -> None:
    _check(ctx, load().ocsc_history_accumulate(ctx))


def ocsc_dict_update(ctx) -> None:
    _check(ctx, load().ocsc_dict_update(ctx))


def ocsc_objective(ctx, x, codes, B):
    out = (ctypes.c_double * int(B))()
    _check(ctx, load().ocsc_objective(ctx, _ptr(x), _ptr(codes), int(B), out))
    return list(out)


def ocsc_objective_terms(ctx, x, codes, B):
    """[(1/2 ||x_b - reconstruction_b||^2, ||U_b||_1) for each sample b]."""
    out = (ctypes.c_double * (2 * int(B)))()
    _check(ctx, load().ocsc_objective_terms(ctx, _ptr(x), _ptr(codes), int(B), out))
    return [(out[2 * b], out[2 * b + 1]) for b in range(int(B))]


def ocsc_objective_noalloc(ctx, x, codes, B, out) -> None:
    """Objective per sample into the device tensor ``out`` (B doubles), using the
    library's static scratch; enqueued, not waited for."""
    _check(ctx, load().ocsc_objective_noalloc(ctx, _ptr(x), _ptr(codes), int(B), _ptr(out)))


def ocsc_surrogate(ctx, D=None) -> float:
    out = ctypes.c_double()
    _check(ctx, load().ocsc_surrogate(ctx, _ptr(D), ctypes.byref(out)))
    return out.value


def ocsc_diagnostics(ctx, K):
    """Dict with the primal residual, the dictionary norm and per-filter norms."""
    out = (ctypes.c_double * (2 + 2 * int(K)))()
    _check(ctx, load().ocsc_diagnostics(ctx, out))
    v = list(out)
    return {"primal_residual": v[0], "dict_norm": v[1], "V_norms": v[2:2 + K], "D_norms": v[2 + K:2 + 2 * K]}


def ocsc_graph_create(ctx, x, B, codes_out=None):
    """Returns an opaque graph handle (c_void_p) for two captured steps."""
    h = ctypes.c_void_p()
    _check(ctx, load().ocsc_graph_create(ctx, _ptr(x), int(B), _ptr(codes_out), ctypes.byref(h)))
    return h


def ocsc_graph_launch(ctx, h) -> None:
    _check(ctx, load().ocsc_graph_launch(h))


def ocsc_graph_destroy(h) -> None:
    _check(None, load().ocsc_graph_destroy(h))


TUNING_FIELDS = ("plane_threads", "zstep_freqs", "zstep_samples", "col_bytes", "row_block", "chunk_samples",
                 "two_pass")


def ocsc_get_tuning(ctx) -> dict:
    t = OcscTuning()
    _check(ctx, load().ocsc_get_tuning(ctx, ctypes.byref(t)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def ocsc_set_tuning(ctx, **shape) -> None:
    """Change some fields of the launch shape (the others stay)."""
    cur = ocsc_get_tuning(ctx)
    unknown = set(shape) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    cur.update(shape)
    t = OcscTuning(**cur)
    _check(ctx, load().ocsc_set_tuning(ctx, ctypes.byref(t)))


def ocsc_autotune(ctx, B):
    """Returns (chosen shape as a dict, ms of one Z-step + one plane launch)."""
    t, ms = OcscTuning(), ctypes.c_double()
    _check(ctx, load().ocsc_autotune(ctx, int(B), ctypes.byref(t), ctypes.byref(ms)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}, ms.value


def ocsc_sync(ctx) -> None:
    _check(ctx, load().ocsc_sync(ctx))


def ocsc_last_error(ctx) -> str:
    m = load().ocsc_last_error(ctx)
    return m.decode() if m else ""


def ocsc_state_bytes(ctx, which) -> int:
    n = ctypes.c_int64()
    _check(ctx, load().ocsc_state_bytes(ctx, STATE.get(which, which), ctypes.byref(n)))
    return n.value


def ocsc_get_state(ctx, which, dst) -> None:
    _check(ctx, load().ocsc_get_state(ctx, STATE.get(which, which), _ptr(dst)))


def ocsc_set_state(ctx, which, src) -> None:
    _check(ctx, load().ocsc_set_state(ctx, STATE.get(which, which), _ptr(src)))


def ocsc_get_count(ctx) -> int:
    n = ctypes.c_int64()
    _check(ctx, load().ocsc_get_count(ctx, ctypes.byref(n)))
    return n.value


def ocsc_set_count(ctx, t) -> None:
    _check(ctx, load().ocsc_set_count(ctx, int(t)))


def ocsc_profile_enable(ctx, classes=()) -> None:
    mask = 0
    for c in classes:
        mask |= 1 << KERNEL_CLASS.get(c, c)
    _check(ctx, load().ocsc_profile_enable(ctx, mask))


def ocsc_profile_read(ctx, cls):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(ctx, load().ocsc_profile_read(ctx, KERNEL_CLASS.get(cls, cls), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------------------
# Convenience wrapper: owns a context, allocates output tensors.
# ---------------------------------------------------------------------------

class OCSC:
    """A learner on the current CUDA/HIP device (see include/ocsc.h)."""

    def __init__(self, K, filt_h, filt_w, pad_h, pad_w, lam, rho, *, iters_code=10, iters_dict=10,
                 max_batch=1, precision="f64", rho_dict=0.0, keep_history=False, warm_start=False,
                 cholesky=False, refine=False, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.K, self.filt, self.shape = K, (filt_h, filt_w), (pad_h, pad_w)
        self.max_batch = max_batch
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        with torch.cuda.device(self.device):
            flags = ((OCSC_FLAG_KEEP_HISTORY if keep_history else 0) | (OCSC_FLAG_WARM_START if warm_start else 0)
                     | (OCSC_FLAG_CHOLESKY if cholesky else 0) | (OCSC_FLAG_REFINE if refine else 0))
            self.ctx = ocsc_init(K, filt_h, filt_w, pad_h, pad_w, lam, rho, iters_code=iters_code,
                                 iters_dict=iters_dict, max_batch=max_batch, precision=precision,
                                 rho_dict=rho_dict, flags=flags)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            ocsc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        t = self.torch.as_tensor(a, dtype=self.dtype, device=self.device)
        return t.contiguous()

    def set_dictionary(self, D):
        D = self._dev(D)
        if tuple(D.shape) != (self.K,) + self.filt:
            raise ValueError("dictionary must have shape (K, filt_h, filt_w)")
        ocsc_set_dictionary(self.ctx, D)
        ocsc_sync(self.ctx)

    def get_dictionary(self):
        D = self.torch.empty((self.K,) + self.filt, dtype=self.dtype, device=self.device)
        ocsc_get_dictionary(self.ctx, D)
        ocsc_sync(self.ctx)
        return D

    def code_update(self, x, codes=None, want_codes=True):
        x = self._dev(x)
        if x.dim() == 2:
            x = x[None]
        B = x.shape[0]
        if tuple(x.shape[1:]) != self.shape:
            raise ValueError("samples must have shape (B, pad_h, pad_w)")
        if codes is None and want_codes:
            codes = self.torch.empty((B, self.K) + self.shape, dtype=self.dtype, device=self.device)
        ocsc_code_update(self.ctx, x, B, codes)
        self._x_keep = x
        return codes

    def code_append(self, x, codes=None, want_codes=True):
        """Code samples into the next pending slots (see ocsc_code_append)."""
        x = self._dev(x)
        if x.dim() == 2:
            x = x[None]
        B = x.shape[0]
        if tuple(x.shape[1:]) != self.shape:
            raise ValueError("samples must have shape (B, pad_h, pad_w)")
        if codes is None and want_codes:
            codes = self.torch.empty((B, self.K) + self.shape, dtype=self.dtype, device=self.device)
        ocsc_code_append(self.ctx, x, B, codes)
        return codes

    def history_accumulate(self):
        ocsc_history_accumulate(self.ctx)

    def dict_update(self):
        ocsc_dict_update(self.ctx)

    @staticmethod
    def code_update_group(models, xs, want_codes=True):
        """Code xs[i] (B_i x pad_h_i x pad_w_i) on models[i], all iterations of
        all grids in one persistent launch; returns the codes per model."""
        xs = [m._dev(x) for m, x in zip(models, xs)]
        xs = [x[None] if x.dim() == 2 else x for x in xs]
        for m, x in zip(models, xs):
            if tuple(x.shape[1:]) != m.shape:
                raise ValueError("samples must have shape (B, pad_h, pad_w) of their model")
        codes = None
        if want_codes:
            codes = [m.torch.empty((x.shape[0], m.K) + m.shape, dtype=m.dtype, device=m.device)
                     for m, x in zip(models, xs)]
        ocsc_code_update_group([m.ctx for m in models], xs, [x.shape[0] for x in xs], codes)
        for m, x in zip(models, xs):
            m._x_keep = x
        return codes

    @staticmethod
    def dict_update_group(models):
        """Shared-dictionary DictOCSC over learners on different grids."""
        ocsc_dict_update_group([m.ctx for m in models])

    def step(self, x, codes=None, want_codes=True):
        c = self.code_update(x, codes, want_codes)
        self.history_accumulate()
        self.dict_update()
        return c

    def objective(self, x, codes):
        x = self._dev(x)
        if x.dim() == 2:
            x = x[None]
        codes = self._dev(codes)
        if codes.dim() == 3:
            codes = codes[None]
        return ocsc_objective(self.ctx, x, codes, x.shape[0])

    def objective_noalloc(self, x, codes, out=None):
        """Objective per sample into a device tensor of B doubles, through the
        allocation-free call (the library's static scratch); not waited for."""
        x = self._dev(x)
        if x.dim() == 2:
            x = x[None]
        codes = self._dev(codes)
        if codes.dim() == 3:
            codes = codes[None]
        if out is None:
            out = self.torch.empty(x.shape[0], dtype=self.torch.float64, device=self.device)
        ocsc_objective_noalloc(self.ctx, x, codes, x.shape[0], out)
        return out

    def objective_terms(self, x, codes):
        x = self._dev(x)
        if x.dim() == 2:
            x = x[None]
        codes = self._dev(codes)
        if codes.dim() == 3:
            codes = codes[None]
        return ocsc_objective_terms(self.ctx, x, codes, x.shape[0])

    def surrogate(self, D=None):
        """Online surrogate F_t at the current dictionary, or at spatial filters D."""
        if D is not None:
            D = self._dev(D)
            if tuple(D.shape) != (self.K,) + self.filt:
                raise ValueError("filters must have shape (K, filt_h, filt_w)")
        return ocsc_surrogate(self.ctx, D)

    def diagnostics(self):
        return ocsc_diagnostics(self.ctx, self.K)

    def sync(self):
        ocsc_sync(self.ctx)

    @property
    def tuning(self) -> dict:
        return ocsc_get_tuning(self.ctx)

    def set_tuning(self, **shape):
        ocsc_set_tuning(self.ctx, **shape)

    def autotune(self, B=None):
        """Pick the fastest code-update launch shapes for batches of B samples
        (default max_batch); returns (shape, ms per code iteration)."""
        return ocsc_autotune(self.ctx, self.max_batch if B is None else B)

    def state(self, which):
        n = ocsc_state_bytes(self.ctx, which)
        dt = self.torch.float64 if which in ("sums", STATE["sums"]) else self.dtype
        buf = self.torch.empty(n // dt.itemsize, dtype=dt, device=self.device)
        ocsc_get_state(self.ctx, which, buf)
        return buf

    def set_state(self, which, flat):
        if which in ("sums", STATE["sums"]):
            t = self.torch.as_tensor(flat, dtype=self.torch.float64, device=self.device).contiguous()
        else:
            t = self._dev(flat)
        ocsc_set_state(self.ctx, which, t.reshape(-1))

    @property
    def count(self):
        return ocsc_get_count(self.ctx)

    @count.setter
    def count(self, t):
        ocsc_set_count(self.ctx, t)
