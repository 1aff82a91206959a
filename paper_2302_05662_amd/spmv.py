"""ctypes binding of libspmv.so (include/spmv.h), with the same function names.

Argument marshalling only: every computation runs in the library's HIP
kernels. Torch tensors supply device memory and ``torch.cuda`` streams; host
inputs may also be NumPy arrays. The library must have been built
(``paper_2302_05662_amd.build.build()``); importing this module without it
raises ImportError rather than falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspmv.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "spmv.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2302_05662_amd.build.build()")

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7) as
# /opt/rocm's. Loading torch first makes that one runtime serve the whole
# process, so torch tensors, streams and the library share one device context.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---- enums (mirror include/spmv.h) -------------------------------------------------

SPMV_OK = 0
STATUS_NAMES = ("OK", "INVALID_ARG", "OUT_OF_BOUNDS", "DUPLICATE", "NOT_CONVERTED",
                "NOT_APPLICABLE", "OOM", "HIP", "NO_MODEL")
SPMV_FMT_CSR, SPMV_FMT_COO, SPMV_FMT_ELL, SPMV_FMT_HYB, SPMV_FMT_SELL, SPMV_FMT_BELL = range(6)
FORMAT_NAMES = ("CSR", "COO", "ELL", "HYB", "SELL", "BELL")
SPMV_NUM_FORMATS = 6
SPMV_F32, SPMV_F64 = 0, 1
KERNEL_NAMES = ("csr_scalar", "csr_vector", "coo", "ell", "hyb", "coo_panel", "coo_sorted", "coo_split",
                "csr_stream", "sell", "bell")
SPMV_SELECT_MODEL, SPMV_SELECT_EXHAUSTIVE, SPMV_SELECT_RULE = 0, 1, 2


class SpmvError(RuntimeError):
    def __init__(self, status: int, where: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        msg = _lib.spmv_last_error().decode(errors="replace")
        super().__init__(f"{where}: {name}: {msg}")
        self.status = name
        self.code = status


class spmv_variant_info(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("block", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("unroll", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("pipelined", ctypes.c_int32), ("ksplit", ctypes.c_int32)]


class spmv_arrays(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("K", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("nnz_tail", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("row", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("ell_col", ctypes.c_void_p),
                ("ell_val", ctypes.c_void_p), ("tail_row", ctypes.c_void_p),
                ("tail_col", ctypes.c_void_p), ("tail_val", ctypes.c_void_p),
                ("sigma", ctypes.c_int32), ("n_slices", ctypes.c_int32), ("block", ctypes.c_int32),
                ("slots", ctypes.c_int64), ("slice_ptr", ctypes.c_void_p), ("perm", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I32, _I64, _D, _F = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float


def _sig(name, res, *args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = list(args)
    return fn


_sig("spmv_create", _I32, ctypes.POINTER(_P), _I32, _I32, _I64, _P, _P, _P, _I32, ctypes.c_int, _P)
_sig("spmv_destroy", None, _P)
_sig("spmv_convert", _I32, _P, _I32, _I32, _P)
_sig("spmv_run", _I32, _P, _I32, _D, _P, _D, _P, _P)
_sig("spmv_get_arrays", _I32, _P, _I32, ctypes.POINTER(spmv_arrays))
_sig("spmv_variant_count", _I32, _I32, _I32)
_sig("spmv_variant_describe", _I32, _I32, _I32, _I32, ctypes.POINTER(spmv_variant_info))
_sig("spmv_set_variant", _I32, _P, _I32, _I32)
_sig("spmv_get_variant", _I32, _P, _I32, ctypes.POINTER(_I32))
_sig("spmv_time", _I32, _P, _I32, _I32, _P, _P, _I32, _I32, ctypes.c_int, _P, _P)


class spmv_energy_result(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("joules", ctypes.c_double),
                ("watts", ctypes.c_double), ("runs", ctypes.c_int64),
                ("ms_per_run", ctypes.c_double), ("joules_per_run", ctypes.c_double),
                ("mflops_per_watt", ctypes.c_double)]


_sig("spmv_energy", _I32, _P, _I32, _I32, _P, _P, ctypes.c_double,
     ctypes.POINTER(spmv_energy_result), _P)
_sig("spmv_idle_power", _I32, ctypes.c_double, ctypes.POINTER(ctypes.c_double))
_sig("spmv_energy_formats", _I32, _P, _I32, _P, _P, _P, _P, ctypes.c_double,
     ctypes.POINTER(spmv_energy_result), _P)
_sig("spmv_tune", _I32, _P, _I32, _P, _P, _I32, ctypes.c_int, ctypes.POINTER(_I32),
     ctypes.POINTER(_F), _P)
_sig("spmv_stored_bytes", _I32, _P, _I32, _I32, ctypes.POINTER(_I64))
_sig("spmv_features", _I32, _P, _P, _P)
_sig("spmv_features_noalloc", _I32, _P, _P, _P)
_sig("spmv_select_format", _I32, _P, _I32, ctypes.POINTER(_I32), _P, _P)


class spmv_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("lr", ctypes.c_float), ("l2", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("classes", ctypes.c_int32)]


SPMV_SELECTOR_PARAMS = 5252
SPMV_SELECTOR_MODEL = 5276
SPMV_SELECTOR_PARAMS6 = 5382
SPMV_SELECTOR_MODEL6 = 5406
_PARAMS_OF = {4: SPMV_SELECTOR_PARAMS, 6: SPMV_SELECTOR_PARAMS6}
_MODEL_OF = {4: SPMV_SELECTOR_MODEL, 6: SPMV_SELECTOR_MODEL6}
_sig("spmv_selector_train", _I32, _P, _P, _I32, _P, _P, ctypes.POINTER(spmv_train_opts), _P, _P, _P)
_sig("spmv_selector_loss_grad", _I32, _P, _I32, _P, _P, _I32, _F, _P, _P, _P)
_sig("spmv_selector_predict", _I32, _P, _I32, _P, _I32, _P, _P, _P, _P)
_sig("spmv_selector_set_weights", _I32, _P, _I64)
_sig("spmv_selector_get_weights", _I32, _P, _I64)
_sig("spmv_selector_classes", _I32)


def _classes_from(numel, table, name):
    for c, n in table.items():
        if int(numel) == n:
            return c
    raise ValueError(f"{name} has {numel} values; expected one of {sorted(table.values())}")
_sig("spmv_status_string", ctypes.c_char_p, _I32)
_sig("spmv_last_error", ctypes.c_char_p)


def _check(st: int, where: str):
    if st != SPMV_OK:
        raise SpmvError(st, where)


def declared_functions() -> list:
    """Names of the functions include/spmv.h declares."""
    with open(HEADER_PATH) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spmv_[a-z0-9_]+)\s*\(", text)))


# ---- marshalling helpers ---------------------------------------------------------------

def _stream_ptr(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(dtype) -> int:
    name = str(dtype)
    if name.endswith("float32"):
        return SPMV_F32
    if name.endswith("float64"):
        return SPMV_F64
    raise ValueError(f"unsupported value dtype {dtype}")


def _buffer(a, want_dtype=None):
    """(pointer, on_device, keepalive) for a torch tensor or NumPy array.

    A tensor must already have `want_dtype` (no silent reinterpretation); a host
    array is converted to it, after a range check for integer targets.
    """
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if want_dtype is not None and str(a.dtype) != "torch." + np.dtype(want_dtype).name:
            raise ValueError(f"tensor dtype {a.dtype} where {np.dtype(want_dtype).name} is required")
        return ctypes.c_void_p(a.data_ptr() if a.numel() else 0), a.is_cuda, a
    if want_dtype is not None:
        src = np.asarray(a)
        wd = np.dtype(want_dtype)
        if wd.kind == "i" and src.size:
            if src.dtype.kind not in "iu":
                raise ValueError(f"integer indices required, got {src.dtype}")
            info = np.iinfo(wd)
            if src.min() < info.min or src.max() > info.max:
                raise ValueError(f"index outside the {wd.name} range")
        arr = np.ascontiguousarray(src, dtype=wd)
    else:
        arr = np.ascontiguousarray(a)
    return ctypes.c_void_p(arr.ctypes.data if arr.size else 0), False, arr


def _check_vector(t, n, h, name):
    """x / y of a run on handle h: a contiguous device tensor on h's device, of h's
    value dtype, with at least n elements (checked before any call into the library)."""
    want = "torch." + np.dtype(h.value_dtype).name
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if str(t.dtype) != want:
        raise ValueError(f"{name} has dtype {t.dtype}, the matrix holds {want}")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, the matrix needs {n}")
    dev = getattr(h, "device", None)
    if dev is not None and t.device.index is not None and t.device.index != dev:
        raise ValueError(f"{name} is on device {t.device.index}, the matrix on device {dev}")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


class Handle:
    """Owns one spmv_handle; destroyed by spmv_destroy (or when collected)."""

    def __init__(self, ptr, n_rows, n_cols, nnz, dtype_code, device=None):
        self.ptr = ptr
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, nnz
        self.dtype_code = dtype_code
        self.device = device  # the HIP device current at spmv_create

    @property
    def value_dtype(self):
        return np.float64 if self.dtype_code == SPMV_F64 else np.float32

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.spmv_destroy(self.ptr)
            self.ptr = None


# ---- the ABI, one wrapper per function ----------------------------------------------

def spmv_create(n_rows, n_cols, row, col, val, stream=None) -> Handle:
    """COO (any order) -> handle with canonical COO/CSR on the device."""
    dt = _dtype_code(val.dtype)
    pr, dr, kr = _buffer(row, np.int32)
    pc, dc, kc = _buffer(col, np.int32)
    pv, dv, kv = _buffer(val)
    if not (dr == dc == dv):
        raise ValueError("row, col and val must all be on the host or all on the device")
    if not (len(kr.shape) == len(kc.shape) == len(kv.shape) == 1):
        raise ValueError("row, col and val must be 1-D")
    nnz = int(kr.shape[0])
    if int(kc.shape[0]) != nnz or int(kv.shape[0]) != nnz:
        raise ValueError("row, col and val must have the same length")
    import torch
    device = torch.cuda.current_device() if torch.cuda.is_available() else None
    if dr and device is not None and kr.device.index not in (None, device):
        raise ValueError("device inputs must be on the current device")
    out = ctypes.c_void_p()
    _check(_lib.spmv_create(ctypes.byref(out), int(n_rows), int(n_cols), nnz, pr, pc, pv, dt,
                            int(dr), _stream_ptr(stream)), "spmv_create")
    return Handle(out, int(n_rows), int(n_cols), nnz, dt, device)


def spmv_destroy(h: Handle):
    if h.ptr:
        _lib.spmv_destroy(h.ptr)
        h.ptr = None


def spmv_convert(h: Handle, fmt: int, param: int = -1, stream=None):
    """Build a format; param: HYB width, SELL sigma, BELL block edge (-1: the rule)."""
    _check(_lib.spmv_convert(h.ptr, int(fmt), int(param), _stream_ptr(stream)), "spmv_convert")


def _device_buffer(a, name):
    p, on_dev, _ = _buffer(a)
    if not on_dev and p.value:
        raise ValueError(f"{name} must be a device tensor")
    return p


def spmv_run(h: Handle, fmt: int, alpha, x, beta, y, stream=None):
    """y = alpha * A x + beta * y on the device (x, y: device tensors)."""
    px = _check_vector(x, h.n_cols, h, "x")
    py = _check_vector(y, h.n_rows, h, "y")
    _check(_lib.spmv_run(h.ptr, int(fmt), float(alpha), px, float(beta), py, _stream_ptr(stream)),
           "spmv_run")


def spmv_get_arrays(h: Handle, fmt: int) -> spmv_arrays:
    v = spmv_arrays()
    _check(_lib.spmv_get_arrays(h.ptr, int(fmt), ctypes.byref(v)), "spmv_get_arrays")
    return v


def spmv_variant_count(fmt: int, dtype_code: int) -> int:
    return int(_lib.spmv_variant_count(int(fmt), int(dtype_code)))


def spmv_variant_describe(fmt: int, dtype_code: int, idx: int) -> dict:
    v = spmv_variant_info()
    _check(_lib.spmv_variant_describe(int(fmt), int(dtype_code), int(idx), ctypes.byref(v)),
           "spmv_variant_describe")
    return {"kernel": KERNEL_NAMES[v.kernel], "block": v.block, "lanes": v.lanes,
            "unroll": v.unroll, "vec": v.vec, "pipelined": v.pipelined, "ksplit": v.ksplit}


def spmv_set_variant(h: Handle, fmt: int, idx: int):
    _check(_lib.spmv_set_variant(h.ptr, int(fmt), int(idx)), "spmv_set_variant")


def spmv_get_variant(h: Handle, fmt: int) -> int:
    out = _I32()
    _check(_lib.spmv_get_variant(h.ptr, int(fmt), ctypes.byref(out)), "spmv_get_variant")
    return int(out.value)


def spmv_time(h: Handle, fmt: int, x, y, variant=-1, warmup=2, reps=10, flush=True,
              stream=None) -> np.ndarray:
    out = np.zeros(max(int(reps), 0), dtype=np.float32)
    px = _check_vector(x, h.n_cols, h, "x")
    py = _check_vector(y, h.n_rows, h, "y")
    _check(_lib.spmv_time(h.ptr, int(fmt), int(variant), px, py, int(warmup), int(reps),
                          int(bool(flush)), ctypes.c_void_p(out.ctypes.data if out.size else 0),
                          _stream_ptr(stream)), "spmv_time")
    return out


def spmv_tune(h: Handle, fmt: int, x, y, reps=10, flush=True, stream=None):
    """Time every variant of fmt, keep the fastest; returns (variant, median ms)."""
    px = _check_vector(x, h.n_cols, h, "x")
    py = _check_vector(y, h.n_rows, h, "y")
    bi, bm = _I32(), _F()
    _check(_lib.spmv_tune(h.ptr, int(fmt), px, py, int(reps), int(bool(flush)), ctypes.byref(bi),
                          ctypes.byref(bm), _stream_ptr(stream)), "spmv_tune")
    return int(bi.value), float(bm.value)


def spmv_energy(h: Handle, fmt: int, x, y, seconds=0.25, variant=-1, stream=None) -> dict:
    """Board energy and average power of fmt's SpMV run back to back (amd-smi counter)."""
    px = _check_vector(x, h.n_cols, h, "x")
    py = _check_vector(y, h.n_rows, h, "y")
    r = spmv_energy_result()
    _check(_lib.spmv_energy(h.ptr, int(fmt), int(variant), px, py, float(seconds), ctypes.byref(r),
                            _stream_ptr(stream)), "spmv_energy")
    return {k: getattr(r, k) for k, _ in spmv_energy_result._fields_}


def spmv_energy_formats(h: Handle, formats, x, y, seconds=0.2, variants=None, stream=None) -> list:
    """spmv_energy of several formats in one sweep (one counter period per format)."""
    px = _check_vector(x, h.n_cols, h, "x")
    py = _check_vector(y, h.n_rows, h, "y")
    f = np.ascontiguousarray(formats, dtype=np.int32)
    v = None if variants is None else np.ascontiguousarray(variants, dtype=np.int32)
    if v is not None and v.shape != f.shape:
        raise ValueError("variants must match formats")
    out = (spmv_energy_result * len(f))()
    _check(_lib.spmv_energy_formats(h.ptr, int(len(f)), ctypes.c_void_p(f.ctypes.data),
                                    ctypes.c_void_p(v.ctypes.data if v is not None else 0), px, py,
                                    float(seconds), out, _stream_ptr(stream)),
           "spmv_energy_formats")
    return [{k: getattr(r, k) for k, _ in spmv_energy_result._fields_} for r in out]


def spmv_idle_power(seconds=0.25) -> float:
    """Average board power between two counter updates with no work of this library."""
    w = ctypes.c_double()
    _check(_lib.spmv_idle_power(float(seconds), ctypes.byref(w)), "spmv_idle_power")
    return float(w.value)


def spmv_stored_bytes(h: Handle, fmt: int, variant: int = -1) -> int:
    """Bytes a run of (fmt, variant) reads besides x and y (its layout, padding included)."""
    out = _I64()
    _check(_lib.spmv_stored_bytes(h.ptr, int(fmt), int(variant), ctypes.byref(out)),
           "spmv_stored_bytes")
    return int(out.value)


def spmv_features(h: Handle, stream=None) -> np.ndarray:
    out = np.zeros(12, dtype=np.float32)
    _check(_lib.spmv_features(h.ptr, ctypes.c_void_p(out.ctypes.data), _stream_ptr(stream)),
           "spmv_features")
    return out


SPMV_FEATURES_NOALLOC_MAX_LEN = 262143  # longest row spmv_features_noalloc accepts


def spmv_features_noalloc(h: Handle, stream=None) -> np.ndarray:
    """spmv_features with its temporaries in the library's fixed device array."""
    out = np.zeros(12, dtype=np.float32)
    _check(_lib.spmv_features_noalloc(h.ptr, ctypes.c_void_p(out.ctypes.data),
                                      _stream_ptr(stream)), "spmv_features_noalloc")
    return out


def spmv_select_format(h: Handle, mode: int, stream=None):
    """(format, scores[SPMV_NUM_FORMATS]) chosen by MODEL / EXHAUSTIVE / RULE."""
    f = _I32()
    scores = np.zeros(SPMV_NUM_FORMATS, dtype=np.float32)
    _check(_lib.spmv_select_format(h.ptr, int(mode), ctypes.byref(f),
                                   ctypes.c_void_p(scores.ctypes.data), _stream_ptr(stream)),
           "spmv_select_format")
    return int(f.value), scores


def _dev_ptr(t, name, allow_none=False):
    if t is None:
        if allow_none:
            return ctypes.c_void_p(0)
        raise ValueError(f"{name} is required")
    p, on_dev, _ = _buffer(t)
    if not on_dev:
        raise ValueError(f"{name} must be a device tensor")
    return p


def spmv_selector_train(feats, labels, init_params, perms, epochs=200, batch=200, lr=1e-3,
                        l2=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, max_steps=0, out_model=None,
                        out_losses=None, stream=None):
    """Train on the device; returns the model tensor (float32[5276] or [5406] on the device).
    The class count (4 or 6) follows the size of init_params."""
    import torch
    n = int(feats.shape[0])
    classes = _classes_from(init_params.numel(), _PARAMS_OF, "init_params")
    if out_model is None:
        out_model = torch.empty(_MODEL_OF[classes], dtype=torch.float32, device=feats.device)
    elif out_model.numel() != _MODEL_OF[classes]:
        raise ValueError(f"out_model must hold {_MODEL_OF[classes]} values")
    o = spmv_train_opts(int(epochs), int(batch), int(max_steps), float(lr), float(l2),
                        float(beta1), float(beta2), float(eps), classes)
    _check(_lib.spmv_selector_train(_dev_ptr(feats, "feats"), _dev_ptr(labels, "labels"), n,
                                     _dev_ptr(init_params, "init_params"), _dev_ptr(perms, "perms"),
                                     ctypes.byref(o), _dev_ptr(out_model, "out_model"),
                                     _dev_ptr(out_losses, "out_losses", True), _stream_ptr(stream)),
           "spmv_selector_train")
    return out_model


def spmv_selector_loss_grad(params, z, labels, l2=1e-4, stream=None):
    """(loss tensor[1], grad tensor[params]) of one minibatch, on the device; the class count
    follows the size of params."""
    import torch
    classes = _classes_from(params.numel(), _PARAMS_OF, "params")
    loss = torch.empty(1, dtype=torch.float32, device=z.device)
    grad = torch.empty(_PARAMS_OF[classes], dtype=torch.float32, device=z.device)
    _check(_lib.spmv_selector_loss_grad(_dev_ptr(params, "params"), classes, _dev_ptr(z, "z"),
                                        _dev_ptr(labels, "labels"), int(z.shape[0]), float(l2),
                                        _dev_ptr(loss, "loss"), _dev_ptr(grad, "grad"),
                                        _stream_ptr(stream)), "spmv_selector_loss_grad")
    return loss, grad


def spmv_selector_predict(model, feats, applicable=None, stream=None):
    """(logits[n][C], cls[n]) device tensors; model None = the weights set on this device."""
    import torch
    n = int(feats.shape[0])
    if model is None:
        classes = int(_lib.spmv_selector_classes())
        if classes == 0:
            raise SpmvError(8, "spmv_selector_predict")
    else:
        classes = _classes_from(model.numel(), _MODEL_OF, "model")
    if applicable is not None and tuple(applicable.shape) != (n, classes):
        raise ValueError(f"applicable must be [{n}][{classes}]")
    logits = torch.empty((n, classes), dtype=torch.float32, device=feats.device)
    cls = torch.empty(n, dtype=torch.int32, device=feats.device)
    _check(_lib.spmv_selector_predict(_dev_ptr(model, "model", True), classes if model is not None else 0,
                                      _dev_ptr(feats, "feats"), n,
                                      _dev_ptr(applicable, "applicable", True),
                                      _dev_ptr(logits, "logits"), _dev_ptr(cls, "cls"),
                                      _stream_ptr(stream)), "spmv_selector_predict")
    return logits, cls


def spmv_selector_set_weights(params):
    """Install a 5276-float (4 classes) or 5406-float (6 classes) model on the current
    device; None forgets it."""
    if params is None:
        _check(_lib.spmv_selector_set_weights(ctypes.c_void_p(0), 0), "spmv_selector_set_weights")
        return
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.spmv_selector_set_weights(ctypes.c_void_p(a.ctypes.data), a.size),
           "spmv_selector_set_weights")


def spmv_selector_classes() -> int:
    """Classes of the network installed on the current device (0: none)."""
    return int(_lib.spmv_selector_classes())


def spmv_selector_get_weights() -> np.ndarray:
    classes = spmv_selector_classes()
    out = np.zeros(_MODEL_OF.get(classes, SPMV_SELECTOR_MODEL), dtype=np.float32)
    _check(_lib.spmv_selector_get_weights(ctypes.c_void_p(out.ctypes.data), out.size),
           "spmv_selector_get_weights")
    return out


SPMV_RUNTIME_MODEL = 96


class spmv_runtime_decision(ctypes.Structure):
    _fields_ = [("current", ctypes.c_int32), ("predicted", ctypes.c_int32),
                ("chosen", ctypes.c_int32), ("converted", ctypes.c_int32),
                ("features_ms", ctypes.c_float), ("predict_ms", ctypes.c_float),
                ("convert_ms", ctypes.c_float), ("t_current_ms", ctypes.c_float),
                ("t_predicted_ms", ctypes.c_float), ("gain_ms", ctypes.c_double),
                ("overhead_ms", ctypes.c_double)]


_sig("spmv_runtime_set_model", _I32, _P, _I64)
_sig("spmv_select_runtime", _I32, _P, _I32, _I64, ctypes.POINTER(spmv_runtime_decision), _P)


def spmv_runtime_set_model(params):
    """Install the 96-float run-time model on the current device; None forgets it."""
    if params is None:
        _check(_lib.spmv_runtime_set_model(ctypes.c_void_p(0), 0), "spmv_runtime_set_model")
        return
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.spmv_runtime_set_model(ctypes.c_void_p(a.ctypes.data), a.size),
           "spmv_runtime_set_model")


def spmv_select_runtime(h: Handle, current: int, iterations: int, stream=None) -> dict:
    """Overhead-aware run-time mode: the decision as a dict (fields of spmv_runtime_decision)."""
    d = spmv_runtime_decision()
    _check(_lib.spmv_select_runtime(h.ptr, int(current), int(iterations), ctypes.byref(d),
                                    _stream_ptr(stream)), "spmv_select_runtime")
    return {f: getattr(d, f) for f, _ in d._fields_}


class spmv_batch_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("passes_per_tile", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lanes_divisor", ctypes.c_int32), ("tiling", ctypes.c_int32),
                ("total_tiles", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("tuned_ms", ctypes.c_float)]


_sig("spmv_batch_create", _I32, ctypes.POINTER(_P), _P, _I32, _P, _P, _P, _P, ctypes.c_int, _P)
_sig("spmv_batch_run", _I32, _P, _P, _P, _P, _P, _P)
_sig("spmv_batch_update", _I32, _P, _P, _P, _P, _P, _P)
_sig("spmv_batch_get_config", _I32, _P, ctypes.POINTER(spmv_batch_config), _P)
_sig("spmv_batch_set_config", _I32, _P, ctypes.POINTER(spmv_batch_config), _P)
_sig("spmv_batch_destroy", None, _P)


class Batch:
    """Owns one spmv_batch (and keeps its handles and vectors alive)."""

    def __init__(self, ptr, handles, xs, ys):
        self.ptr, self.handles, self.xs, self.ys = ptr, list(handles), list(xs), list(ys)

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.spmv_batch_destroy(self.ptr)
            self.ptr = None


def _ptr_array(items, name, handles=None, dim=None):
    """Host array of device pointers; with handles, each tensor is checked against
    its matrix (dtype, device, at least getattr(handle, dim) elements)."""
    if handles is not None and len(items) != len(handles):
        raise ValueError(f"{name} must have {len(handles)} entries")
    arr = (ctypes.c_void_p * len(items))()
    for i, t in enumerate(items):
        if handles is not None:
            arr[i] = _check_vector(t, getattr(handles[i], dim), handles[i], f"{name}[{i}]").value
        else:
            arr[i] = _dev_ptr(t, f"{name}[{i}]").value
    return arr


def spmv_batch_create(handles, xs, ys, alphas=None, betas=None, tune=True, stream=None) -> Batch:
    n = len(handles)
    for name, arr in (("alphas", alphas), ("betas", betas)):
        if arr is not None and len(arr) != n:
            raise ValueError(f"{name} must have {n} entries")
    hs = (ctypes.c_void_p * n)(*[h.ptr.value if isinstance(h.ptr, ctypes.c_void_p) else h.ptr
                                 for h in handles])
    pa = (ctypes.c_double * n)(*alphas) if alphas is not None else None
    pb = (ctypes.c_double * n)(*betas) if betas is not None else None
    out = ctypes.c_void_p()
    _check(_lib.spmv_batch_create(ctypes.byref(out), ctypes.cast(hs, ctypes.c_void_p), n,
                                  ctypes.cast(_ptr_array(xs, "xs", handles, "n_cols"), ctypes.c_void_p),
                                  ctypes.cast(_ptr_array(ys, "ys", handles, "n_rows"), ctypes.c_void_p),
                                  ctypes.cast(pa, ctypes.c_void_p) if pa is not None else None,
                                  ctypes.cast(pb, ctypes.c_void_p) if pb is not None else None,
                                  int(bool(tune)), _stream_ptr(stream)), "spmv_batch_create")
    return Batch(out, handles, xs, ys)


def spmv_batch_run(b: Batch, alphas=None, xs=None, betas=None, ys=None, stream=None):
    """One graph launch of the batch; given alphas/xs/betas/ys replace the held ones."""
    n = len(b.handles)
    for name, arr in (("alphas", alphas), ("betas", betas)):
        if arr is not None and len(arr) != n:
            raise ValueError(f"{name} must have {n} entries")
    pa = ctypes.cast((ctypes.c_double * n)(*alphas), ctypes.c_void_p) if alphas is not None else None
    px = ctypes.cast(_ptr_array(xs, "xs", b.handles, "n_cols"), ctypes.c_void_p) if xs is not None else None
    pb = ctypes.cast((ctypes.c_double * n)(*betas), ctypes.c_void_p) if betas is not None else None
    py = ctypes.cast(_ptr_array(ys, "ys", b.handles, "n_rows"), ctypes.c_void_p) if ys is not None else None
    _check(_lib.spmv_batch_run(b.ptr, pa, px, pb, py, _stream_ptr(stream)), "spmv_batch_run")
    if xs is not None:
        b.xs = list(xs)
    if ys is not None:
        b.ys = list(ys)


def spmv_batch_update(b: Batch, xs=None, ys=None, alphas=None, betas=None, stream=None):
    n = len(b.handles)
    for name, arr in (("alphas", alphas), ("betas", betas)):
        if arr is not None and len(arr) != n:
            raise ValueError(f"{name} must have {n} entries")
    px = ctypes.cast(_ptr_array(xs, "xs", b.handles, "n_cols"), ctypes.c_void_p) if xs is not None else None
    py = ctypes.cast(_ptr_array(ys, "ys", b.handles, "n_rows"), ctypes.c_void_p) if ys is not None else None
    pa = ctypes.cast((ctypes.c_double * n)(*alphas), ctypes.c_void_p) if alphas is not None else None
    pb = ctypes.cast((ctypes.c_double * n)(*betas), ctypes.c_void_p) if betas is not None else None
    _check(_lib.spmv_batch_update(b.ptr, px, py, pa, pb, _stream_ptr(stream)), "spmv_batch_update")
    if xs is not None:
        b.xs = list(xs)
    if ys is not None:
        b.ys = list(ys)


def spmv_batch_get_config(b: Batch):
    c = spmv_batch_config()
    lanes = np.zeros(len(b.handles), dtype=np.int32)
    _check(_lib.spmv_batch_get_config(b.ptr, ctypes.byref(c), ctypes.c_void_p(lanes.ctypes.data)),
           "spmv_batch_get_config")
    return {f: getattr(c, f) for f, _ in c._fields_}, lanes


def spmv_batch_set_config(b: Batch, stream=None, **setting):
    """Rebuild the batch's graph with the given setting (keys of spmv_batch_config)."""
    cur, _ = spmv_batch_get_config(b)
    cur.update(setting)
    c = spmv_batch_config(**{f: cur[f] for f, _ in spmv_batch_config._fields_})
    _check(_lib.spmv_batch_set_config(b.ptr, ctypes.byref(c), _stream_ptr(stream)),
           "spmv_batch_set_config")


def spmv_batch_destroy(b: Batch):
    if b.ptr:
        _lib.spmv_batch_destroy(b.ptr)
        b.ptr = None


def spmv_status_string(status: int) -> str:
    return _lib.spmv_status_string(int(status)).decode()


def spmv_last_error() -> str:
    return _lib.spmv_last_error().decode(errors="replace")


# ---- device-array views -------------------------------------------------------------------

class _DeviceView:
    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr,
                                         "data": (int(ptr or 0), False), "version": 2}


def device_tensor(ptr, n, np_dtype):
    """A torch tensor aliasing n elements of library-owned device memory (borrowed)."""
    import torch
    if n == 0 or not ptr:
        return torch.zeros(0, dtype=torch.from_numpy(np.zeros(0, np_dtype)).dtype, device="cuda")
    return torch.as_tensor(_DeviceView(ptr, n, np.dtype(np_dtype).str), device="cuda")


def arrays_to_host(h: Handle, fmt: int) -> dict:
    """Copy every device array of a format to NumPy (for checks)."""
    v = spmv_get_arrays(h, fmt)
    vd = h.value_dtype
    out = {"K": v.K, "pitch": v.pitch, "nnz_tail": v.nnz_tail}
    if fmt == SPMV_FMT_CSR:
        out["row_ptr"] = device_tensor(v.row_ptr, h.n_rows + 1, np.int32).cpu().numpy()
        out["col"] = device_tensor(v.col, h.nnz, np.int32).cpu().numpy()
        out["val"] = device_tensor(v.val, h.nnz, vd).cpu().numpy()
    elif fmt == SPMV_FMT_COO:
        out["row"] = device_tensor(v.row, h.nnz, np.int32).cpu().numpy()
        out["col"] = device_tensor(v.col, h.nnz, np.int32).cpu().numpy()
        out["val"] = device_tensor(v.val, h.nnz, vd).cpu().numpy()
    elif fmt == SPMV_FMT_SELL:
        out.update(sigma=v.sigma, n_slices=v.n_slices, slots=v.slots)
        out["slice_ptr"] = device_tensor(v.slice_ptr, v.n_slices + 1, np.int64).cpu().numpy()
        out["perm"] = (device_tensor(v.perm, h.n_rows, np.int32).cpu().numpy() if v.perm
                       else np.arange(h.n_rows, dtype=np.int32))
        out["col"] = device_tensor(v.ell_col, v.slots, np.int32).cpu().numpy()
        out["val"] = device_tensor(v.ell_val, v.slots, vd).cpu().numpy()
    elif fmt == SPMV_FMT_BELL:
        out.update(b=v.block)
        out["bcol"] = device_tensor(v.ell_col, v.slots, np.int32).cpu().numpy()
        out["bval"] = device_tensor(v.ell_val, v.slots * v.block * v.block, vd).cpu().numpy()
    else:
        n = v.K * v.pitch
        out["ell_col"] = device_tensor(v.ell_col, n, np.int32).cpu().numpy()
        out["ell_val"] = device_tensor(v.ell_val, n, vd).cpu().numpy()
        if fmt == SPMV_FMT_HYB:
            t = v.nnz_tail
            out["tail_row"] = device_tensor(v.tail_row, t, np.int32).cpu().numpy()
            out["tail_col"] = device_tensor(v.tail_col, t, np.int32).cpu().numpy()
            out["tail_val"] = device_tensor(v.tail_val, t, vd).cpu().numpy()
    return out
