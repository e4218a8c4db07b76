"""ctypes access to the plain-C oracle (oracle.c).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and never calls it.

Masks are numpy uint8 arrays of 0/1, shape (H, W).  Images are numpy arrays
of shape (C, H, W) (or (H, W) for one channel), dtype float32, uint8 or
uint16.
"""
import ctypes
import os

import numpy as np

from .build import LIB_PATH, build

CMP = {">": 0, "<": 1, ">=": 2, "<=": 3}
_DT = {np.dtype(np.float32): 0, np.dtype(np.uint8): 1, np.dtype(np.uint16): 2}
_lib = None


class OracleError(RuntimeError):
    pass


def _load(path=None):
    # ORACLE_LIB selects another build of oracle.c (used by the mutation test)
    path = path or os.environ.get("ORACLE_LIB") or LIB_PATH
    if not os.path.exists(path):
        build(path)
    L = ctypes.CDLL(path)
    P, I, I64, D, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    L.oracle_run.argtypes = [ctypes.c_char_p, P, I, I, I, I, P, I, ctypes.c_char_p, I]
    L.oracle_run3.argtypes = [ctypes.c_char_p, P, I, I, I, I, I, P, I, ctypes.c_char_p, I]
    L.oracle_near3.argtypes = [P, I, I, I, P]
    L.oracle_reach3.argtypes = [P, P, I, I, I, P]
    L.oracle_ccl3.argtypes = [P, I, I, I, P]
    L.oracle_count_outputs.argtypes = [ctypes.c_char_p, ctypes.c_char_p, I]
    L.oracle_not.argtypes = [P, I64, P]
    L.oracle_and.argtypes = [P, P, I64, P]
    L.oracle_or.argtypes = [P, P, I64, P]
    L.oracle_near.argtypes = [P, I, I, P]
    for fn in (L.oracle_reach, L.oracle_surrounded, L.oracle_grow):
        fn.argtypes = [P, P, I, I, P]
    L.oracle_interior.argtypes = [P, I, I, P]
    L.oracle_ccl.argtypes = [P, I, I, P]
    L.oracle_ccl_max.argtypes = [P, I, I, P]
    L.oracle_ccl_pj.argtypes = [P, I, I, I, I, P, ctypes.POINTER(I64)]
    L.oracle_percentile.argtypes = [P, I, I, I, I, I, D, ctypes.POINTER(F)]
    L.oracle_threshold.argtypes = [P, I, I, I, I, I, I, F, P]
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _img3(img):
    img = np.ascontiguousarray(img)
    if img.ndim == 2:
        img = img[None]
    if img.ndim != 3 or img.dtype not in _DT:
        raise ValueError("image must be (C,H,W) float32, uint8 or uint16")
    return img


def _mask(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError("mask must be 2-D")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def count_outputs(src):
    err = ctypes.create_string_buffer(512)
    n = lib().oracle_count_outputs(src.encode(), err, 512)
    if n < 0:
        raise OracleError(err.value.decode())
    return n


def run(src, img):
    """Evaluate every `output` of the formula text `src` on `img`."""
    img = _img3(img)
    C, H, W = img.shape
    nout = count_outputs(src)
    out = np.zeros((max(nout, 1), H, W), np.uint8)
    err = ctypes.create_string_buffer(512)
    rc = lib().oracle_run(src.encode(), _ptr(img), _DT[img.dtype], C, H, W, _ptr(out), nout,
                          err, 512)
    if rc < 0:
        raise OracleError(f"oracle error {rc}: {err.value.decode()}")
    return [out[i] for i in range(nout)]


def run3(src, vol):
    """Evaluate every `output` of `src` on a volume (C, D, H, W) or (D, H, W):
    26-neighbourhood N and 26-connected paths."""
    vol = np.ascontiguousarray(vol)
    if vol.ndim == 3:
        vol = vol[None]
    if vol.ndim != 4 or vol.dtype not in _DT:
        raise ValueError("volume must be (C,D,H,W) float32, uint8 or uint16")
    C, D, H, W = vol.shape
    nout = count_outputs(src)
    out = np.zeros((max(nout, 1), D, H, W), np.uint8)
    err = ctypes.create_string_buffer(512)
    rc = lib().oracle_run3(src.encode(), _ptr(vol), _DT[vol.dtype], C, D, H, W, _ptr(out), nout, err, 512)
    if rc < 0:
        raise OracleError(f"oracle error {rc}: {err.value.decode()}")
    return [out[i] for i in range(nout)]


def _vol(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.ndim != 3:
        raise ValueError("volume mask must be 3-D")
    return a


def near3(a):
    a = _vol(a)
    out = np.zeros_like(a)
    lib().oracle_near3(_ptr(a), *a.shape, _ptr(out))
    return out


def reach3(a, b):
    a, b = _vol(a), _vol(b)
    out = np.zeros_like(a)
    rc = lib().oracle_reach3(_ptr(a), _ptr(b), *a.shape, _ptr(out))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return out


def ccl3(a):
    """26-connected labels; label = smallest linear index in the component, -1 = background."""
    a = _vol(a)
    lab = np.zeros(a.shape, np.int32)
    rc = lib().oracle_ccl3(_ptr(a), *a.shape, _ptr(lab))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return lab


def _unary(fn, a):
    a = _mask(a)
    out = np.zeros_like(a)
    rc = fn(_ptr(a), a.shape[0], a.shape[1], _ptr(out))
    if rc is not None and rc < 0:
        raise OracleError(f"oracle error {rc}")
    return out


def _binary(fn, a, b):
    a, b = _mask(a), _mask(b)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    out = np.zeros_like(a)
    rc = fn(_ptr(a), _ptr(b), a.shape[0], a.shape[1], _ptr(out))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return out


def near(a):
    return _unary(lib().oracle_near, a)


def interior(a):
    return _unary(lib().oracle_interior, a)


def reach(a, b):
    return _binary(lib().oracle_reach, a, b)


def surrounded(a, b):
    return _binary(lib().oracle_surrounded, a, b)


def grow(a, b):
    return _binary(lib().oracle_grow, a, b)


def lnot(a):
    a = _mask(a)
    out = np.zeros_like(a)
    lib().oracle_not(_ptr(a), a.size, _ptr(out))
    return out


def land(a, b):
    a, b = _mask(a), _mask(b)
    out = np.zeros_like(a)
    lib().oracle_and(_ptr(a), _ptr(b), a.size, _ptr(out))
    return out


def lor(a, b):
    a, b = _mask(a), _mask(b)
    out = np.zeros_like(a)
    lib().oracle_or(_ptr(a), _ptr(b), a.size, _ptr(out))
    return out


def ccl(a):
    """8-connected labels; label = smallest row-major index in the component, -1 = background."""
    a = _mask(a)
    lab = np.zeros(a.shape, np.int32)
    rc = lib().oracle_ccl(_ptr(a), a.shape[0], a.shape[1], _ptr(lab))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return lab


def ccl_max(a):
    """8-connected labels of the paper's labelling once terminated: label =
    largest row-major index in the component, -1 = background."""
    a = _mask(a)
    lab = np.zeros(a.shape, np.int32)
    rc = lib().oracle_ccl_max(_ptr(a), a.shape[0], a.shape[1], _ptr(lab))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return lab


def ccl_pj(a, k=16, max_rounds=100000):
    """The paper's labelling algorithm (Alg. CCL) run step by step: returns
    (labels as in ccl_max, number of main iterations).  Raises OracleError
    when the termination check still fails after max_rounds rounds."""
    a = _mask(a)
    lab = np.zeros(a.shape, np.int32)
    it = ctypes.c_int64()
    rc = lib().oracle_ccl_pj(_ptr(a), a.shape[0], a.shape[1], k, max_rounds, _ptr(lab), ctypes.byref(it))
    if rc < 0:
        raise OracleError(f"oracle error {rc} after {it.value} main iterations")
    return lab, it.value


def percentile(img, c, q):
    img = _img3(img)
    C, H, W = img.shape
    r = ctypes.c_float()
    rc = lib().oracle_percentile(_ptr(img), _DT[img.dtype], C, H, W, c, q, ctypes.byref(r))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return np.float32(r.value)


def threshold(img, c, op, t):
    img = _img3(img)
    C, H, W = img.shape
    out = np.zeros((H, W), np.uint8)
    rc = lib().oracle_threshold(_ptr(img), _DT[img.dtype], C, H, W, c, CMP[op], float(t),
                                _ptr(out))
    if rc < 0:
        raise OracleError(f"oracle error {rc}")
    return out
