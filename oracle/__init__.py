"""CPU oracle for the Canny edge detector -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here; the two
share no code.

This is a thin ctypes wrapper around ``canny_oracle.c`` (plain C, fp64 for all
floating point), plus ``build()`` which compiles it with gcc.  Every function
cites the step of the paper (Section 2.2.1, Steps 1-4) it follows; the C file
carries the definitions.

``paper_design_canny_f32`` wraps ``paper_design.c``: the same float operator
in the paper's parallel design (row-parallel Steps 1-3, serial hysteresis,
OpenMP), a measured CPU baseline for the benchmark, not an oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "canny_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_PD_SRC = os.path.join(_HERE, "paper_design.c")
_PD_LIB = os.path.join(_HERE, "libpaper_design.so")
_lib = None
_pd_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single-threaded, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_PD_LIB):
        tmp = _PD_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, _PD_SRC, _SRC, "-lm"])
        os.replace(tmp, _PD_LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    i, d, l = C.c_int, C.c_double, C.c_long
    sig = {
        "oracle_blur_binomial": (None, [P, i, i, P]),
        "oracle_sobel_i32": (None, [P, i, i, P, P]),
        "oracle_sector": (i, [i, i]),
        "oracle_sector_array": (None, [P, P, l, P]),
        "oracle_classify_u8": (None, [P, i, i, i, i, P, P, P]),
        "oracle_hysteresis": (l, [P, i, i, P]),
        "oracle_canny_u8": (None, [P, i, i, i, i, P, P]),
        "oracle_gauss_weights": (None, [d, i, P]),
        "oracle_gauss_weights_dsigma": (None, [d, i, P]),
        "oracle_gauss_blur": (None, [P, i, i, d, i, P]),
        "oracle_sobel_f64": (None, [P, i, i, P, P]),
        "oracle_classify_f32": (l, [P, i, i, d, i, d, d, i, d, P, P, P, P]),
        "oracle_sector_f64": (i, [d, d]),
        "oracle_classify_f32_sector": (l, [P, i, i, d, i, d, d, i, d, P, P, P, P]),
        "oracle_mag_forward": (None, [P, i, i, d, i, P]),
        "oracle_mag_backward": (None, [P, i, i, d, i, P, P, P]),
        "oracle_laplace_i32": (None, [P, i, i, P]),
        "oracle_zero_crossings": (l, [P, i, i, i, P]),
        "oracle_log_u8": (l, [P, i, i, i, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- integer path (Steps 1-4) -------------------------------------------

def blur_binomial(img):
    img = _u8(img)
    H, W = img.shape
    out = np.empty_like(img)
    _load().oracle_blur_binomial(_p(img), H, W, _p(out))
    return out


def sobel_i32(B):
    B = _u8(B)
    H, W = B.shape
    gx = np.empty((H, W), np.int32)
    gy = np.empty((H, W), np.int32)
    _load().oracle_sobel_i32(_p(B), H, W, _p(gx), _p(gy))
    return gx, gy


def sector(gx, gy):
    gx = np.ascontiguousarray(gx, dtype=np.int32)
    gy = np.ascontiguousarray(gy, dtype=np.int32)
    out = np.empty(gx.shape, np.uint8)
    _load().oracle_sector_array(_p(gx), _p(gy), gx.size, _p(out))
    return out


def classify_u8(img, low, high):
    """Returns (class map uint8, magnitude int32, sector uint8)."""
    img = _u8(img)
    H, W = img.shape
    cls = np.empty((H, W), np.uint8)
    M = np.empty((H, W), np.int32)
    sec = np.empty((H, W), np.uint8)
    _load().oracle_classify_u8(_p(img), H, W, int(low), int(high), _p(cls), _p(M), _p(sec))
    return cls, M, sec


def hysteresis(cls):
    """Returns (edges uint8 {0,255}, deepest BFS level)."""
    cls = _u8(cls)
    H, W = cls.shape
    edges = np.empty((H, W), np.uint8)
    depth = _load().oracle_hysteresis(_p(cls), H, W, _p(edges))
    return edges, int(depth)


def canny_u8(img, low, high):
    """Returns (edges, class map)."""
    img = _u8(img)
    H, W = img.shape
    edges = np.empty((H, W), np.uint8)
    cls = np.empty((H, W), np.uint8)
    _load().oracle_canny_u8(_p(img), H, W, int(low), int(high), _p(edges), _p(cls))
    return edges, cls


# ---- floating-point path (fp64) -----------------------------------------

def gauss_weights(sigma, R):
    g = np.empty(2 * R + 1, np.float64)
    _load().oracle_gauss_weights(float(sigma), int(R), _p(g))
    return g


def gauss_weights_dsigma(sigma, R):
    g = np.empty(2 * R + 1, np.float64)
    _load().oracle_gauss_weights_dsigma(float(sigma), int(R), _p(g))
    return g


def gauss_blur(X, sigma, R):
    X = _f64(X)
    H, W = X.shape
    out = np.empty_like(X)
    _load().oracle_gauss_blur(_p(X), H, W, float(sigma), int(R), _p(out))
    return out


def sobel_f64(B):
    B = _f64(B)
    H, W = B.shape
    gx = np.empty_like(B)
    gy = np.empty_like(B)
    _load().oracle_sobel_f64(_p(B), H, W, _p(gx), _p(gy))
    return gx, gy


def classify_f32(X, sigma=1.4, R=3, low=0.05, high=0.15, relative=True, tol=1e-5):
    """Returns (class map, M fp64, ambiguity bit flags, max M)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    H, W = X.shape
    cls = np.empty((H, W), np.uint8)
    M = np.empty((H, W), np.float64)
    amb = np.empty((H, W), np.uint8)
    mx = C.c_double(0.0)
    _load().oracle_classify_f32(_p(X), H, W, float(sigma), int(R), float(low), float(high),
                                int(bool(relative)), float(tol), _p(cls), _p(M), _p(amb),
                                C.byref(mx))
    return cls, M, amb, mx.value


def sector_f64(gx, gy):
    """Four-sector code of a float gradient (Section 2.2.1, Step 2 direction)."""
    return _load().oracle_sector_f64(float(gx), float(gy))


def classify_f32_sector(X, sigma=1.4, R=3, low=20.0, high=60.0, relative=False, tol=1e-5):
    """Float path with the four-sector direction (Step 3 against p -/+ d).
    Returns (class map, M fp64, ambiguity bit flags (bits 0, 1, 3), max M)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    H, W = X.shape
    cls = np.empty((H, W), np.uint8)
    M = np.empty((H, W), np.float64)
    amb = np.empty((H, W), np.uint8)
    mx = C.c_double(0.0)
    _load().oracle_classify_f32_sector(_p(X), H, W, float(sigma), int(R), float(low), float(high),
                                       int(bool(relative)), float(tol), _p(cls), _p(M), _p(amb),
                                       C.byref(mx))
    return cls, M, amb, mx.value


def canny_f32(X, sigma=1.4, R=3, low=0.05, high=0.15, relative=True):
    cls, _, _, _ = classify_f32(X, sigma, R, low, high, relative)
    edges, _ = hysteresis(cls)
    return edges, cls


# ---- differentiable front end (fp64) ------------------------------------

def mag_forward(I, sigma, R=9):
    I = _f64(I)
    H, W = I.shape
    M = np.empty_like(I)
    _load().oracle_mag_forward(_p(I), H, W, float(sigma), int(R), _p(M))
    return M


def mag_backward(I, sigma, gM, R=9):
    """Returns (dL/dI, dL/dsigma) for one image."""
    I = _f64(I)
    gM = _f64(gM)
    H, W = I.shape
    dI = np.empty_like(I)
    ds = C.c_double(0.0)
    _load().oracle_mag_backward(_p(I), H, W, float(sigma), int(R), _p(gM), _p(dI), C.byref(ds))
    return dI, ds.value


# ---- the paper's parallel design on the CPU (baseline, not an oracle) ------

# ---- Laplacian zero-crossing detector (the introduction's Laplace operator) ----

def laplace_i32(B):
    """L = B(x-1) + B(x+1) + B(y-1) + B(y+1) - 4 B with replicate borders."""
    B = _u8(B)
    H, W = B.shape
    L = np.empty((H, W), np.int32)
    _load().oracle_laplace_i32(_p(B), H, W, _p(L))
    return L


def zero_crossings(L, t):
    """Edges (255 / 0) at the zero crossings of L: between 4-neighbours of
    strictly opposite signs with |L(p) - L(q)| >= t (marked on the pixel of
    the pair nearer the zero, the earlier one on a tie), and at zeros whose
    opposite neighbours (left/right or up/down) have strictly opposite signs
    with a difference >= t."""
    L = np.ascontiguousarray(L, dtype=np.int32)
    H, W = L.shape
    e = np.empty((H, W), np.uint8)
    _load().oracle_zero_crossings(_p(L), H, W, int(t), _p(e))
    return e


def log_u8(img, t):
    """The whole detector on a uint8 image: binomial blur (Step 1 of the
    integer path), Laplacian, zero crossings.  Returns (edges, L)."""
    img = _u8(img)
    H, W = img.shape
    e = np.empty((H, W), np.uint8)
    L = np.empty((H, W), np.int32)
    _load().oracle_log_u8(_p(img), H, W, int(t), _p(e), _p(L))
    return e, L


def _load_pd():
    global _pd_lib
    if _pd_lib is not None:
        return _pd_lib
    if (not os.path.exists(_PD_LIB) or os.path.getmtime(_PD_LIB) < os.path.getmtime(_PD_SRC)
            or os.path.getmtime(_PD_LIB) < os.path.getmtime(_SRC)):
        build()
    lib = C.CDLL(_PD_LIB)
    lib.pd_canny_f32.restype = C.c_int
    lib.pd_canny_f32.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                 C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    _pd_lib = lib
    return lib


def paper_design_canny_f32(X, nthreads, sigma=1.4, R=3, low=0.05, high=0.15, relative=True):
    """Float Canny with row-parallel Steps 1-3 on ``nthreads`` threads and
    serial hysteresis.  Returns (edges, seconds parallel part, seconds serial part)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    H, W = X.shape
    edges = np.empty((H, W), np.uint8)
    tp, ts = C.c_double(0.0), C.c_double(0.0)
    rc = _load_pd().pd_canny_f32(_p(X), H, W, float(sigma), int(R), float(low), float(high),
                                 int(bool(relative)), int(nthreads), _p(edges), C.byref(tp),
                                 C.byref(ts))
    if rc != 0:
        raise MemoryError("paper-design baseline: allocation failed")
    return edges, tp.value, ts.value
