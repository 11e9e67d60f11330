"""FP64 CPU oracle for the shiftable bilateral filter (ctypes binding).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library neither imports
nor links anything here, and nothing here imports the product package.

The C source (``bsk_oracle.c``) evaluates eq. (3) of the paper directly with a
box spatial window and the rescaled raised-cosine range kernel of eq. (6),
cos^N(t / (sigma_r sqrt N)); the ``*_sp`` entry points add the separable
raised-cosine spatial kernel of Algorithms 1 and 2 with M > 1, and the
``*_poly`` entry points use the polynomial range kernel p_N of Section 3 in the
scaling of eq. (5), (1 - t^2 / (2 N sigma_r^2))^N; the ``nlm2`` entry points
compute the two-pixel-patch non-local means of Section 5.  See its header
for the definitions.  This module only marshals NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsk_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_llp = ctypes.POINTER(ctypes.c_longlong)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.oracle_order_for.restype = ctypes.c_int
    lib.oracle_order_for.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_kernel.restype = ctypes.c_double
    lib.oracle_kernel.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_kernel_deriv.restype = ctypes.c_double
    lib.oracle_kernel_deriv.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_trunc_terms.restype = ctypes.c_int
    lib.oracle_trunc_terms.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
    lib.oracle_trunc_kernel.restype = ctypes.c_double
    lib.oracle_trunc_kernel.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double]
    lib.oracle_bilateral_f64.restype = None
    lib.oracle_bilateral_f64.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_bilateral.restype = None
    lib.oracle_bilateral.argtypes = [_fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_bilateral_at.restype = None
    lib.oracle_bilateral_at.argtypes = [_fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_int, _llp, ctypes.c_longlong,
                                        _dp, _dp, _dp]
    lib.oracle_bilateral_grad_f64.restype = None
    lib.oracle_bilateral_grad_f64.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_spatial_weight.restype = ctypes.c_double
    lib.oracle_spatial_weight.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_bilateral_sp_f64.restype = None
    lib.oracle_bilateral_sp_f64.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_bilateral_sp.restype = None
    lib.oracle_bilateral_sp.argtypes = [_fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_bilateral_sp_at.restype = None
    lib.oracle_bilateral_sp_at.argtypes = [_fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_int, _llp, ctypes.c_longlong,
                                           _dp, _dp, _dp]
    lib.oracle_poly_order_for.restype = ctypes.c_int
    lib.oracle_poly_order_for.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_poly_kernel.restype = ctypes.c_double
    lib.oracle_poly_kernel.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_bilateral_poly_f64.restype = None
    lib.oracle_bilateral_poly_f64.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_bilateral_poly.restype = None
    lib.oracle_bilateral_poly.argtypes = [_fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_bilateral_poly_at.restype = None
    lib.oracle_bilateral_poly_at.argtypes = [_fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_int, _llp, ctypes.c_longlong, _dp]
    _ci = ctypes.c_int
    _cd = ctypes.c_double
    lib.oracle_nlm2_f64.restype = None
    lib.oracle_nlm2_f64.argtypes = [_dp, _ci, _ci, _ci, _cd, _ci, _cd, _ci, _ci, _ci, _dp, _dp, _dp]
    lib.oracle_nlm2.restype = None
    lib.oracle_nlm2.argtypes = [_fp, _ci, _ci, _ci, _cd, _ci, _cd, _ci, _ci, _ci, _dp, _dp, _dp]
    lib.oracle_nlm2_at.restype = None
    lib.oracle_nlm2_at.argtypes = [_fp, _ci, _ci, _ci, _cd, _ci, _cd, _ci, _ci, _ci, _llp, ctypes.c_longlong, _dp]
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def order_for(sigma_r: float, T: float) -> int:
    """N_0: the smallest order keeping the kernel non-negative and unimodal on [-T, T]."""
    return _load().oracle_order_for(float(sigma_r), float(T))


def kernel(t: float, sigma_r: float, N: int) -> float:
    return _load().oracle_kernel(float(t), float(sigma_r), int(N))


def kernel_deriv(t: float, sigma_r: float, N: int) -> float:
    return _load().oracle_kernel_deriv(float(t), float(sigma_r), int(N))


def trunc_terms(N: int, eps: float):
    """(number of kept terms, dropped weight mass) for truncation threshold eps."""
    d = ctypes.c_double(0.0)
    kept = _load().oracle_trunc_terms(int(N), float(eps), ctypes.byref(d))
    return kept, d.value


def trunc_kernel(t: float, sigma_r: float, N: int, eps: float) -> float:
    return _load().oracle_trunc_kernel(float(t), float(sigma_r), int(N), float(eps))


def num_threads() -> int:
    return _load().oracle_num_threads()


def bilateral(f, radius: int, sigma_r: float, N: int, eps: float = 0.0, truncated: bool = False,
              return_pq: bool = False):
    """Whole-image filter.  float32 input is widened exactly; float64 input is used as is."""
    f = np.ascontiguousarray(f)
    H, W = f.shape
    out = np.empty((H, W), np.float64)
    P = np.empty((H, W), np.float64) if return_pq else None
    Q = np.empty((H, W), np.float64) if return_pq else None
    lib = _load()
    if f.dtype == np.float64:
        lib.oracle_bilateral_f64(_ptr(f, _dp), H, W, int(radius), float(sigma_r), int(N), float(eps),
                                 int(bool(truncated)), _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    else:
        f = np.ascontiguousarray(f, dtype=np.float32)
        lib.oracle_bilateral(_ptr(f, _fp), H, W, int(radius), float(sigma_r), int(N), float(eps),
                             int(bool(truncated)), _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    return (out, P, Q) if return_pq else out


def bilateral_at(f, idx, radius: int, sigma_r: float, N: int, eps: float = 0.0, truncated: bool = False,
                 return_pq: bool = False):
    """Filter output at the flat (row-major) pixel indices ``idx`` only."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    H, W = f.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = idx.size
    out = np.empty(n, np.float64)
    P = np.empty(n, np.float64) if return_pq else None
    Q = np.empty(n, np.float64) if return_pq else None
    _load().oracle_bilateral_at(_ptr(f, _fp), H, W, int(radius), float(sigma_r), int(N), float(eps),
                                int(bool(truncated)), _ptr(idx, _llp), n, _ptr(out, _dp), _ptr(P, _dp),
                                _ptr(Q, _dp))
    return (out, P, Q) if return_pq else out


def bilateral_grad(f, gbar, radius: int, sigma_r: float, N: int):
    """(dL/df, dL/dsigma_r, out) for upstream gradient gbar = dL/d out; FP64 throughout."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    gbar = np.ascontiguousarray(gbar, dtype=np.float64)
    H, W = f.shape
    gf = np.empty((H, W), np.float64)
    u = np.empty((H, W), np.float64)
    gs = ctypes.c_double(0.0)
    _load().oracle_bilateral_grad_f64(_ptr(f, _dp), _ptr(gbar, _dp), H, W, int(radius), float(sigma_r),
                                      int(N), _ptr(gf, _dp), ctypes.byref(gs), _ptr(u, _dp))
    return gf, gs.value, u


def spatial_weight(d: float, sigma_s: float, Ns: int) -> float:
    """One-dimensional spatial weight cos^Ns(d / (sigma_s sqrt Ns)); 1 for Ns = 0."""
    return _load().oracle_spatial_weight(float(d), float(sigma_s), int(Ns))


def bilateral_sp(f, radius: int, sigma_r: float, N: int, sigma_s: float, Ns: int, return_pq: bool = False):
    """Whole image with the separable spatial kernel w(dy) w(dx); N = 0 is Algorithm 1."""
    f = np.ascontiguousarray(f)
    H, W = f.shape
    out = np.empty((H, W), np.float64)
    P = np.empty((H, W), np.float64) if return_pq else None
    Q = np.empty((H, W), np.float64) if return_pq else None
    if f.dtype == np.float64:
        _load().oracle_bilateral_sp_f64(_ptr(f, _dp), H, W, int(radius), float(sigma_r), int(N), float(sigma_s),
                                        int(Ns), _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    else:
        f32 = np.ascontiguousarray(f, dtype=np.float32)
        _load().oracle_bilateral_sp(_ptr(f32, _fp), H, W, int(radius), float(sigma_r), int(N), float(sigma_s),
                                    int(Ns), _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    return (out, P, Q) if return_pq else out


def bilateral_sp_at(f, idx, radius: int, sigma_r: float, N: int, sigma_s: float, Ns: int):
    """The spatial-kernel filter at the flat (row-major) pixel indices ``idx`` only."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    H, W = f.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, np.float64)
    _load().oracle_bilateral_sp_at(_ptr(f, _fp), H, W, int(radius), float(sigma_r), int(N), float(sigma_s),
                                   int(Ns), _ptr(idx, _llp), idx.size, _ptr(out, _dp), None, None)
    return out


def poly_order_for(sigma_r: float, T: float) -> int:
    """Smallest N keeping the polynomial kernel non-negative and unimodal on [-T, T]."""
    return _load().oracle_poly_order_for(float(sigma_r), float(T))


def poly_kernel(t: float, sigma_r: float, N: int) -> float:
    """(1 - t^2 / (2 N sigma_r^2))^N; 1 for N = 0."""
    return _load().oracle_poly_kernel(float(t), float(sigma_r), int(N))


def bilateral_poly(f, radius: int, sigma_r: float, N: int, return_pq: bool = False):
    """Whole image with the polynomial range kernel and the box window."""
    f = np.ascontiguousarray(f)
    H, W = f.shape
    out = np.empty((H, W), np.float64)
    P = np.empty((H, W), np.float64) if return_pq else None
    Q = np.empty((H, W), np.float64) if return_pq else None
    if f.dtype == np.float64:
        _load().oracle_bilateral_poly_f64(_ptr(f, _dp), H, W, int(radius), float(sigma_r), int(N),
                                          _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    else:
        f32 = np.ascontiguousarray(f, dtype=np.float32)
        _load().oracle_bilateral_poly(_ptr(f32, _fp), H, W, int(radius), float(sigma_r), int(N),
                                      _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    return (out, P, Q) if return_pq else out


def bilateral_poly_at(f, idx, radius: int, sigma_r: float, N: int):
    """The polynomial-kernel filter at the flat (row-major) pixel indices ``idx`` only."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    H, W = f.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, np.float64)
    _load().oracle_bilateral_poly_at(_ptr(f, _fp), H, W, int(radius), float(sigma_r), int(N),
                                     _ptr(idx, _llp), idx.size, _ptr(out, _dp))
    return out


def nlm2(f, radius: int, sigma_1: float, N1: int, sigma_2: float, N2: int, offset, return_pq: bool = False):
    """Two-pixel-patch non-local means (Section 5, p = 2): patches {y, y + offset}, range kernel
    cos^N1(t1 / (sigma_1 sqrt N1)) cos^N2(t2 / (sigma_2 sqrt N2)); offset = (uy, ux)."""
    f = np.ascontiguousarray(f)
    H, W = f.shape
    uy, ux = (int(v) for v in offset)
    out = np.empty((H, W), np.float64)
    P = np.empty((H, W), np.float64) if return_pq else None
    Q = np.empty((H, W), np.float64) if return_pq else None
    if f.dtype == np.float64:
        _load().oracle_nlm2_f64(_ptr(f, _dp), H, W, int(radius), float(sigma_1), int(N1), float(sigma_2), int(N2),
                                uy, ux, _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    else:
        f32 = np.ascontiguousarray(f, dtype=np.float32)
        _load().oracle_nlm2(_ptr(f32, _fp), H, W, int(radius), float(sigma_1), int(N1), float(sigma_2), int(N2),
                            uy, ux, _ptr(out, _dp), _ptr(P, _dp), _ptr(Q, _dp))
    return (out, P, Q) if return_pq else out


def nlm2_at(f, idx, radius: int, sigma_1: float, N1: int, sigma_2: float, N2: int, offset):
    """The two-pixel-patch filter at the flat (row-major) pixel indices ``idx`` only."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    H, W = f.shape
    uy, ux = (int(v) for v in offset)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, np.float64)
    _load().oracle_nlm2_at(_ptr(f, _fp), H, W, int(radius), float(sigma_1), int(N1), float(sigma_2), int(N2),
                           uy, ux, _ptr(idx, _llp), idx.size, _ptr(out, _dp))
    return out
