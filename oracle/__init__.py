"""FP64 CPU oracle for one Vegas iteration (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The product path (the HIP library and its Python
binding) never imports it, and the two share no code.

The arithmetic lives in ``vegas_oracle.c`` (plain C, binary64, no FMA
contraction, no fast-math); this module compiles it with gcc and marshals
numpy arrays through ctypes. Every function cites, in the C source, the step
of the method it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vegas_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F_CONST, F_SUM, F_GAUSS, F_LO_TOY, F_RAMBO24, F_BW_FLAT = range(6)


def build() -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (always recompiles)."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
        "-Wall", "-Wextra", "-Wno-unused-parameter",
        "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int)
_pu32 = ctypes.POINTER(ctypes.c_uint32)
_pi64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.vo_philox4x32_10.argtypes = [_pu32, _pu32, _pu32]
        L.vo_philox4x32_10.restype = None
        L.vo_uniform_grid.argtypes = [ctypes.c_int, ctypes.c_int, _pd]
        L.vo_map_dim.argtypes = [ctypes.c_int, _pd, ctypes.c_uint32, _pd, _pi, _pd]
        L.vo_map_dim.restype = None
        L.vo_rambo4.argtypes = [_d, _pd, _pd]
        L.vo_rambo4.restype = _d
        L.vo_integrand.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd]
        L.vo_integrand.restype = _d
        L.vo_weights.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd,
                                 ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_int64, _pd]
        L.vo_points.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64,
                                _pd, _pi, _pd]
        L.vo_iterate.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd,
                                 ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_uint32, _pd, _pd, _pd, _pi64]
        L.vo_refine.argtypes = [ctypes.c_int, ctypes.c_int, _pd, _pd, _d, _pd]
        L.vo_combine.argtypes = [ctypes.c_int, _pd, _pd, _pd, _pd, _pd]
        L.vo_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int,
                             ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, _d,
                             _pd, _pd, _pd, _pi64]
        for name in ("vo_uniform_grid", "vo_weights", "vo_points", "vo_iterate",
                     "vo_refine", "vo_combine", "vo_run"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_pd):
    return a.ctypes.data_as(t)


def _params(params):
    if params is None or len(params) == 0:
        return None, 0, np.zeros(1)
    p = _f64(params)
    return _p(p), len(p), p


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {rc})")


def philox4x32_10(counter, key):
    """Raw Philox4x32-10 bijection: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().vo_philox4x32_10(_p(c, _pu32), _p(k, _pu32), _p(out, _pu32))
    return out


def uniform_grid(dim, nb):
    e = np.zeros(dim * (nb + 1))
    _check(lib().vo_uniform_grid(dim, nb, _p(e)), "uniform_grid")
    return e.reshape(dim, nb + 1)


def map_dim(nb, edges_row, r):
    e = _f64(edges_row)
    x = ctypes.c_double()
    k = ctypes.c_int()
    j = ctypes.c_double()
    lib().vo_map_dim(nb, _p(e), ctypes.c_uint32(int(r)), ctypes.byref(x), ctypes.byref(k),
                     ctypes.byref(j))
    return x.value, k.value, j.value


def rambo4(sqrt_s, u):
    uu = _f64(u)
    p = np.zeros(16)
    W = lib().vo_rambo4(sqrt_s, _p(uu), _p(p))
    return p.reshape(4, 4), W


def integrand(fid, x, params=None):
    xx = _f64(x)
    pp, np_, _keep = _params(params)
    return lib().vo_integrand(fid, len(xx), pp, np_, _p(xx))


def weights(edges, fid, params, seed, t, first, count):
    e = _f64(edges)
    dim, nb1 = e.shape
    pp, np_, _keep = _params(params)
    w = np.zeros(count)
    _check(lib().vo_weights(dim, nb1 - 1, _p(e), fid, pp, np_, seed, t, first, count, _p(w)),
           "weights")
    return w


def points(edges, seed, t, first, count):
    e = _f64(edges)
    dim, nb1 = e.shape
    x = np.zeros((count, dim))
    k = np.zeros((count, dim), dtype=np.int32)
    jac = np.zeros(count)
    _check(lib().vo_points(dim, nb1 - 1, _p(e), seed, t, first, count, _p(x), _p(k, _pi),
                           _p(jac)), "points")
    return x, k, jac


def iterate(edges, fid, params, n_events, seed, t):
    """One iteration: returns (I, sigma, hist[dim][nb], n_nonfinite)."""
    e = _f64(edges)
    dim, nb1 = e.shape
    pp, np_, _keep = _params(params)
    I = ctypes.c_double()
    s = ctypes.c_double()
    h = np.zeros((dim, nb1 - 1))
    bad = ctypes.c_int64()
    _check(lib().vo_iterate(dim, nb1 - 1, _p(e), fid, pp, np_, n_events, seed, t,
                            ctypes.byref(I), ctypes.byref(s), _p(h), ctypes.byref(bad)),
           "iterate")
    return I.value, s.value, h, bad.value


def refine(edges, hist, alpha):
    e = _f64(edges)
    h = _f64(hist)
    dim, nb1 = e.shape
    out = np.zeros_like(e)
    _check(lib().vo_refine(dim, nb1 - 1, _p(e), _p(h), alpha, _p(out)), "refine")
    return out


def combine(I_t, sigma_t):
    a = _f64(I_t)
    b = _f64(sigma_t)
    I = ctypes.c_double()
    s = ctypes.c_double()
    c = ctypes.c_double()
    _check(lib().vo_combine(len(a), _p(a), _p(b), ctypes.byref(I), ctypes.byref(s),
                            ctypes.byref(c)), "combine")
    return I.value, s.value, c.value


def run(dim, nb, fid, params, n_events, seed, n_iter, alpha):
    """A whole run from the uniform grid: returns (I_t, sigma_t, final edges, n_nonfinite)."""
    pp, np_, _keep = _params(params)
    I_t = np.zeros(n_iter)
    s_t = np.zeros(n_iter)
    e = np.zeros((dim, nb + 1))
    bad = ctypes.c_int64()
    _check(lib().vo_run(dim, nb, fid, pp, np_, n_events, seed, n_iter, alpha, _p(I_t),
                        _p(s_t), _p(e), ctypes.byref(bad)), "run")
    return I_t, s_t, e, bad.value
