"""ctypes wrapper over the oracle's C ray tracer (test infrastructure).

The C source states the model: travel-time-parameterised ray equations from
the Eikonal equation (Eq. 6), spreading from the Transport equation (Eq. 7),
absorption accumulated along rays (Eq. 5), first-arrival interpolation of
the wavefront mesh onto pixels and receivers.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import LIB, build

_lib = None


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("h", ctypes.c_double), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("m", ctypes.c_int32), ("R", ctypes.c_double), ("s_bg", ctypes.c_double),
                ("n_rays", ctypes.c_int32), ("dtau", ctypes.c_double), ("nmax", ctypes.c_int32),
                ("r_die", ctypes.c_double), ("j_min", ctypes.c_double),
                ("bary_tol", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = ctypes.CDLL(LIB)
        _lib.orc_tables.restype = ctypes.c_int
        _lib.orc_trace_fan.restype = ctypes.c_int
        _lib.orc_rx_links.restype = ctypes.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_params(geom, topts) -> Params:
    """Resolve the ray options.  dtau and tau_max must be given (> 0): they
    fix the node count nmax = floor(tau_max / dtau).  Rays end at the first
    node beyond R + 2h; j_min defaults to h/4."""
    if not (topts.dtau > 0.0 and topts.tau_max > 0.0):
        raise ValueError("dtau and tau_max must be positive")
    j_min = topts.j_min if topts.j_min > 0.0 else 0.25 * geom.h
    return Params(nx=geom.nx, ny=geom.ny, h=geom.h, x0=geom.x0, y0=geom.y0, m=geom.m,
                  R=geom.ring_radius, s_bg=1.0 / geom.c_background, n_rays=topts.n_rays,
                  dtau=topts.dtau, nmax=int(math.floor(topts.tau_max / topts.dtau)),
                  r_die=geom.ring_radius + 2.0 * geom.h, j_min=j_min, bary_tol=1e-12)


def trace_fan(geom, topts, s: np.ndarray, alpha, e: int) -> dict:
    """All nodes of emitter e's fan: arrays [(nmax+1)][n_rays] and L[n_rays]."""
    P = make_params(geom, topts)
    s = np.ascontiguousarray(s, np.float64).reshape(-1)
    al = None if alpha is None else np.ascontiguousarray(alpha, np.float64).reshape(-1)
    shape = (P.nmax + 1, P.n_rays)
    out = {k: np.full(shape, np.nan) for k in ("x", "y", "px", "py", "b", "amp")}
    L = np.zeros(P.n_rays, np.int32)
    lib().orc_trace_fan(ctypes.byref(P), _p(s), None if al is None else _p(al), int(e),
                        _p(out["x"]), _p(out["y"]), _p(out["px"]), _p(out["py"]),
                        _p(out["b"]), _p(out["amp"]), _p(L))
    out["L"] = L
    out["tau"] = np.arange(P.nmax + 1) * P.dtau
    return out


def rx_links(geom, topts, s: np.ndarray, alpha, e: int) -> dict:
    """Emitter e's fan and its first arrivals at the ring elements with the
    winning triangle: x, y [(nmax+1)][n_rays], L [n_rays], T [m] (NaN if
    uncovered), tri [m] = 2 (n n_rays + j) + t (-1 if uncovered) and the
    barycentrics bary [m][3] of the element in that triangle."""
    P = make_params(geom, topts)
    s = np.ascontiguousarray(s, np.float64).reshape(-1)
    al = None if alpha is None else np.ascontiguousarray(alpha, np.float64).reshape(-1)
    shape = (P.nmax + 1, P.n_rays)
    x = np.full(shape, np.nan)
    y = np.full(shape, np.nan)
    L = np.zeros(P.n_rays, np.int32)
    T = np.empty(geom.m)
    W = np.empty(geom.m, np.int64)
    bary = np.empty((geom.m, 3))
    rc = lib().orc_rx_links(ctypes.byref(P), _p(s), None if al is None else _p(al), int(e), _p(x), _p(y),
                            _p(L), _p(T), _p(W), _p(bary))
    if rc != 0:
        raise MemoryError("oracle rx_links: allocation failed")
    return {"x": x, "y": y, "L": L, "T": T, "tri": W, "bary": bary, "nmax": P.nmax}


def tables(geom, topts, s: np.ndarray, alpha, e0: int = 0, e1: int | None = None):
    """Ray-to-grid tables for emitters [e0, e1).

    Returns T [ne][N], amp [ne][N], att [ne][N] (pixel-major, FP64; T = NaN
    where no ray triangle covers the pixel) and the same at the ring elements
    T_rx, amp_rx, att_rx [ne][m]."""
    if e1 is None:
        e1 = geom.m
    P = make_params(geom, topts)
    ne, N, m = e1 - e0, geom.n_pixels, geom.m
    s = np.ascontiguousarray(s, np.float64).reshape(-1)
    al = None if alpha is None else np.ascontiguousarray(alpha, np.float64).reshape(-1)
    T = np.empty((ne, N)); A = np.empty((ne, N)); B = np.empty((ne, N))
    Tr = np.empty((ne, m)); Ar = np.empty((ne, m)); Br = np.empty((ne, m))
    rc = lib().orc_tables(ctypes.byref(P), _p(s), None if al is None else _p(al),
                          int(e0), int(e1), _p(T), _p(A), _p(B), _p(Tr), _p(Ar), _p(Br))
    if rc != 0:
        raise MemoryError("oracle tables: allocation failed")
    return T, A, B, Tr, Ar, Br


def bilinear(geom, f: np.ndarray, out: float, x: np.ndarray, y: np.ndarray):
    """Bilinear value and gradient of a grid field at points (x, y)."""
    P = make_params(geom, type("o", (), {"dtau": 1.0, "tau_max": 1.0, "j_min": 0.0,
                                          "n_rays": 3})())
    f = np.ascontiguousarray(f, np.float64).reshape(-1)
    x = np.ascontiguousarray(x, np.float64).reshape(-1)
    y = np.ascontiguousarray(y, np.float64).reshape(-1)
    v = np.empty_like(x); gx = np.empty_like(x); gy = np.empty_like(x)
    lib().orc_bilinear(ctypes.byref(P), _p(f), ctypes.c_double(out), int(x.size),
                       _p(x), _p(y), _p(v), _p(gx), _p(gy))
    return v, gx, gy
