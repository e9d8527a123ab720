"""Data weights, the diagonally weighted single step and the frequency sweep.

Plain NumPy FP64, test infrastructure.  Follows the paper's Inverse Problem
section (Eqs. 8-10 and the single-step paragraph) and the data handling of
its Results section.  Readings taken where the paper is silent:

* receiver selection ("opposite 75 % of the ring"): receiver r is used for
  emitter e iff the circular index distance d(e, r) >= ceil((1-f) m / 2);
  for f = 0.75 that is 8 d >= m, i.e. 0.75 m + 1 receivers per emitter;
* outlier zeroing ("largest 1 % of values set to zero"): per frequency,
  over the selected pairs, the floor(0.01 n_valid) pairs with the largest
  measured |p|^2 (computed as re*re + im*im) get weight 0; ties go to the
  smaller flat index e*m + r;
* residual D = p_meas - p_model, modelled data p_er = G_e(x_r) (Eq. 2 with
  s(omega) = 1, the Green's function evaluated at the receiver);
* single step: grad = J^T (W D) and Hd = diag(J^T W J) summed over the set;
  the solution-space weight is 1 / (Hd + eps max_S Hd) on the support S
  (pixels inside |x| < R - margin reached by every emitter's rays), zero
  elsewhere; the weighted direction v = S grad / (Hd + eps max_S Hd) is
  scaled by the exact minimiser of the linearised objective along it,
  beta = Re<J v, W D> / <J v, W J v>, so delta = beta v;
* update of q = 1/c^2: c_new = (1/c^2 + delta)^(-1/2) where delta != 0,
  c unchanged elsewhere; a non-positive q is an error;
* reported update norm: sqrt(sum_x (c_new - c)^2) in m/s.
"""
from __future__ import annotations

import math

import numpy as np

from . import born, rays


class NumericError(RuntimeError):
    pass


def receiver_dmin(m: int, recv_fraction: float) -> int:
    return int(math.ceil((1.0 - recv_fraction) * 0.5 * m - 1e-9))


def receiver_mask(m: int, recv_fraction: float = 0.75) -> np.ndarray:
    """[m][m] bool: True where r is on the opposite part of the ring from e."""
    e = np.arange(m)[:, None]
    r = np.arange(m)[None, :]
    d = np.abs(e - r)
    d = np.minimum(d, m - d)
    return d >= receiver_dmin(m, recv_fraction)


def outlier_weights(p_meas: np.ndarray, mask: np.ndarray, outlier_fraction: float) -> np.ndarray:
    """[m][m] float 0/1: zero at the k largest |p_meas|^2 among masked pairs."""
    m = mask.shape[0]
    w = mask.astype(np.float64)
    idx = np.flatnonzero(mask.reshape(-1))
    k = int(math.floor(outlier_fraction * idx.size))
    if k <= 0:
        return w
    p = p_meas.reshape(-1)[idx]
    mag2 = p.real * p.real + p.imag * p.imag
    order = np.lexsort((idx, -mag2))
    w.reshape(-1)[idx[order[:k]]] = 0.0
    return w


def support(geom, T: np.ndarray) -> np.ndarray:
    """[N] bool: pixel centre inside |x| < R - margin and covered for every e."""
    X, Y = geom.pixel_centres()
    rs = geom.ring_radius - geom.support_margin
    inside = (X * X + Y * Y < rs * rs).reshape(-1)
    return inside & np.all(np.isfinite(T), axis=0)


def invert_frequency_set(geom, topts, iopts, c: np.ndarray, alpha, freqs, p_meas,
                         return_parts: bool = False):
    """One linearised, diagonally weighted single step for one frequency set.

    c: [ny][nx] m/s; alpha: [ny][nx] Np/(m MHz^y) or None; p_meas: [nf][m][m].
    Returns (c_new, dc_l2) or, with return_parts, a dict of intermediates."""
    c = np.asarray(c, np.float64)
    s = 1.0 / c
    T, A, B, Tr, Ar, Br = rays.tables(geom, topts, s, alpha)
    m, N = geom.m, geom.n_pixels
    dA = geom.h * geom.h
    mask = receiver_mask(m, iopts.recv_fraction)
    grad = np.zeros(N)
    hd = np.zeros(N)
    Gs, Ds, Ws = [], [], []
    for k, f in enumerate(freqs):
        G = born.green(T, A, B, f, iopts.y_pow)
        p = born.green(Tr, Ar, Br, f, iopts.y_pow)
        D = p_meas[k] - p
        W = outlier_weights(p_meas[k], mask, iopts.outlier_fraction)
        grad += born.born_adjoint(G, W * D, f, dA)
        hd += born.hessian_diag(G, W, f, dA)
        Gs.append(G); Ds.append(D); Ws.append(W)
    S = support(geom, T)
    hmax = float(np.max(hd[S])) if S.any() else 0.0
    den = hd + iopts.eps * hmax
    ok = S & (den > 0.0)
    v = np.zeros(N)
    v[ok] = grad[ok] / den[ok]
    num = 0.0
    dsq = 0.0
    us = []
    for k, f in enumerate(freqs):
        u = born.born_forward(Gs[k], v, f, dA)
        us.append(u)
        num += float(np.sum(Ws[k] * np.real(np.conj(u) * Ds[k])))
        dsq += float(np.sum(Ws[k] * (u.real * u.real + u.imag * u.imag)))
    beta = num / dsq if dsq > 0.0 else 0.0
    delta = beta * v
    q = s.reshape(-1) * s.reshape(-1) + delta
    if np.any(q[delta != 0.0] <= 0.0):
        raise NumericError("1/c^2 + delta is not positive")
    c_flat = c.reshape(-1)
    c_new = c_flat.copy()
    nz = delta != 0.0
    c_new[nz] = 1.0 / np.sqrt(q[nz])
    dc = c_new - c_flat
    dc_l2 = math.sqrt(float(np.sum(dc * dc)))
    c_new = c_new.reshape(c.shape)
    if return_parts:
        return {"c_new": c_new, "dc_l2": dc_l2, "grad": grad, "hdiag": hd, "support": S,
                "direction": v, "beta": beta, "delta": delta, "T": T, "amp": A, "att": B,
                "T_rx": Tr, "amp_rx": Ar, "att_rx": Br, "W": Ws, "D": Ds, "Jv": us,
                "hmax": hmax}
    return c_new, dc_l2


def sweep(geom, topts, iopts, c0, alpha, freq_sets, p_meas_sets):
    """Low-to-high frequency sweep: each set's image starts the next set."""
    c = np.asarray(c0, np.float64).copy()
    hist = []
    for fs, pm in zip(freq_sets, p_meas_sets):
        c, dl2 = invert_frequency_set(geom, topts, iopts, c, alpha, fs, pm)
        hist.append(dl2)
    return c, hist
