"""Data weights, the diagonally weighted single step, the CG solution of the
linear subproblem and the frequency sweep.

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
* reported update norm: sqrt(sum_x (c_new - c)^2) in m/s;
* CG (the paper's earlier, iterative solution of the linearised equation):
  see invert_frequency_set_cg for its readings;
* asymptotic (amplitude-normalised) weights: see
  invert_frequency_set_asymptotic (parity with the cited weights unpinned).
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


def linearise(geom, topts, iopts, c: np.ndarray, alpha, freqs, p_meas) -> dict:
    """Everything one frequency set's linear subproblem needs, in the model c.

    Rays and tables in c, G and the modelled data per frequency, residual D,
    data weight W, gradient grad = J^T W D, Hessian diagonal Hd, support S,
    the diagonal weight den = Hd + eps max_S Hd and the pixels where it is
    used, ok = S and den > 0."""
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
    return {"c": c, "s": s, "dA": dA, "freqs": list(freqs), "T": T, "amp": A, "att": B,
            "T_rx": Tr, "amp_rx": Ar, "att_rx": Br, "G": Gs, "D": Ds, "W": Ws,
            "grad": grad, "hdiag": hd, "support": S, "hmax": hmax, "den": den, "ok": ok}


def apply_update(c: np.ndarray, s: np.ndarray, delta: np.ndarray):
    """q = 1/c^2 + delta where delta != 0; returns (c_new, dc_l2)."""
    q = s.reshape(-1) * s.reshape(-1) + delta
    if np.any(q[delta != 0.0] <= 0.0):
        raise NumericError("1/c^2 + delta is not positive")
    c_flat = c.reshape(-1)
    c_new = c_flat.copy()
    nz = delta != 0.0
    c_new[nz] = 1.0 / np.sqrt(q[nz])
    dc = c_new - c_flat
    dc_l2 = math.sqrt(float(np.sum(dc * dc)))
    return c_new.reshape(c.shape), dc_l2


def invert_frequency_set(geom, topts, iopts, c: np.ndarray, alpha, freqs, p_meas,
                         return_parts: bool = False):
    """One linearised, diagonally weighted single step for one frequency set.

    c: [ny][nx] m/s; alpha: [ny][nx] Np/(m MHz^y) or None; p_meas: [nf][m][m].
    Returns (c_new, dc_l2) or, with return_parts, a dict of intermediates."""
    L = linearise(geom, topts, iopts, c, alpha, freqs, p_meas)
    N = geom.n_pixels
    grad, den, ok = L["grad"], L["den"], L["ok"]
    v = np.zeros(N)
    v[ok] = grad[ok] / den[ok]
    num = 0.0
    dsq = 0.0
    us = []
    for k, f in enumerate(freqs):
        u = born.born_forward(L["G"][k], v, f, L["dA"])
        us.append(u)
        num += float(np.sum(L["W"][k] * np.real(np.conj(u) * L["D"][k])))
        dsq += float(np.sum(L["W"][k] * (u.real * u.real + u.imag * u.imag)))
    beta = num / dsq if dsq > 0.0 else 0.0
    delta = beta * v
    c_new, dc_l2 = apply_update(L["c"], L["s"], delta)
    if return_parts:
        parts = {k: L[k] for k in ("grad", "hdiag", "support", "T", "amp", "att", "T_rx", "amp_rx",
                                   "att_rx", "W", "D", "hmax")}
        parts.update({"c_new": c_new, "dc_l2": dc_l2, "direction": v, "beta": beta, "delta": delta,
                      "Jv": us})
        return parts
    return c_new, dc_l2


def hessian_action(L: dict, x: np.ndarray) -> np.ndarray:
    """J^T W J x summed over the frequency set (Eq. 10's Gauss-Newton Hessian
    applied to x): a Born forward, the data weight, then the adjoint."""
    out = np.zeros_like(x)
    for k, f in enumerate(L["freqs"]):
        u = born.born_forward(L["G"][k], x, f, L["dA"])
        out += born.born_adjoint(L["G"][k], L["W"][k] * u, f, L["dA"])
    return out


def invert_frequency_set_cg(geom, topts, iopts, c: np.ndarray, alpha, freqs, p_meas, n_iter: int,
                            return_parts: bool = False):
    """The linear subproblem of one frequency set solved by conjugate gradients.

    The paper's earlier method (Inverse Problem section, the paragraph on
    solving the linearised equation iteratively) solves H delta = -grad F,
    i.e. (J^T W J) delta = J^T W D, by CG.  Readings taken: the unknown lives
    on the pixels where the single step's weight is defined (ok = S and
    den > 0, zero elsewhere); the CG is preconditioned by that same diagonal
    weight den = Hd + eps max_S Hd (Jacobi), so its first iterate is exactly
    the single step's beta v; it starts from delta = 0 and runs n_iter
    iterations (early stopping is the regularisation), stopping early, with
    zero steps from then on, once r.z or p.Hp is not positive.  Textbook
    preconditioned CG (Hestenes-Stiefel), in this order per iteration i:
        q = H p;  alpha_i = r.z / p.q;  delta += alpha_i p;  r -= alpha_i q;
        z = r / den on ok;  beta = (r.z)_new / (r.z);  p = z + beta p.
    Returns (c_new, dc_l2) or, with return_parts, a dict holding also the
    step lengths alpha_i and the values r_i.z_i before each iteration."""
    if n_iter < 1:
        raise ValueError("n_iter must be >= 1")
    L = linearise(geom, topts, iopts, c, alpha, freqs, p_meas)
    ok, den = L["ok"], L["den"]
    N = geom.n_pixels
    x = np.zeros(N)
    r = np.where(ok, L["grad"], 0.0)
    z = np.zeros(N)
    z[ok] = r[ok] / den[ok]
    p = z.copy()
    rz = float(np.dot(r, z))
    alphas = np.zeros(n_iter)
    rzs = np.zeros(n_iter)
    for i in range(n_iter):
        rzs[i] = rz
        if not rz > 0.0:
            break
        q = np.where(ok, hessian_action(L, p), 0.0)
        pq = float(np.dot(p, q))
        if not pq > 0.0:
            break
        a = rz / pq
        alphas[i] = a
        x = x + a * p
        r = r - a * q
        z = np.zeros(N)
        z[ok] = r[ok] / den[ok]
        rz_new = float(np.dot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    c_new, dc_l2 = apply_update(L["c"], L["s"], x)
    if return_parts:
        parts = dict(L)
        parts.update({"c_new": c_new, "dc_l2": dc_l2, "delta": x, "alpha": alphas, "rz": rzs})
        return parts
    return c_new, dc_l2


def invert_frequency_set_asymptotic(geom, topts, iopts, c: np.ndarray, alpha, freqs, p_meas,
                                    return_parts: bool = False):
    """The frequency set with asymptotic (amplitude-normalised) weights in
    place of the Hessian-diagonal weight (the single-step paragraph's
    weighting that diagonalises the Hessian, in its ray-Born asymptotic form).

    Readings: each selected pair (e, r) on its own determines a pixel's
    perturbation exactly, D_er / (omega^2 dA G_e(x) G_r(x)), when the data
    are the Born data of that pixel alone; the direction is the W-weighted
    mean of these per-pair estimates over the pairs and frequencies whose
    Green's functions are nonzero at x,
        g_A(x) = sum_k Re sum_{e,r} W_er D_er / (omega_k^2 dA G_e(x) G_r(x)),
        n_A(x) = sum_k sum_{e,r} W_er [G_e(x) != 0] [G_r(x) != 0],
        v(x)   = g_A(x) / n_A(x) on the support S where n_A > 0, else 0;
    no obliquity factor.  The step length beta is the exact minimiser of the
    linearised objective along v and the update is that of the single step.
    (The cited reference's exact weights are not in the paper.)"""
    L = linearise(geom, topts, iopts, c, alpha, freqs, p_meas)
    N = geom.n_pixels
    gA = np.zeros(N)
    nA = np.zeros(N)
    for k, f in enumerate(freqs):
        G = L["G"][k]
        om2dA = (2.0 * math.pi * f) ** 2 * L["dA"]
        nz = G != 0
        Ginv = np.zeros_like(G)
        Ginv[nz] = 1.0 / G[nz]
        Y = (L["W"][k] * L["D"][k]) @ Ginv            # sum over r
        gA += np.real(np.sum(Ginv * Y, axis=0)) / om2dA
        ind = nz.astype(np.float64)
        nA += np.sum(ind * (L["W"][k] @ ind), axis=0)
    ok = L["support"] & (nA > 0.0)
    v = np.zeros(N)
    v[ok] = gA[ok] / nA[ok]
    num = 0.0
    dsq = 0.0
    us = []
    for k, f in enumerate(freqs):
        u = born.born_forward(L["G"][k], v, f, L["dA"])
        us.append(u)
        num += float(np.sum(L["W"][k] * np.real(np.conj(u) * L["D"][k])))
        dsq += float(np.sum(L["W"][k] * (u.real * u.real + u.imag * u.imag)))
    beta = num / dsq if dsq > 0.0 else 0.0
    delta = beta * v
    c_new, dc_l2 = apply_update(L["c"], L["s"], delta)
    if return_parts:
        parts = dict(L)
        parts.update({"c_new": c_new, "dc_l2": dc_l2, "direction": v, "beta": beta, "delta": delta,
                      "g_A": gA, "n_A": nA, "Jv": us})
        return parts
    return c_new, dc_l2


def sweep(geom, topts, iopts, c0, alpha, freq_sets, p_meas_sets):
    """Low-to-high frequency sweep: each set's image starts the next set."""
    c = np.asarray(c0, np.float64).copy()
    hist = []
    for fs, pm in zip(freq_sets, p_meas_sets):
        c, dl2 = invert_frequency_set(geom, topts, iopts, c, alpha, fs, pm)
        hist.append(dl2)
    return c, hist
