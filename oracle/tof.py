"""Time-of-flight (ToF) initial model by bent-ray ToF inversion, plain NumPy
FP64 (test infrastructure).

The paper's ray-Born reconstructions start from a low-resolution,
low-contrast image obtained from three iterations of a ToF-based method
that minimises the misfit between measured ToFs and ToFs modelled along
rays (Results section; Inverse Problem section for the smooth starting
guess; Discussion for ray linking).  The paper defers the method itself to
its references; the readings taken here:

* measured ToF: an input T_meas [m][m] (NaN where no ToF was picked);
* modelled ToF T_er(c): the first-arrival travel time at element r of
  emitter e's ray fan, i.e. the receiver table of the Green's functions;
* linking path: the first-arrival triangle of the wavefront mesh at r (cell
  (n, j), triangle t, barycentrics la, lb, lc) gives the step index
  u = la u_a + lb u_b + lc u_c and the weight w of ray j + 1 (t = 0:
  lb + lc; t = 1: lb); the path is ray j with weight 1 - w and ray j + 1
  with weight w, each from its emitter node to the point at parameter u
  (nodes 0 .. floor(u), then x_K + frac(u) (x_{K+1} - x_K));
* linearisation (Fermat's principle): dT_er = integral of ds along the
  path, with ds bilinear in the pixel values as the tracer interpolates s;
  along each polyline by the trapezoid rule, i.e. node i carries half of
  its two adjacent segment lengths, and its bilinear weights go to the four
  surrounding pixel centres (corners outside the grid are water and carry
  no unknown): L[er, p];
* one iteration: retrace in c; dT = T_meas - T on the pairs that are
  selected (receiver selection of the ray-Born step), measured and covered;
  g = L^T dT and the ray density C = L^T 1; on the support S (pixel centre
  inside |x| < R - margin and C > 0) the diagonally weighted direction
  v = g / (C + eps max_S C), zero elsewhere; the exact minimiser of the
  linearised misfit along v, beta = <L v, dT> / <L v, L v>; s += beta v;
  c = 1/s where beta v != 0.  A non-positive s is an error.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import invert, rays


def hat_weights(geom, x: np.ndarray, y: np.ndarray):
    """Bilinear weights of the pixel values at points (x, y): pixel indices
    [n][4] (-1 where the corner is outside the grid) and weights [n][4]."""
    u = (np.asarray(x) - geom.x0) / geom.h
    v = (np.asarray(y) - geom.y0) / geom.h
    fi = np.floor(u)
    fj = np.floor(v)
    fu = u - fi
    fv = v - fj
    i = fi.astype(np.int64)
    j = fj.astype(np.int64)
    ci = np.stack([i, i + 1, i, i + 1], -1)
    cj = np.stack([j, j, j + 1, j + 1], -1)
    w = np.stack([(1 - fu) * (1 - fv), fu * (1 - fv), (1 - fu) * fv, fu * fv], -1)
    ok = (ci >= 0) & (ci < geom.nx) & (cj >= 0) & (cj < geom.ny)
    idx = np.where(ok, cj * geom.nx + ci, -1)
    return idx, np.where(ok, w, 0.0)


def path_nodes(x: np.ndarray, y: np.ndarray, q: int, u: float):
    """Points of ray q from its emitter node to parameter u, and the
    trapezoid weight of each point (half its adjacent segment lengths)."""
    K = int(math.floor(u))
    fr = u - K
    px = list(x[: K + 1, q])
    py = list(y[: K + 1, q])
    if fr > 0.0:
        px.append(x[K, q] + fr * (x[K + 1, q] - x[K, q]))
        py.append(y[K, q] + fr * (y[K + 1, q] - y[K, q]))
    px = np.array(px)
    py = np.array(py)
    seg = np.hypot(np.diff(px), np.diff(py))
    wt = np.zeros(px.size)
    wt[:-1] += 0.5 * seg
    wt[1:] += 0.5 * seg
    return px, py, wt


def link_path(links: dict, r: int):
    """(j, w, u) of the linking path at element r, or None if uncovered."""
    tri = int(links["tri"][r])
    if tri < 0:
        return None
    nr = links["x"].shape[1]
    t = tri & 1
    cell = tri >> 1
    n, j = cell // nr, cell % nr
    la, lb, lc = links["bary"][r]
    if t == 0:   # (n, j), (n, j+1), (n+1, j+1)
        u = la * n + lb * n + lc * (n + 1)
        w = lb + lc
    else:        # (n, j), (n+1, j+1), (n+1, j)
        u = la * n + lb * (n + 1) + lc * (n + 1)
        w = lb
    u = min(max(u, 0.0), float(n + 1))
    return j, w, u


def pair_kernel(geom, links: dict, r: int):
    """Row L[e r, :] as (pixel indices, weights), or None if uncovered."""
    lp = link_path(links, r)
    if lp is None:
        return None
    j, w, u = lp
    idx_all, val_all = [], []
    for q, wq in ((j, 1.0 - w), (j + 1, w)):
        px, py, wt = path_nodes(links["x"], links["y"], q, u)
        idx, hw = hat_weights(geom, px, py)
        val = wq * wt[:, None] * hw
        ok = idx >= 0
        idx_all.append(idx[ok])
        val_all.append(val[ok])
    idx = np.concatenate(idx_all)
    val = np.concatenate(val_all)
    row = np.zeros(geom.n_pixels)
    np.add.at(row, idx, val)
    nz = np.flatnonzero(row)
    return nz, row[nz]


def tof_system(geom, topts, iopts, c: np.ndarray, T_meas: np.ndarray):
    """Modelled ToFs T [m][m], the used-pair mask [m][m] and the sparse
    path matrix L [m m][N] (rows of unused pairs empty)."""
    m, N = geom.m, geom.n_pixels
    s = 1.0 / np.asarray(c, np.float64)
    sel = invert.receiver_mask(m, iopts.recv_fraction)
    T = np.full((m, m), np.nan)
    used = np.zeros((m, m), bool)
    rows, cols, vals = [], [], []
    for e in range(m):
        lk = rays.rx_links(geom, topts, s, None, e)
        T[e] = lk["T"]
        for r in range(m):
            if not (sel[e, r] and np.isfinite(T_meas[e, r]) and np.isfinite(lk["T"][r])):
                continue
            row = pair_kernel(geom, lk, r)
            if row is None:
                continue
            used[e, r] = True
            rows.append(np.full(row[0].size, e * m + r))
            cols.append(row[0])
            vals.append(row[1])
    if rows:
        L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(m * m, N))
    else:
        L = sp.csr_matrix((m * m, N))
    return T, used, L


def tof_step(geom, topts, iopts, c: np.ndarray, T_meas: np.ndarray, return_parts: bool = False):
    """One linearised ToF iteration.  Returns (c_new, rms dT before the step)."""
    c = np.asarray(c, np.float64)
    s = 1.0 / c.reshape(-1)
    T, used, L = tof_system(geom, topts, iopts, c, T_meas)
    dT = np.where(used, T_meas - np.where(used, T, 0.0), 0.0).reshape(-1)
    n_used = int(used.sum())
    rms = math.sqrt(float(np.sum(dT * dT)) / n_used) if n_used else 0.0
    g = L.T @ dT
    C = L.T @ used.reshape(-1).astype(np.float64)
    X, Y = geom.pixel_centres()
    rs = geom.ring_radius - geom.support_margin
    S = ((X * X + Y * Y) < rs * rs).reshape(-1) & (C > 0.0)
    cmax = float(np.max(C[S])) if S.any() else 0.0
    v = np.zeros(geom.n_pixels)
    den = C + iopts.eps * cmax
    v[S] = g[S] / den[S]
    Lv = L @ v
    dd = float(np.dot(Lv, Lv))
    beta = float(np.dot(Lv, dT)) / dd if dd > 0.0 else 0.0
    ds = beta * v
    s_new = s + ds
    if np.any(s_new[ds != 0.0] <= 0.0):
        raise invert.NumericError("slowness update is not positive")
    c_new = c.reshape(-1).copy()
    nz = ds != 0.0
    c_new[nz] = 1.0 / s_new[nz]
    c_new = c_new.reshape(c.shape)
    if return_parts:
        return {"c_new": c_new, "rms": rms, "T": T, "used": used, "L": L, "dT": dT, "g": g, "C": C,
                "support": S, "direction": v, "beta": beta, "Lv": Lv}
    return c_new, rms


def tof_invert(geom, topts, iopts, c0: np.ndarray, T_meas: np.ndarray, n_iter: int = 3):
    """n_iter ToF iterations from c0 (each retraces).  Returns (c, [rms dT
    before each iteration])."""
    c = np.asarray(c0, np.float64).copy()
    hist = []
    for _ in range(n_iter):
        c, rms = tof_step(geom, topts, iopts, c, T_meas)
        hist.append(rms)
    return c, hist
