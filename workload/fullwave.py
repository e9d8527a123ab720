"""Full-wave synthetic transmission data (frequency-domain Helmholtz FD).

An input generator, not part of the inversion: it produces measured-data
stand-ins from a wave model other than the inversion's ray model, so that
tests and experiments need not commit the inverse crime (inverting data
made with the inversion's own forward model).  The Helmholtz equation of
the paper's Forward Problem section (Eq. 1, time factor exp(-i omega t)),

    (laplacian + k(x)^2) G_e = -delta(x - x_e),
    k = omega s(x) + i alpha0(x) (f / 1 MHz)^y,

is solved for every emitter on a uniform grid `refine` times finer than the
pixel grid, with s and alpha0 bilinear between pixel centres (water, no
absorption, outside the grid), a second-order five-point stencil and a
perfectly matched layer (complex coordinate stretch s_x = 1 + i sigma/omega,
quadratic profile) around the ring.  Multiplying the stretched operator by
s_x s_y makes the matrix complex symmetric, so the data are reciprocal.
Sources are spread to and receivers read from the four surrounding nodes
with bilinear weights.  p[e][r] = G_e(x_r): the same normalisation as the
Green's functions of the inversion (s(omega) = 1, Eq. 2); the diagonal is 0.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _bilinear_field(geom, f_grid: np.ndarray, outside: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of a pixel field at points; `outside` beyond
    the pixel centres (one padded ring of cells, then constant)."""
    pad = np.full((geom.ny + 2, geom.nx + 2), outside, np.float64)
    pad[1:-1, 1:-1] = f_grid
    u = (x - geom.x0) / geom.h + 1.0
    v = (y - geom.y0) / geom.h + 1.0
    inside = (u >= 0.0) & (u <= geom.nx + 1.0) & (v >= 0.0) & (v <= geom.ny + 1.0)
    uc = np.clip(u, 0.0, geom.nx + 1.0 - 1e-9)
    vc = np.clip(v, 0.0, geom.ny + 1.0 - 1e-9)
    i = np.floor(uc).astype(np.int64)
    j = np.floor(vc).astype(np.int64)
    fu = uc - i
    fv = vc - j
    i1 = np.minimum(i + 1, geom.nx + 1)
    j1 = np.minimum(j + 1, geom.ny + 1)
    val = ((1 - fu) * (1 - fv) * pad[j, i] + fu * (1 - fv) * pad[j, i1]
           + (1 - fu) * fv * pad[j1, i] + fu * fv * pad[j1, i1])
    return np.where(inside, val, outside)


class HelmholtzGrid:
    """FD grid covering the pixel grid and the ring, plus the PML."""

    def __init__(self, geom, refine: int = 4, pml_wavelengths: float = 1.5, f_min: float = 2e5):
        self.geom = geom
        self.hf = geom.h / refine
        half = max(geom.ring_radius + 2.0 * geom.h,
                   max(abs(geom.x0), abs(geom.x0 + (geom.nx - 1) * geom.h),
                       abs(geom.y0), abs(geom.y0 + (geom.ny - 1) * geom.h)) + geom.h)
        self.pml = pml_wavelengths * geom.c_background / f_min
        self.half_in = half
        n_half = int(math.ceil((half + self.pml) / self.hf))
        self.n = 2 * n_half + 1
        self.coords = (np.arange(self.n) - n_half) * self.hf

    def sigma(self, xs: np.ndarray) -> np.ndarray:
        d = np.clip(np.abs(xs) - self.half_in, 0.0, None) / self.pml
        smax = 3.0 * self.geom.c_background * math.log(1e6) / (2.0 * self.pml)
        return smax * d * d

    def matrix(self, k2: np.ndarray, omega: float) -> sp.csc_matrix:
        """s_x s_y (laplacian_stretched + k^2) on the nodes (Dirichlet
        outside), complex symmetric."""
        n, hf = self.n, self.hf
        x = self.coords
        sx = 1.0 + 1j * self.sigma(x) / omega
        sxh = 1.0 + 1j * self.sigma(x[:-1] + 0.5 * hf) / omega   # between nodes a and a+1
        # 1-D second-difference with stretching: D^T diag(1/s_half) D / hf^2
        main = np.zeros(n, np.complex128)
        main[:-1] -= 1.0 / sxh
        main[1:] -= 1.0 / sxh
        off = 1.0 / sxh
        L1 = sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="csr") / (hf * hf)
        I = sp.identity(n, format="csr")
        Sx = sp.diags(sx, 0, format="csr")
        # node index = b * n + a (row b = y, column a = x)
        A = sp.kron(Sx, L1, format="csr") + sp.kron(L1, Sx, format="csr")
        A = A + sp.diags((np.outer(sx, sx) * k2).reshape(-1), 0, format="csr")
        del I
        return A.tocsc()

    def spread(self, px: float, py: float) -> sp.csr_matrix:
        """Bilinear weights of a point on the nodes, as a 1 x n^2 row."""
        n, hf = self.n, self.hf
        u = (px - self.coords[0]) / hf
        v = (py - self.coords[0]) / hf
        a, b = int(math.floor(u)), int(math.floor(v))
        fu, fv = u - a, v - b
        cols = [b * n + a, b * n + a + 1, (b + 1) * n + a, (b + 1) * n + a + 1]
        vals = [(1 - fu) * (1 - fv), fu * (1 - fv), (1 - fu) * fv, fu * fv]
        return sp.csr_matrix((vals, ([0, 0, 0, 0], cols)), shape=(1, n * n))


def helmholtz_data(geom, c: np.ndarray, alpha: np.ndarray | None, freqs, y_pow: float = 1.0,
                   refine: int = 4) -> np.ndarray:
    """[nf][m][m] complex128: G_e(x_r) from the Helmholtz equation."""
    fr = np.asarray(freqs, np.float64)
    H = HelmholtzGrid(geom, refine=refine, f_min=float(fr.min()))
    X, Y = np.meshgrid(H.coords, H.coords)
    s = _bilinear_field(geom, 1.0 / np.asarray(c, np.float64), 1.0 / geom.c_background, X, Y)
    al = np.zeros_like(s) if alpha is None else _bilinear_field(geom, np.asarray(alpha, np.float64), 0.0, X, Y)
    pos = geom.element_positions()
    m = geom.m
    B = sp.vstack([H.spread(pos[e, 0], pos[e, 1]) for e in range(m)]).tocsr()   # [m][n^2]
    out = np.zeros((len(fr), m, m), np.complex128)
    for k, f in enumerate(fr):
        omega = 2.0 * math.pi * f
        kk = omega * s + 1j * al * (f * 1e-6) ** y_pow
        A = H.matrix(kk * kk, omega)
        lu = spla.splu(A, permc_spec="COLAMD")
        rhs = -(B.T.toarray()) / (H.hf * H.hf)
        U = lu.solve(rhs.astype(np.complex128))
        P = B @ U                         # P[r][e] = G_e(x_r)
        out[k] = P.T
        out[k][np.arange(m), np.arange(m)] = 0.0
    return out
