"""Green's functions and Born operators, plain NumPy FP64 (test infrastructure).

Conventions: time factor exp(-i omega t); omega = 2 pi f; the unknown is the
perturbation delta of the squared slowness q = 1/c^2 on the pixel grid;
Delta A = h^2 is the pixel area.

* Green's function on the ray tables (Eqs. 4-5):
      G_e(x, omega) = a_e(x) omega^(-1/2) exp(-B_e(x) (f / 1 MHz)^y)
                      exp(i 2 pi frac(f T_e(x) + 1/8)),
  i.e. A_geom * A_abs * exp(i [omega T + pi/4]); zero where uncovered.
* Born forward operator.  Perturbing omega^2 q in the Helmholtz equation
  (Eq. 1) by omega^2 delta gives, to first order and with s(omega) = 1
  (Eq. 2) and reciprocity g(x_r, x) = G_r(x),
      (J delta)_er = omega^2 dA sum_x G_e(x) G_r(x) delta(x).
* Its adjoint for real delta under Re<.,.> on the data:
      (J^T d)(x) = omega^2 dA Re sum_{e,r} conj(G_e(x) G_r(x)) d_er.
* The diagonal of the data-weighted Gauss-Newton Hessian J^T W J (Eq. 10):
      Hd(x) = omega^4 dA^2 sum_{e,r} W_er |G_e(x)|^2 |G_r(x)|^2.
"""
from __future__ import annotations

import math

import numpy as np


def green(T: np.ndarray, amp: np.ndarray, att: np.ndarray, f: float, y_pow: float = 1.0):
    """G(f) on a table (any shape); NaN travel time means uncovered -> 0."""
    omega = 2.0 * math.pi * f
    T = np.asarray(T, np.float64)
    cov = np.isfinite(T)
    Tz = np.where(cov, T, 0.0)
    cycles = f * Tz + 0.125
    frac = cycles - np.floor(cycles)
    mag = np.asarray(amp, np.float64) * omega ** -0.5 * np.exp(
        -np.asarray(att, np.float64) * (f * 1e-6) ** y_pow)
    G = mag * np.exp(2j * math.pi * frac)
    return np.where(cov, G, 0.0 + 0.0j)


def born_forward(G: np.ndarray, delta: np.ndarray, f: float, dA: float) -> np.ndarray:
    """d[e][r] = omega^2 dA sum_x G[e,x] G[r,x] delta[x]  (G is [m][N])."""
    omega = 2.0 * math.pi * f
    return (omega * omega * dA) * ((G * delta[None, :]) @ G.T)


def born_adjoint(G: np.ndarray, d: np.ndarray, f: float, dA: float) -> np.ndarray:
    """grad[x] = omega^2 dA Re sum_{e,r} conj(G[e,x] G[r,x]) d[e,r].

    Computed as Y = d @ conj(G) (sum over r), then Re sum_e conj(G_e) Y_e."""
    omega = 2.0 * math.pi * f
    Y = d @ np.conj(G)
    return (omega * omega * dA) * np.real(np.sum(np.conj(G) * Y, axis=0))


def hessian_diag(G: np.ndarray, w: np.ndarray, f: float, dA: float) -> np.ndarray:
    """Hd[x] = omega^4 dA^2 sum_{e,r} w[e,r] |G[e,x]|^2 |G[r,x]|^2."""
    omega = 2.0 * math.pi * f
    g2 = np.abs(G) ** 2
    return (omega ** 4 * dA * dA) * np.sum(g2 * (w @ g2), axis=0)


def jacobian(G: np.ndarray, f: float, dA: float) -> np.ndarray:
    """Explicit J as a [m*m][N] complex matrix (tiny problems only)."""
    omega = 2.0 * math.pi * f
    m = G.shape[0]
    return (omega * omega * dA) * (G[:, None, :] * G[None, :, :]).reshape(m * m, -1)
