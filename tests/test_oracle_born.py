"""Pins for the oracle's Green's functions and Born operators (CPU only).

Independent references: the exact 2-D Green's function (i/4) H0(kr) from
scipy (Eq. 3), its far-field form with the +pi/4 phase (Eq. 4), the first
Born term of the Helmholtz equation (Eq. 1) built from exact Hankel
functions, the dot-product identity of an operator and its adjoint, and the
Hessian diagonal assembled column by column through the forward operator.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special

import workload as W
from oracle import born, rays
from oracle.invert import receiver_mask

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


@pytest.fixture(scope="module")
def water():
    g = W.centred_grid(81, 0.5e-3, 16, 18e-3, 1500.0)
    c = np.full((g.ny, g.nx), 1500.0)
    to = W.resolve_trace_opts(g, c, 720)
    tabs = rays.tables(g, to, 1.0 / c, None)
    return g, tabs


def test_green_phase_convention_at_source_point():
    """T = 0 gives the phase offset pi/4 of Eq. 4 exactly; a/sqrt(omega) magnitude."""
    gold = json.load(open(GOLD))["green_phase_offset_rad"]["value"]
    f = 300e3
    G = born.green(np.array([0.0]), np.array([10.0]), np.array([0.0]), f)
    assert abs(np.angle(G[0]) - gold) < 1e-15
    assert abs(abs(G[0]) - 10.0 / math.sqrt(2 * math.pi * f)) < 1e-15
    # absorption: exp(-B (f / 1 MHz)^y)
    G2 = born.green(np.array([0.0]), np.array([10.0]), np.array([0.3]), 2e6, y_pow=1.0)
    assert abs(abs(G2[0]) - 10.0 / math.sqrt(2 * math.pi * 2e6) * math.exp(-0.6)) < 1e-15
    # uncovered -> 0
    assert born.green(np.array([np.nan]), np.array([1.0]), np.array([0.0]), f)[0] == 0


def test_green_matches_exact_2d_hankel(water):
    """Ray G in water vs (i/4) H0^(1)(kr): relative error ~ 1/(8 kr)."""
    g, (T, A, B, Tr, Ar, Br) = water
    X, Y = g.pixel_centres()
    pos = g.element_positions()
    for f in (250e3, 400e3):
        k = 2 * math.pi * f / 1500.0
        G = born.green(T, A, B, f)
        for e in (0, 5, 9):
            r = np.hypot(X - pos[e, 0], Y - pos[e, 1]).ravel()
            ok = np.isfinite(T[e]) & (k * r > 20.0)
            gex = 0.25j * special.hankel1(0, k * r[ok])
            rel = np.abs(G[e][ok] - gex) / np.abs(gex)
            assert np.all(rel <= 1.05 / (8.0 * k * r[ok]) + 5e-4)


def test_born_point_scatterer_closed_form_and_hankel(water):
    """d_er for one scattering pixel: the closed form
    omega^2 dA delta exp(i(k(r_e + r_r) + pi/2)) / (8 pi k sqrt(r_e r_r)), and
    the first Born term of Eq. 1 with exact Green's functions."""
    g, (T, A, B, Tr, Ar, Br) = water
    X, Y = g.pixel_centres()
    pos = g.element_positions()
    f = 400e3
    om = 2 * math.pi * f
    k = om / 1500.0
    G = born.green(T, A, B, f)
    ic = 40 * 81 + 40
    xs, ys = X.ravel()[ic], Y.ravel()[ic]
    dval = 1e-8
    delta = np.zeros(g.n_pixels)
    delta[ic] = dval
    d = born.born_forward(G, delta, f, g.h ** 2)
    rr = np.hypot(pos[:, 0] - xs, pos[:, 1] - ys)
    closed = om * om * g.h ** 2 * dval * np.exp(1j * (k * (rr[:, None] + rr[None, :]) + 0.5 * math.pi)) \
        / (8 * math.pi * k * np.sqrt(rr[:, None] * rr[None, :]))
    assert np.max(np.abs(d - closed)) / np.max(np.abs(closed)) < 2e-3
    gh = 0.25j * special.hankel1(0, k * rr)
    exact = om * om * g.h ** 2 * dval * np.outer(gh, gh)
    msk = receiver_mask(g.m)
    assert np.max(np.abs(d - exact)[msk]) / np.max(np.abs(exact)) < 2.2 / (8 * k * rr.min())
    assert np.allclose(d, d.T, rtol=0, atol=1e-14 * np.abs(d).max())   # reciprocity


def test_adjoint_dot_product(water):
    g, (T, A, B, Tr, Ar, Br) = water
    rng = np.random.default_rng(0)
    for f in (250e3, 600e3):
        G = born.green(T, A, B, f)
        dl = rng.standard_normal(g.n_pixels) * 1e-8
        dd = rng.standard_normal((g.m, g.m)) + 1j * rng.standard_normal((g.m, g.m))
        lhs = np.real(np.vdot(born.born_forward(G, dl, f, g.h ** 2), dd))
        rhs = np.dot(dl, born.born_adjoint(G, dd, f, g.h ** 2))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_hessian_diagonal_equals_explicit_jtwj(water):
    g, (T, A, B, Tr, Ar, Br) = water
    f = 300e3
    G = born.green(T, A, B, f)
    rng = np.random.default_rng(1)
    Wt = receiver_mask(g.m).astype(float) * (rng.uniform(size=(g.m, g.m)) > 0.1)
    Hd = born.hessian_diag(G, Wt, f, g.h ** 2)
    cols = rng.choice(np.flatnonzero(np.isfinite(T).all(axis=0)), 12, replace=False)
    for x in cols:
        ex = np.zeros(g.n_pixels)
        ex[x] = 1.0
        jc = born.born_forward(G, ex, f, g.h ** 2)
        ref = np.sum(Wt * (jc.real ** 2 + jc.imag ** 2))
        assert abs(Hd[x] - ref) <= 1e-12 * ref
    # the explicit J^T W J has this diagonal too (on a handful of pixels)
    Jm = born.jacobian(G[:, cols], f, g.h ** 2)
    H = np.real(Jm.conj().T @ (Wt.reshape(-1, 1) * Jm))
    assert np.allclose(np.diag(H), Hd[cols], rtol=1e-12, atol=0)


def test_brute_force_tiny_loops():
    """Pure-Python loops over (e, r, x) on a tiny problem reproduce the
    vectorised forward and adjoint operators (transposes, conjugations)."""
    rng = np.random.default_rng(5)
    m, n = 4, 64
    G = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    dl = rng.standard_normal(n)
    dd = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    for f in (2e5, 2.5e5):
        om2 = (2 * math.pi * f) ** 2
        dA = 0.25e-6
        fwd = np.zeros((m, m), complex)
        for e in range(m):
            for r in range(m):
                acc = 0j
                for x in range(n):
                    acc += G[e, x] * G[r, x] * dl[x]
                fwd[e, r] = om2 * dA * acc
        adj = np.zeros(n)
        for x in range(n):
            acc = 0.0
            for e in range(m):
                for r in range(m):
                    acc += (np.conj(G[e, x] * G[r, x]) * dd[e, r]).real
            adj[x] = om2 * dA * acc
        assert np.allclose(born.born_forward(G, dl, f, dA), fwd, rtol=1e-13, atol=0)
        assert np.allclose(born.born_adjoint(G, dd, f, dA), adj, rtol=1e-12, atol=1e-30)
