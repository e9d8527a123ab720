"""Pins for the oracle's data weights and single step (CPU only).

References: the paper's printed parameters (golden fixture), brute-force
selection, exact recovery of a point perturbation (the single step inverts
the weighted Hessian exactly when it is 1x1), numpy's least-squares solver
for a one-pixel problem, and optimality of the step length.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import workload as W
from oracle import born, invert, rays

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


@pytest.mark.parametrize("case", ["in_vitro", "in_vivo_cyst", "in_vivo_malignancy"])
def test_receiver_mask_counts_paper_geometries(case):
    """Opposite 75 % of the ring: 0.75 m + 1 receivers per emitter, symmetric."""
    P = GOLD[case]
    m = P["elements"]
    msk = invert.receiver_mask(m, P["receiver_fraction"])
    assert np.all(msk.sum(axis=1) == int(0.75 * m) + 1)
    assert np.array_equal(msk, msk.T)
    assert not msk[np.arange(m), np.arange(m)].any()
    # the kept receivers are the far ones: no kept neighbour closer than a kept-out one
    e = 0
    d = np.minimum(np.arange(m), m - np.arange(m))
    assert d[msk[e]].min() > d[~msk[e]].max() - 1


def test_outlier_count_and_brute_force():
    m = 64
    rng = np.random.default_rng(11)
    p = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    p[3, 40] = p[40, 3] = 7.0       # an exact tie among the largest
    msk = invert.receiver_mask(m, 0.75)
    w = invert.outlier_weights(p, msk, GOLD["in_vitro"]["outlier_fraction"])
    n_valid = int(msk.sum())
    k = int(math.floor(0.01 * n_valid))
    assert k == 31
    assert int((msk & (w == 0)).sum()) == k
    assert np.all(w[~msk] == 0)
    # brute force: sort (magnitude desc, flat index asc) in plain Python
    items = []
    for e in range(m):
        for r in range(m):
            if msk[e, r]:
                z = complex(p[e, r])
                items.append((-(z.real * z.real + z.imag * z.imag), e * m + r))
    items.sort()
    zeroed = {idx for _, idx in items[:k]}
    got = {int(i) for i in np.flatnonzero((w == 0).reshape(-1) & msk.reshape(-1))}
    assert got == zeroed
    assert 3 * m + 40 in got and 40 * m + 3 in got


def _tiny_problem(n=33, m=24, R=12e-3, margin=None):
    g = W.centred_grid(n, 0.5e-3, m, R, 1500.0)
    if margin is not None:
        g = dataclasses.replace(g, support_margin=margin)
    X, Y = g.pixel_centres()
    c = 1500.0 + 12.0 * np.exp(-((X - 2e-3) ** 2 + (Y + 1e-3) ** 2) / (2 * (3e-3) ** 2))
    al = np.full_like(c, 2.0)
    to = W.resolve_trace_opts(g, c, 240)
    return g, c, al, to


def _model_data(g, to, c, al, freqs):
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / c, al)
    Gs = [born.green(T, A, B, f) for f in freqs]
    ps = [born.green(Tr, Ar, Br, f) for f in freqs]
    return Gs, ps


def test_single_pixel_support_recovers_point_perturbation_exactly():
    """With S = {centre} and data p = p(c) + J (a e_c), the diagonal weight is
    the exact inverse of the 1x1 weighted Hessian: delta(centre) = a."""
    g, c, al, to = _tiny_problem(margin=12e-3 - 0.5 * 0.5e-3)
    freqs = np.array([250e3, 320e3])
    Gs, ps = _model_data(g, to, c, al, freqs)
    ic = (g.ny // 2) * g.nx + g.nx // 2
    a = 3e-9
    e_c = np.zeros(g.n_pixels)
    e_c[ic] = a
    p_meas = np.stack([ps[k] + born.born_forward(Gs[k], e_c, f, g.h ** 2) for k, f in enumerate(freqs)])
    parts = invert.invert_frequency_set(g, to, W.InvertOpts(), c, al, freqs, p_meas, return_parts=True)
    assert int(parts["support"].sum()) == 1 and parts["support"][ic]
    assert abs(parts["delta"][ic] - a) <= 1e-12 * a
    s = 1.0 / c.reshape(-1)[ic]
    assert abs(parts["c_new"].reshape(-1)[ic] - 1.0 / math.sqrt(s * s + a)) < 1e-9
    others = np.ones(g.n_pixels, bool)
    others[ic] = False
    assert np.array_equal(parts["c_new"].reshape(-1)[others], c.reshape(-1)[others])


def test_one_pixel_grid_matches_weighted_least_squares():
    """A 1x1 grid: delta is the weighted least-squares solution of the
    stacked real system sqrt(W)[Re J; Im J] delta = sqrt(W)[Re D; Im D]."""
    g = W.Geometry(nx=1, ny=1, h=0.5e-3, x0=0.0, y0=0.0, m=20, ring_radius=10e-3,
                   support_margin=5e-3, c_background=1500.0)
    c = np.array([[1510.0]])
    al = np.array([[1.0]])
    to = W.resolve_trace_opts(g, c, 180)
    freqs = np.array([300e3, 350e3, 410e3])
    rng = np.random.default_rng(2)
    Gs, ps = _model_data(g, to, c, al, freqs)
    p_meas = np.stack([ps[k] * (1 + 0.05 * (rng.standard_normal(ps[k].shape)
                                           + 1j * rng.standard_normal(ps[k].shape)))
                       for k in range(3)])
    parts = invert.invert_frequency_set(g, to, W.InvertOpts(eps=0.0), c, al, freqs, p_meas,
                                        return_parts=True)
    rows, rhs = [], []
    for k, f in enumerate(freqs):
        col = born.born_forward(Gs[k], np.ones(1), f, g.h ** 2).reshape(-1)
        sw = np.sqrt(parts["W"][k].reshape(-1))
        Dk = parts["D"][k].reshape(-1)
        rows += [sw * col.real, sw * col.imag]
        rhs += [sw * Dk.real, sw * Dk.imag]
    Amat = np.concatenate(rows)[:, None]
    bvec = np.concatenate(rhs)
    sol = np.linalg.lstsq(Amat, bvec, rcond=None)[0][0]
    assert abs(parts["delta"][0] - sol) <= 1e-10 * abs(sol)


def test_step_length_minimises_linearised_objective():
    g, c, al, to = _tiny_problem()
    freqs = np.array([220e3, 260e3])
    p = W.custom(33, 0.5e-3, 24, 12e-3, 240, [list(freqs)], seed=3)
    parts = invert.invert_frequency_set(g, to, W.InvertOpts(), c, al, freqs, p.p_meas[0],
                                        return_parts=True)
    v, beta = parts["direction"], parts["beta"]
    assert beta != 0.0

    def phi(b):
        return sum(float(np.sum(parts["W"][k] * np.abs(parts["D"][k] - b * parts["Jv"][k]) ** 2))
                   for k in range(len(freqs)))
    assert phi(beta) < phi(0.0)
    assert phi(beta) <= phi(beta * 1.01) and phi(beta) <= phi(beta * 0.99)


def test_nonpositive_slowness_squared_is_an_error():
    g, c, al, to = _tiny_problem(margin=12e-3 - 0.5 * 0.5e-3)
    freqs = np.array([250e3])
    Gs, ps = _model_data(g, to, c, al, freqs)
    ic = (g.ny // 2) * g.nx + g.nx // 2
    s2 = 1.0 / c.reshape(-1)[ic] ** 2
    e_c = np.zeros(g.n_pixels)
    e_c[ic] = -2.0 * s2
    p_meas = np.stack([ps[0] + born.born_forward(Gs[0], e_c, 250e3, g.h ** 2)])
    with pytest.raises(invert.NumericError):
        invert.invert_frequency_set(g, to, W.InvertOpts(), c, al, freqs, p_meas)


def test_sweep_is_deterministic_and_resumable():
    p = W.custom(41, 0.5e-3, 20, 12e-3, 180, [[200e3, 240e3], [280e3, 330e3]], seed=9)
    to = W.resolve_trace_opts(p.geom, p.c_start, 180)
    c1, h1 = invert.sweep(p.geom, to, p.inv, p.c_start, p.alpha0, p.freq_sets, p.p_meas)
    c2, h2 = invert.sweep(p.geom, to, p.inv, p.c_start, p.alpha0, p.freq_sets, p.p_meas)
    assert np.array_equal(c1, c2) and h1 == h2
    # resume from the checkpoint after set 0
    ck, _ = invert.invert_frequency_set(p.geom, to, p.inv, p.c_start, p.alpha0, p.freq_sets[0], p.p_meas[0])
    c3, h3 = invert.sweep(p.geom, to, p.inv, ck, p.alpha0, p.freq_sets[1:], p.p_meas[1:])
    assert np.array_equal(c1, c3) and h1[1:] == h3
    assert all(np.isfinite(h1)) and h1[0] > 0


def _dense_hessian(L, freqs):
    """Re(J^H W J) on the ok pixels from the explicit Jacobian."""
    ok = L["ok"]
    n = int(ok.sum())
    H = np.zeros((n, n))
    for k, f in enumerate(freqs):
        J = born.jacobian(L["G"][k], f, L["dA"])[:, ok]
        w = L["W"][k].reshape(-1)
        H += np.real(J.conj().T @ (w[:, None] * J))
    return H


def test_cg_first_iterate_is_the_single_step():
    """Jacobi-preconditioned CG from zero: its first iterate is beta v."""
    g, c, al, to = _tiny_problem()
    freqs = np.array([220e3, 260e3])
    p = W.custom(33, 0.5e-3, 24, 12e-3, 240, [list(freqs)], seed=3)
    one = invert.invert_frequency_set(g, to, W.InvertOpts(), c, al, freqs, p.p_meas[0], return_parts=True)
    cg = invert.invert_frequency_set_cg(g, to, W.InvertOpts(), c, al, freqs, p.p_meas[0], 1,
                                        return_parts=True)
    scale = np.max(np.abs(one["delta"]))
    assert scale > 0
    assert np.max(np.abs(cg["delta"] - one["delta"])) <= 1e-12 * scale
    assert abs(cg["alpha"][0] - one["beta"]) <= 1e-12 * abs(one["beta"])


@pytest.mark.parametrize("n_iter", [1, 2, 3, 5])
def test_cg_iterates_minimise_quadratic_over_krylov_subspace(n_iter):
    """The k-th preconditioned CG iterate minimises 1/2 x.Hx - g.x over the
    Krylov space span{M^-1 g, (M^-1 H) M^-1 g, ...} of dimension k (Galerkin
    solution from an explicit basis and the explicit Jacobian's Hessian)."""
    g, c, al, to = _tiny_problem()
    freqs = np.array([220e3, 260e3])
    p = W.custom(33, 0.5e-3, 24, 12e-3, 240, [list(freqs)], seed=3)
    cg = invert.invert_frequency_set_cg(g, to, W.InvertOpts(), c, al, freqs, p.p_meas[0], n_iter,
                                        return_parts=True)
    ok = cg["ok"]
    assert int(ok.sum()) > 100
    H = _dense_hessian(cg, freqs)
    rhs = cg["grad"][ok]
    den = cg["den"][ok]
    basis = [rhs / den]
    for _ in range(1, n_iter):
        basis.append((H @ basis[-1]) / den)
    Q, _ = np.linalg.qr(np.stack(basis, axis=1))
    x_star = Q @ np.linalg.solve(Q.T @ H @ Q, Q.T @ rhs)
    x = cg["delta"][ok]
    assert np.max(np.abs(x - x_star)) <= 1e-10 * np.max(np.abs(x_star))
    assert np.all(cg["delta"][~ok] == 0.0)
    assert np.all(cg["alpha"] > 0) and np.all(cg["rz"] > 0)


def test_cg_recovers_perturbation_on_small_support():
    """Consistent Born data p(c) + J d on a 9-pixel support, no outliers: CG
    on the normal equations returns d (finite termination, run to 2n)."""
    rs = 0.75e-3
    g, c, al, to = _tiny_problem(margin=12e-3 - rs)
    freqs = np.array([250e3, 320e3])
    Gs, ps = _model_data(g, to, c, al, freqs)
    T = rays.tables(g, to, 1.0 / c, al)[0]
    S = invert.support(g, T)
    n = int(S.sum())
    assert n == 9
    rng = np.random.default_rng(5)
    d = np.zeros(g.n_pixels)
    d[S] = 3e-9 * (1.0 + rng.standard_normal(n))
    p_meas = np.stack([ps[k] + born.born_forward(Gs[k], d, f, g.h ** 2) for k, f in enumerate(freqs)])
    cg = invert.invert_frequency_set_cg(g, to, W.InvertOpts(outlier_fraction=0.0), c, al, freqs, p_meas,
                                        2 * n, return_parts=True)
    assert np.max(np.abs(cg["delta"] - d)) <= 1e-9 * np.max(np.abs(d))


def test_cg_zero_residual_stops_with_zero_steps():
    """Data equal to the model's own: grad = 0, so r.z = 0 and every step is 0."""
    g, c, al, to = _tiny_problem()
    freqs = np.array([250e3])
    _, ps = _model_data(g, to, c, al, freqs)
    cg = invert.invert_frequency_set_cg(g, to, W.InvertOpts(), c, al, freqs, np.stack(ps), 4,
                                        return_parts=True)
    assert np.all(cg["alpha"] == 0.0) and cg["rz"][0] == 0.0
    assert cg["dc_l2"] == 0.0 and np.array_equal(cg["c_new"], c)


def test_asymptotic_direction_recovers_a_point_scatterer_at_its_pixel():
    """Born data of one pixel's perturbation a, no outliers: every selected
    pair's normalised estimate at that pixel is exactly a, so the direction
    there is a (before the step length)."""
    g, c, al, to = _tiny_problem()
    freqs = np.array([250e3, 320e3])
    Gs, ps = _model_data(g, to, c, al, freqs)
    ic = (g.ny // 2) * g.nx + g.nx // 2 + 3
    a = 4e-9
    e_c = np.zeros(g.n_pixels)
    e_c[ic] = a
    p_meas = np.stack([ps[k] + born.born_forward(Gs[k], e_c, f, g.h ** 2) for k, f in enumerate(freqs)])
    parts = invert.invert_frequency_set_asymptotic(g, to, W.InvertOpts(outlier_fraction=0.0), c, al, freqs,
                                                   p_meas, return_parts=True)
    assert parts["support"][ic]
    assert abs(parts["direction"][ic] - a) <= 1e-10 * a
    assert parts["beta"] > 0


def test_asymptotic_direction_matches_brute_force_loops():
    """g_A and n_A by explicit loops over pairs on a tiny problem."""
    g = W.centred_grid(9, 0.5e-3, 8, 4e-3, 1500.0)
    c = np.full((g.ny, g.nx), 1500.0)
    c[4, 4] = 1510.0
    to = W.resolve_trace_opts(g, c, 60)
    freqs = np.array([300e3])
    rng = np.random.default_rng(4)
    p_meas = (rng.standard_normal((1, g.m, g.m)) + 1j * rng.standard_normal((1, g.m, g.m))) * 1e-3
    parts = invert.invert_frequency_set_asymptotic(g, to, W.InvertOpts(outlier_fraction=0.0), c, None, freqs,
                                                   p_meas, return_parts=True)
    G = parts["G"][0]
    Wk, Dk = parts["W"][0], parts["D"][0]
    om2dA = (2 * math.pi * freqs[0]) ** 2 * g.h ** 2
    for x in range(g.n_pixels):
        gs, ns = 0.0, 0.0
        for e in range(g.m):
            for r in range(g.m):
                if Wk[e, r] != 0 and G[e, x] != 0 and G[r, x] != 0:
                    gs += (Wk[e, r] * Dk[e, r] / (om2dA * G[e, x] * G[r, x])).real
                    ns += Wk[e, r]
        assert abs(parts["g_A"][x] - gs) <= 1e-9 * max(1e-30, abs(gs)) + 1e-300
        assert parts["n_A"][x] == ns
