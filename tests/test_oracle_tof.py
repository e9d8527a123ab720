"""Pins for the oracle's bent-ray ToF starting model (CPU only).

References: path lengths of straight rays in a homogeneous medium (the path
weights of a pair sum to c T), Fermat's principle against central
differences of the ray tracer's own first-arrival times (a different code
path: RK4 plus mesh interpolation), exact recovery of a one-pixel slowness
perturbation from consistent linear data, and a decreasing misfit over the
three iterations the paper uses.
"""
import dataclasses

import numpy as np
import pytest

import workload as W
from oracle import rays, tof


def _bump_problem(n=33, m=24, R=12e-3):
    g = W.centred_grid(n, 0.5e-3, m, R, 1500.0)
    X, Y = g.pixel_centres()
    c = 1500.0 + 12.0 * np.exp(-((X - 2e-3) ** 2 + (Y + 1e-3) ** 2) / (2 * (3e-3) ** 2))
    to = W.resolve_trace_opts(g, c, 240)
    return g, c, to


def test_path_weights_sum_to_path_length_in_homogeneous_medium():
    """Straight rays at speed c0 on a grid that covers the ring: the
    bilinear weights sum to one everywhere, so every row of L sums to the
    length of its (two equal) polylines, c0 T."""
    g = W.centred_grid(61, 0.5e-3, 24, 12e-3, 1500.0)
    c = np.full((g.ny, g.nx), 1500.0)
    to = W.resolve_trace_opts(g, c, 240)
    T, used, L = tof.tof_system(g, to, W.InvertOpts(), c, np.zeros((g.m, g.m)))
    assert int(used.sum()) == g.m * (int(0.75 * g.m) + 1)
    rows = np.asarray(L.sum(axis=1)).reshape(g.m, g.m)
    ok = used
    assert np.max(np.abs(rows[ok] / (1500.0 * T[ok]) - 1.0)) <= 1e-12
    assert L.data.min() >= 0.0
    # the chords: c0 T exceeds the straight distance only by the wavefront sag
    pos = g.element_positions()
    d = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
    assert np.all(np.abs(1500.0 * T[ok] / d[ok] - 1.0) <= 1e-4)


@pytest.mark.parametrize("dtau_scale,tol", [(1.0, 1.5e-2), (0.25, 5e-3)])
def test_fermat_linearisation_matches_central_differences(dtau_scale, tol):
    """dT = L ds (Fermat) against (T(s + ds) - T(s - ds)) / 2 from the
    tracer, for a smooth off-centre slowness bump; the discretisation error
    shrinks with the time step."""
    g, c, to = _bump_problem()
    to = dataclasses.replace(to, dtau=to.dtau * dtau_scale)
    X, Y = g.pixel_centres()
    ds = 2e-5 * np.exp(-((X + 1.5e-3) ** 2 + (Y - 2e-3) ** 2) / (2 * (2.5e-3) ** 2))
    s = 1.0 / c
    _, used, L = tof.tof_system(g, to, W.InvertOpts(), c, np.zeros((g.m, g.m)))
    Tp = np.stack([rays.rx_links(g, to, s + ds, None, e)["T"] for e in range(g.m)])
    Tn = np.stack([rays.rx_links(g, to, s - ds, None, e)["T"] for e in range(g.m)])
    fd = (0.5 * (Tp - Tn)).reshape(-1)[used.reshape(-1)]
    lin = (L @ ds.reshape(-1))[used.reshape(-1)]
    assert np.linalg.norm(fd - lin) / np.linalg.norm(lin) <= tol


def test_one_pixel_support_recovers_slowness_perturbation_exactly():
    g, c, to = _bump_problem()
    g = dataclasses.replace(g, support_margin=g.ring_radius - 0.25 * g.h)
    T, used, L = tof.tof_system(g, to, W.InvertOpts(), c, np.zeros((g.m, g.m)))
    ic = (g.ny // 2) * g.nx + g.nx // 2
    a = 3e-7
    e_c = np.zeros(g.n_pixels)
    e_c[ic] = a
    T_meas = np.where(used, T + (L @ e_c).reshape(g.m, g.m), np.nan)
    parts = tof.tof_step(g, to, W.InvertOpts(), c, T_meas, return_parts=True)
    assert int(parts["support"].sum()) == 1 and parts["support"][ic]
    # dT = T_meas - T cancels ~5 digits of T: exact to rounding of that
    assert abs(parts["beta"] * parts["direction"][ic] - a) <= 1e-10 * a
    s_c = 1.0 / c.reshape(-1)[ic]
    assert abs(1.0 / parts["c_new"].reshape(-1)[ic] - (s_c + a)) <= 1e-10 * a
    others = np.ones(g.n_pixels, bool)
    others[ic] = False
    assert np.array_equal(parts["c_new"].reshape(-1)[others], c.reshape(-1)[others])


def test_three_iterations_reduce_the_misfit():
    """ToFs traced in the bump model, start in water: the rms ToF residual
    falls at every iteration and the model error to about a quarter."""
    g, c_true, to = _bump_problem()
    T_meas = np.stack([rays.rx_links(g, to, 1.0 / c_true, None, e)["T"] for e in range(g.m)])
    c0 = np.full_like(c_true, 1500.0)
    c, hist = c0, []
    errs = [np.linalg.norm(c0 - c_true)]
    for _ in range(3):
        c, rms = tof.tof_step(g, to, W.InvertOpts(), c, T_meas)
        hist.append(rms)
        errs.append(np.linalg.norm(c - c_true))
    _, rms_after = tof.tof_step(g, to, W.InvertOpts(), c, T_meas)
    hist.append(rms_after)
    assert all(b < a for a, b in zip(hist, hist[1:])), hist
    assert errs[1] < errs[0] and errs[3] < 0.35 * errs[0], errs
    assert hist[-1] < 0.5 * hist[0]
