"""Pins for the full-wave (Helmholtz FD) data generator, CPU only.

References: the exact 2-D Green's function (i/4) H0(k r) (scipy's Hankel
function) in water, with and without absorption (complex wavenumber);
second-order convergence under grid refinement; reciprocity.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel1

import workload as W
from workload import fullwave as F


def _geom():
    return W.centred_grid(64, 0.5e-3, 32, 14e-3, 1500.0)


def _exact(g, f, alpha=0.0):
    pos = g.element_positions()
    d = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
    k = 2 * math.pi * f / g.c_background + 1j * alpha * (f * 1e-6)
    ex = 0.25j * hankel1(0, k * np.where(d > 0, d, 1.0))
    return d, np.where(d > 0, ex, 0.0)


@pytest.mark.parametrize("alpha", [0.0, 5.0])
def test_homogeneous_medium_matches_hankel_and_converges(alpha):
    g = _geom()
    c = np.full((g.ny, g.nx), 1500.0)
    al = np.full((g.ny, g.nx), alpha)
    f = 250e3
    d, ex = _exact(g, f, alpha)
    sel = d > 10e-3
    errs = []
    for refine in (2, 4):
        p = F.helmholtz_data(g, c, al, [f], refine=refine)[0]
        errs.append(float(np.max(np.abs(p - ex)[sel] / np.abs(ex[sel]))))
    # second order: halving the FD spacing divides the error by about 4
    assert errs[1] <= 0.03
    assert errs[0] / errs[1] >= 3.0


def test_data_are_reciprocal_in_a_heterogeneous_medium():
    g = _geom()
    c, al = W.ellipse_phantom(g, 5, centre_radius=8e-3)
    p = F.helmholtz_data(g, c, al, [2.2e5, 2.9e5], refine=2)
    for k in range(2):
        assert np.max(np.abs(p[k] - p[k].T)) <= 1e-10 * np.max(np.abs(p[k]))
        assert np.all(p[k][np.arange(g.m), np.arange(g.m)] == 0)
