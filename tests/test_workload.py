"""The seeded input generators are deterministic and have the stated shapes."""
import numpy as np

import workload as W


def test_small_ring_is_seeded_and_shaped():
    a = W.small_ring()
    b = W.small_ring()
    assert a.geom.n_pixels == 128 * 128 and a.geom.m == 64
    assert np.array_equal(a.c_true, b.c_true) and np.array_equal(a.p_meas[0], b.p_meas[0])
    assert a.p_meas[0].shape == (2, 64, 64)
    assert np.all(a.p_meas[0][:, np.arange(64), np.arange(64)] == 0)
    assert 1440 < a.c_true.min() and a.c_true.max() < 1560
    c = W.small_ring(seed=1234, with_data=False)
    assert not np.array_equal(a.c_true, c.c_true)


def test_breast_phantom_ranges():
    g = W.centred_grid(120, 2e-3, 32, 110e-3, 1500.0)
    c, al = W.breast_phantom(g, 5)
    X, Y = g.pixel_centres()
    inside = np.hypot(X, Y) <= 0.8 * 110e-3
    assert np.all(c[~inside] == 1500.0)
    assert 1380 < c[inside].min() and c[inside].max() < 1650
    assert np.all(al[inside] > 0) and np.all(al[~inside] == 0)


def test_trace_options_resolution():
    p = W.small_ring(with_data=False)
    to = W.resolve_trace_opts(p.geom, p.c_start, 360)
    assert to.dtau == p.geom.h / (2.0 * 1500.0 * 1.1)
    assert to.j_min == 0.25 * p.geom.h


def test_serving_stream_mix():
    jobs = W.serving_stream(200)
    assert len(jobs) == 200
    t = [j["arrival_s"] for j in jobs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert 300 < t[-1] < 500            # ~ 200 / 0.5 s
    cls = np.bincount([j["size_class"] for j in jobs], minlength=3)
    assert cls[0] > cls[1] > cls[2] > 0
