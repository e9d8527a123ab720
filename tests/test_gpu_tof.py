"""GPU parity of the bent-ray ToF starting model (rb_tof_invert) against the
FP64 oracle (oracle.tof), iteration by iteration.

Measured ToFs are the straight-chord stand-in of the true phantom; the start
is water.  Tolerances: rms residual, beta and the model change within rel
1e-6 (the ray nodes differ from the oracle's at the ulp level and the
back-projection sums with floating-point atomics in no fixed order).
"""
import sys

import numpy as np
import pytest

import workload as W
from oracle import invert as invert_mod
from oracle import tof

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_16633_amd as rbm
    rbm.lib()
    return rbm


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _oracle(geom, topts, inv, c0, T_meas, n_iter):
    c, rms, beta = c0, [], []
    for _ in range(n_iter):
        parts = tof.tof_step(geom, topts, inv, c, T_meas, return_parts=True)
        c = parts["c_new"]
        rms.append(parts["rms"])
        beta.append(parts["beta"])
    return c, rms, beta


def _check(rb, geom, topts, inv, c0, T_meas, n_iter, tol=1e-6):
    c_o, rms_o, beta_o = _oracle(geom, topts, inv, c0, T_meas, n_iter)
    c_in = _t(c0.reshape(-1))
    c_out = torch.empty_like(c_in)
    rms_g, beta_g = rb.tof_invert(geom, topts, inv, c_in, _t(T_meas), n_iter, c_out)
    dc_g = c_out.cpu().numpy() - c0.reshape(-1)
    dc_o = c_o.reshape(-1) - c0.reshape(-1)
    er, eb, ed = _rel(rms_g, rms_o), _rel(beta_g, beta_o), _rel(dc_g, dc_o)
    _say(f"  rms {rms_g} vs {rms_o}; rel rms {er:.2e} beta {eb:.2e} dc {ed:.2e}")
    assert er <= tol and eb <= tol and ed <= tol
    assert np.array_equal(c_in.cpu().numpy(), c0.reshape(-1))
    return rms_g


def test_tof_three_iterations_match_oracle(rb):
    p = W.small_ring()
    T_meas = W.straight_ray_tof(p.geom, p.c_true)
    c0 = np.full_like(p.c_true, p.geom.c_background)
    topts = W.resolve_trace_opts(p.geom, c0, 360)
    _say("tof ring64_grid128, 3 iterations from water")
    rms = _check(rb, p.geom, topts, p.inv, c0, T_meas, 3)
    assert rms[2] < rms[0]


def test_tof_ragged_grid_with_unmeasured_pairs(rb):
    p = W.custom(47, 0.5e-3, 24, 11e-3, 150, [[2.4e5]], seed=13, with_data=False)
    T_meas = W.straight_ray_tof(p.geom, p.c_true)
    rng = np.random.default_rng(3)
    T_meas[rng.random(T_meas.shape) < 0.3] = np.nan
    c0 = np.full_like(p.c_true, p.geom.c_background)
    topts = W.resolve_trace_opts(p.geom, c0, 150)
    _say("tof ragged 47x47 m=24, 30% of the pairs unmeasured, 2 iterations")
    _check(rb, p.geom, topts, p.inv, c0, T_meas, 2)


def test_tof_in_place(rb):
    p = W.small_ring()
    T_meas = W.straight_ray_tof(p.geom, p.c_true)
    c0 = np.full_like(p.c_true, p.geom.c_background)
    topts = W.resolve_trace_opts(p.geom, c0, 360)
    _say("tof ring64_grid128 in place, 1 iteration")
    a = _t(c0.reshape(-1))
    b = torch.empty_like(a)
    rb.tof_invert(p.geom, topts, p.inv, a, _t(T_meas), 1, b)
    b2 = torch.empty_like(a)
    rb.tof_invert(p.geom, topts, p.inv, a, _t(T_meas), 1, b2)
    rb.tof_invert(p.geom, topts, p.inv, a, _t(T_meas), 1, a)
    # the back-projection sums in fixed point: repeated and in-place calls are bitwise equal
    assert torch.equal(b, b2)
    assert torch.equal(a, b)


def test_tof_no_measured_pairs_leaves_model(rb):
    """Every ToF unmeasured: no used pair, empty support, zero step."""
    p = W.small_ring(with_data=False)
    c0 = np.full_like(p.c_true, p.geom.c_background)
    topts = W.resolve_trace_opts(p.geom, c0, 360)
    T_meas = np.full((p.geom.m, p.geom.m), np.nan)
    _say("tof with no measured pair")
    c_in = _t(c0.reshape(-1))
    c_out = _t(np.zeros(p.geom.n_pixels))
    rms, beta = rb.tof_invert(p.geom, topts, p.inv, c_in, _t(T_meas), 2, c_out)
    assert rms == [0.0, 0.0] and beta == [0.0, 0.0]
    assert np.array_equal(c_out.cpu().numpy(), c0.reshape(-1))


def test_tof_refuses_nonpositive_slowness(rb):
    """ToFs a tenth of the modelled ones ask for a negative slowness: the
    oracle raises, the library returns RB_ENUMERIC and leaves c_out alone."""
    p = W.small_ring(with_data=False)
    c0 = np.full_like(p.c_true, p.geom.c_background)
    topts = W.resolve_trace_opts(p.geom, c0, 360)
    T_meas = 0.1 * W.straight_ray_tof(p.geom, c0)
    with pytest.raises(invert_mod.NumericError):
        tof.tof_step(p.geom, topts, p.inv, c0, T_meas)
    _say("tof numeric refusal")
    c_in = _t(c0.reshape(-1))
    c_out = _t(np.full(p.geom.n_pixels, 7.0))
    with pytest.raises(rb.NumericError):
        rb.tof_invert(p.geom, topts, p.inv, c_in, _t(T_meas), 1, c_out)
    assert np.all(c_out.cpu().numpy() == 7.0)
