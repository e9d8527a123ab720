"""GPU parity of the CG solution of the linear subproblem (the library's
rb_invert_frequency_set_cg) against the FP64 oracle's preconditioned CG.

Tolerances: the update and the per-iteration step lengths alpha_i within
rel 1e-5 (f64 and f32 contractions; the remaining difference comes from the
ray tables, |dT| <= 1e-9 s, measured 3e-7 for the update over six
iterations); 16-bit contractions within 5e-3 (bf16) and 1e-3 (f16) of the
FP64 oracle over three iterations (measured 8.7e-4 and 1.1e-4); the first CG
iterate equals the single step up to rounding.
"""
import dataclasses
import sys

import numpy as np
import pytest

import workload as W
from oracle import invert

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


def _pm(p_meas):
    return _t(np.stack([p_meas.real, p_meas.imag], -1))


TOL = {"f64": 1e-5, "f32": 1e-5}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cg_matches_oracle(rb, dtype):
    p = W.small_ring()
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    n_iter = 6
    _say(f"cg ring64_grid128 dtype={dtype} n_iter={n_iter}")
    ref = invert.invert_frequency_set_cg(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0], n_iter,
                                         return_parts=True)
    c_in = _t(p.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    l2, alphas, rzs = rb.invert_frequency_set_cg(p.geom, topts, p.inv, dtype, c_in, _t(p.alpha0.reshape(-1)),
                                                 f, _pm(p.p_meas[0]), n_iter, c_out)
    dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - p.c_start.reshape(-1)
    ea, er, ed = _rel(alphas, ref["alpha"]), _rel(rzs, ref["rz"]), _rel(dc_g, dc_o)
    _say(f"  rel alpha {ea:.2e}  rel r.z {er:.2e}  rel dc {ed:.2e}  norms {l2:.4f} vs {ref['dc_l2']:.4f}")
    tol = TOL[dtype]
    assert np.all(np.asarray(alphas) > 0)
    assert ea <= tol and er <= tol and ed <= tol
    assert abs(l2 - ref["dc_l2"]) <= tol * ref["dc_l2"]
    assert np.array_equal(c_in.cpu().numpy(), p.c_start.reshape(-1))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cg_first_iterate_is_the_single_step(rb, dtype):
    p = W.small_ring()
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    _say(f"cg n_iter=1 vs single step, ring64_grid128 dtype={dtype}")
    c_in = _t(p.c_start.reshape(-1))
    a = torch.empty_like(c_in)
    b = torch.empty_like(c_in)
    al = _t(p.alpha0.reshape(-1))
    l2a = rb.invert_frequency_set(p.geom, topts, p.inv, dtype, c_in, al, f, _pm(p.p_meas[0]), a)
    l2b, alphas, _ = rb.invert_frequency_set_cg(p.geom, topts, p.inv, dtype, c_in, al, f, _pm(p.p_meas[0]), 1, b)
    da = a.cpu().numpy() - p.c_start.reshape(-1)
    db = b.cpu().numpy() - p.c_start.reshape(-1)
    tol = 1e-10 if dtype == "f64" else 1e-4
    assert _rel(db, da) <= tol
    assert abs(l2a - l2b) <= tol * l2a
    assert len(alphas) == 1 and alphas[0] > 0


def test_cg_empty_support_takes_no_step(rb):
    """Support margin >= R: no pixel is solved for, r.z = 0 at the start and
    every step is zero; the model is returned unchanged (oracle agrees)."""
    p = W.small_ring()
    g = dataclasses.replace(p.geom, support_margin=p.geom.ring_radius)
    topts = W.resolve_trace_opts(g, p.c_start, 360)
    f = p.freq_sets[0]
    ref = invert.invert_frequency_set_cg(g, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0], 3,
                                         return_parts=True)
    assert np.all(ref["alpha"] == 0) and np.all(ref["rz"] == 0)
    _say("cg empty support f32")
    c_in = _t(p.c_start.reshape(-1))
    c_out = _t(np.zeros(g.n_pixels))
    l2, alphas, rzs = rb.invert_frequency_set_cg(g, topts, p.inv, "f32", c_in, _t(p.alpha0.reshape(-1)), f,
                                                 _pm(p.p_meas[0]), 3, c_out)
    assert l2 == 0.0 and alphas == [0.0] * 3 and rzs == [0.0] * 3
    assert np.array_equal(c_out.cpu().numpy(), p.c_start.reshape(-1))


def test_cg_ragged_in_place_and_repeatable(rb):
    p = W.custom(47, 0.5e-3, 24, 11e-3, 150, [[2.4e5, 3.1e5, 3.7e5]], seed=13)
    topts = W.resolve_trace_opts(p.geom, p.c_start, 150)
    f = p.freq_sets[0]
    ref = invert.invert_frequency_set_cg(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0], 4,
                                         return_parts=True)
    _say("cg ragged 47x47 m=24 f32 in place, twice")
    outs = []
    ws = torch.empty(rb.invert_cg_workspace_bytes(p.geom, topts, len(f), "f32"), dtype=torch.uint8, device=DEV)
    for _ in range(2):
        c = _t(p.c_start.reshape(-1))
        l2, alphas, _ = rb.invert_frequency_set_cg(p.geom, topts, p.inv, "f32", c, _t(p.alpha0.reshape(-1)), f,
                                                   _pm(p.p_meas[0]), 4, c, ws=ws)
        outs.append((c.cpu().numpy(), l2, alphas))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]
    dc_g = outs[0][0] - p.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - p.c_start.reshape(-1)
    ed, ea = _rel(dc_g, dc_o), _rel(outs[0][2], ref["alpha"])
    _say(f"  rel dc {ed:.2e}  rel alpha {ea:.2e}")
    assert ed <= 1e-4 and ea <= 1e-4


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_cg_16bit_against_fp64_oracle(rb, dtype):
    """Precision form of CG: 16-bit contractions (FP32 accumulation, FP64
    phase) over three iterations against the FP64 oracle."""
    p = W.small_ring()
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    ref = invert.invert_frequency_set_cg(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0], 3,
                                         return_parts=True)
    _say(f"cg ring64_grid128 dtype={dtype} n_iter=3")
    c_in = _t(p.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    l2, alphas, _ = rb.invert_frequency_set_cg(p.geom, topts, p.inv, dtype, c_in, _t(p.alpha0.reshape(-1)), f,
                                               _pm(p.p_meas[0]), 3, c_out)
    dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - p.c_start.reshape(-1)
    ed, ea = _rel(dc_g, dc_o), _rel(alphas, ref["alpha"])
    _say(f"  rel dc {ed:.2e}  rel alpha {ea:.2e}")
    tol = {"bf16": 5e-3, "f16": 1e-3}[dtype]
    assert ed <= tol and ea <= tol
