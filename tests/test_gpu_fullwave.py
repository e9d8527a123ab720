"""The step and the CG solve on full-wave data (Helmholtz FD, no inverse
crime) against the oracle on the same data.  The data come from a model
other than the inversion's, so residuals, outlier choices and the update
differ from the straight-ray stand-in's; parity bounds as for the other
inputs (rel-L2 of the update 1e-4 for the step, 1e-5 for CG)."""
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


@pytest.fixture(scope="module")
def prob():
    return W.small_ring_fullwave(refine=2)


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_step_on_fullwave_data(rb, prob, dtype):
    p = prob
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    ref = invert.invert_frequency_set(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0])
    _say(f"step on full-wave data ring64_grid128 dtype={dtype}")
    c_in = _t(p.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    pm = _t(np.stack([p.p_meas[0].real, p.p_meas[0].imag], -1))
    l2 = rb.invert_frequency_set(p.geom, topts, p.inv, dtype, c_in, _t(p.alpha0.reshape(-1)), f, pm, c_out)
    dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref[0].reshape(-1) - p.c_start.reshape(-1)
    _say(f"  rel dc {_rel(dc_g, dc_o):.2e}  norms {l2:.4f} vs {ref[1]:.4f}")
    assert _rel(dc_g, dc_o) <= 1e-4
    assert abs(l2 - ref[1]) <= 1e-4 * ref[1]


def test_cg_on_fullwave_data(rb, prob):
    p = prob
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    ref = invert.invert_frequency_set_cg(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0], 4,
                                         return_parts=True)
    _say("cg on full-wave data ring64_grid128 f32, 4 iterations")
    c_in = _t(p.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    pm = _t(np.stack([p.p_meas[0].real, p.p_meas[0].imag], -1))
    l2, alphas, _ = rb.invert_frequency_set_cg(p.geom, topts, p.inv, "f32", c_in, _t(p.alpha0.reshape(-1)), f, pm,
                                               4, c_out)
    dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - p.c_start.reshape(-1)
    _say(f"  rel dc {_rel(dc_g, dc_o):.2e}  rel alpha {_rel(np.asarray(alphas), ref['alpha']):.2e}")
    assert _rel(dc_g, dc_o) <= 1e-5
    assert _rel(np.asarray(alphas), ref["alpha"]) <= 1e-5
