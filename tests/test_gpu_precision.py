"""Precision form: the Born contractions in FP16 and BF16 on MFMA (FP32
accumulation, per-frequency scaling of G and of W.D) with travel times and
phase in FP64, against the FP64 oracle, next to the FP32 path.

The image is the update dc of one linearised frequency set.  Bounds (rel-L2
of dc, max |dc difference|): FP64 1e-6 / 1e-5 m/s (the tracer differs from the
oracle at the ulp level), FP32 1e-4 / 0.01 m/s, FP16 2e-3 / 0.1 m/s,
BF16 1e-2 / 0.5 m/s.  Each case prints its measured error.
"""
import numpy as np
import pytest

import workload as W
from oracle import invert

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BOUNDS = {"f64": (1e-6, 1e-5), "f32": (1e-4, 0.01), "f16": (2e-3, 0.1), "bf16": (1e-2, 0.5)}


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_16633_amd as rbm
    rbm.lib()
    return rbm


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


class _Case:
    def __init__(self, prob, n_rays):
        self.p = prob
        self.topts = W.resolve_trace_opts(prob.geom, prob.c_start, n_rays)
        f = prob.freq_sets[0]
        self.f = f
        self.ref_c, self.ref_l2 = invert.invert_frequency_set(prob.geom, self.topts, prob.inv, prob.c_start,
                                                              prob.alpha0, f, prob.p_meas[0])

    def run(self, rb, dtype):
        p = self.p
        c_in = _t(p.c_start.reshape(-1))
        c_out = torch.empty_like(c_in)
        pm = _t(np.stack([p.p_meas[0].real, p.p_meas[0].imag], -1))
        l2 = rb.invert_frequency_set(p.geom, self.topts, p.inv, dtype, c_in, _t(p.alpha0.reshape(-1)), self.f, pm,
                                     c_out)
        dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
        dc_o = self.ref_c.reshape(-1) - p.c_start.reshape(-1)
        rel = float(np.linalg.norm(dc_g - dc_o) / np.linalg.norm(dc_o))
        mx = float(np.max(np.abs(dc_g - dc_o)))
        return rel, mx, l2


@pytest.fixture(scope="module")
def config0():
    return _Case(W.small_ring(), 360)


@pytest.fixture(scope="module")
def config1_set0():
    return _Case(W.breast_ring256(), 720)


@pytest.fixture(scope="module")
def ring1040():
    # a large ring on a small grid: the 16-bit step takes the 128 x 128-tile
    # forward kernel, with its receiver-band skip (dmin = 130)
    return _Case(W.custom(44, 0.5e-3, 1040, 20e-3, 360, [[200e3, 250e3]], seed=9), 360)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_precision_form_ring1040_grid44(rb, ring1040, dtype):
    print(f"[gpu-case] precision ring1040_grid44 dtype={dtype}", flush=True)
    rel, mx, l2 = ring1040.run(rb, dtype)
    print(f"[precision] ring1040_grid44 {dtype}: rel-L2(dc) {rel:.3e}, max|dc diff| {mx:.3e} m/s, "
          f"|dc| {l2:.4f} vs oracle {ring1040.ref_l2:.4f}", flush=True)
    b_rel, b_max = BOUNDS[dtype]
    assert rel <= b_rel and mx <= b_max


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "bf16"])
def test_precision_form_ring64_grid128(rb, config0, dtype):
    print(f"[gpu-case] precision ring64_grid128 dtype={dtype}", flush=True)
    rel, mx, l2 = config0.run(rb, dtype)
    print(f"[precision] ring64_grid128 {dtype}: rel-L2(dc) {rel:.3e}, max|dc diff| {mx:.3e} m/s, "
          f"|dc| {l2:.4f} vs oracle {config0.ref_l2:.4f}", flush=True)
    b_rel, b_max = BOUNDS[dtype]
    assert rel <= b_rel and mx <= b_max


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_precision_form_ring256_grid480_set0(rb, config1_set0, dtype):
    print(f"[gpu-case] precision ring256_grid480 set 0 dtype={dtype}", flush=True)
    rel, mx, l2 = config1_set0.run(rb, dtype)
    print(f"[precision] ring256_grid480 set0 {dtype}: rel-L2(dc) {rel:.3e}, max|dc diff| {mx:.3e} m/s, "
          f"|dc| {l2:.4f} vs oracle {config1_set0.ref_l2:.4f}", flush=True)
    b_rel, b_max = BOUNDS[dtype]
    assert rel <= b_rel and mx <= b_max
