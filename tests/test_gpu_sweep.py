"""The frequency sweep on the GPU (each set's image starts the next, low to
high frequency; Inverse Problem section) against the oracle's sweep: three
sets of two frequencies on a 48-element ring, the model updated in place
as the serving loop and bench.py do."""
import numpy as np
import pytest

import workload as W
from oracle import invert

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BOUNDS = {"f64": (1e-6, 1e-4), "f32": (1e-4, 0.05)}   # rel-L2 of the total update, max |c difference| m/s


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_16633_amd as rbm
    rbm.lib()
    return rbm


@pytest.fixture(scope="module")
def case():
    p = W.custom(64, 0.5e-3, 48, 24e-3, 360, [[2.0e5, 2.5e5], [3.0e5, 3.5e5], [4.0e5, 4.5e5]], seed=11)
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    c_o, hist_o = invert.sweep(p.geom, topts, p.inv, p.c_start, p.alpha0, p.freq_sets, p.p_meas)
    return p, topts, c_o, hist_o


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sweep_matches_oracle(rb, case, dtype):
    p, topts, c_o, hist_o = case
    print(f"[gpu-case] sweep of three sets dtype={dtype}", flush=True)
    c = torch.as_tensor(p.c_start.reshape(-1).copy(), device=DEV)
    al = torch.as_tensor(p.alpha0.reshape(-1), device=DEV)
    hist = []
    for fs, pm in zip(p.freq_sets, p.p_meas):
        pmt = torch.as_tensor(np.stack([pm.real, pm.imag], -1), device=DEV)
        hist.append(rb.invert_frequency_set(p.geom, topts, p.inv, dtype, c, al, fs, pmt, c))
    cg = c.cpu().numpy()
    d_g = cg - p.c_start.reshape(-1)
    d_o = c_o.reshape(-1) - p.c_start.reshape(-1)
    rel = float(np.linalg.norm(d_g - d_o) / np.linalg.norm(d_o))
    mx = float(np.max(np.abs(d_g - d_o)))
    print(f"[sweep] {dtype}: rel-L2 of the total update {rel:.3e}, max |c diff| {mx:.3e} m/s, "
          f"set norms {[round(h, 4) for h in hist]} vs {[round(h, 4) for h in hist_o]}", flush=True)
    b_rel, b_max = BOUNDS[dtype]
    assert rel <= b_rel and mx <= b_max
    assert np.allclose(hist, hist_o, rtol=b_rel, atol=0)
