"""The grouped single step (rb_invert_frequency_sets_grouped): one frequency
set of several problems - different ring sizes, ragged grids, contraction
types - in one call whose backprojection contractions share launches, each
problem's result bitwise the one rb_invert_frequency_set gives it alone.
Twelve problems of one contraction type span two grouped launches (at most
eight problems each); an f64 problem runs its own contraction inside the
call.  One grouped problem is also checked against the FP64 oracle."""
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


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


# (grid n, ny, m, ring radius, rays, frequencies, seed, dtype)
PROBLEMS = [(40, 40, 16, 12e-3, 120, [2.5e5, 3.1e5], 31, "f32"),
            (47, 47, 24, 11e-3, 150, [2.4e5, 3.1e5, 3.7e5], 32, "f32"),
            (41, 33, 20, 10e-3, 120, [3.0e5], 33, "bf16"),
            (44, 44, 64, 14e-3, 180, [2.0e5, 2.5e5], 34, "f32"),
            (36, 36, 12, 9e-3, 96, [2.8e5], 35, "f64"),
            (39, 39, 40, 12e-3, 150, [2.2e5, 2.9e5], 36, "f16"),
            (33, 33, 28, 9e-3, 120, [3.3e5], 37, "bf16")] + \
           [(30 + i, 30 + i, 16 + 4 * i, 9e-3, 96, [2.6e5 + 1e4 * i], 40 + i, "f32") for i in range(9)]


def _problem(spec):
    n, ny, m, R, nr, fs, seed, dtype = spec
    p = W.custom(n, 0.5e-3, m, R, nr, [fs], seed=seed, ny=ny)
    return p, W.resolve_trace_opts(p.geom, p.c_start, nr), dtype


def _inputs(rb, p, topts, dtype):
    f = p.freq_sets[0]
    ws = torch.empty(rb.invert_workspace_bytes(p.geom, topts, len(f), dtype), dtype=torch.uint8, device=DEV)
    return {"g": p.geom, "t": topts, "o": p.inv, "dtype": dtype, "c_in": _t(p.c_start.reshape(-1)),
            "alpha0": _t(p.alpha0.reshape(-1)), "freqs": f,
            "p_meas": _t(np.stack([p.p_meas[0].real, p.p_meas[0].imag], -1)),
            "c_out": torch.empty(p.geom.n_pixels, dtype=torch.float64, device=DEV), "ws": ws}


def test_grouped_equals_alone_bitwise(rb):
    probs = [_problem(s) for s in PROBLEMS]
    n32 = sum(1 for _, _, d in probs if d == "f32")
    assert n32 > 8   # two grouped f32 launches
    _say(f"grouped single step over {len(probs)} problems ({n32} f32)")
    alone = []
    for p, topts, dtype in probs:
        j = _inputs(rb, p, topts, dtype)
        nrm = rb.invert_frequency_set(j["g"], j["t"], j["o"], dtype, j["c_in"], j["alpha0"], j["freqs"],
                                      j["p_meas"], j["c_out"], ws=j["ws"])
        alone.append((j["c_out"].cpu().numpy(), nrm))
    jobs = [_inputs(rb, p, topts, dtype) for p, topts, dtype in probs]
    norms = rb.invert_frequency_sets_grouped(jobs)
    for i, (j, (c_a, n_a)) in enumerate(zip(jobs, alone)):
        c_g = j["c_out"].cpu().numpy()
        assert np.array_equal(c_g, c_a), f"problem {i} ({PROBLEMS[i]}) differs grouped and alone"
        assert norms[i] == n_a
        assert not np.array_equal(c_g, probs[i][0].c_start.reshape(-1))
    # one grouped problem against the FP64 oracle (f32 contractions)
    p, topts, _ = probs[1]
    ref_c, ref_l2 = invert.invert_frequency_set(p.geom, topts, p.inv, p.c_start, p.alpha0, p.freq_sets[0],
                                                p.p_meas[0])
    dc_g = jobs[1]["c_out"].cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref_c.reshape(-1) - p.c_start.reshape(-1)
    rel = float(np.linalg.norm(dc_g - dc_o) / np.linalg.norm(dc_o))
    _say(f"grouped problem 1 vs oracle: rel-L2 {rel:.3e}")
    assert rel <= 1e-4 and np.abs(dc_g - dc_o).max() <= 0.01


def test_grouped_repeat_is_bitwise_and_in_place(rb):
    """In place (c_out = c_in), repeated from the same start: identical."""
    probs = [_problem(s) for s in PROBLEMS[:4]]
    outs = []
    for _ in range(2):
        jobs = [_inputs(rb, p, topts, dtype) for p, topts, dtype in probs]
        for j in jobs:
            j["c_out"] = j["c_in"]
        rb.invert_frequency_sets_grouped(jobs)
        outs.append([j["c_in"].cpu().numpy() for j in jobs])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
