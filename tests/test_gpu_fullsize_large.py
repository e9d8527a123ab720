"""GPU parity at the large instance's full size (1024 elements, 1100 x 1100
grid at 0.2 mm, four frequencies per set) in the launch configuration
`bench.py --workload ring1024_grid1100` times: the backprojection at sampled
pixels (bf16 and f32 tables) and the bf16 forward at sampled pairs (the
128 x 128-tile kernel), against the oracle computed for those outputs one by
one.  The tables are seeded random draws made on the host in blocks of
emitters (the oracle keeps the columns and rows it needs).  Then the ray
tables at sampled emitters, and one whole frequency set in FP32 and BF16
against the same set in FP64."""
import math
import sys

import numpy as np
import pytest

import workload as W
from _parity import close
from oracle import born, invert

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"f32": 1e-5, "bf16": 1e-2}


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
def case():
    """Geometry, frequencies, device tables and the host samples the oracle
    needs: all emitters at 300 pixels, full rows of the sampled emitters."""
    g = W.centred_grid(1100, 0.2e-3, 1024, 110e-3, 1500.0)
    freqs = list(np.linspace(0.3e6, 2.0e6, 48)[:4])
    rng = np.random.default_rng(301)
    xs = np.sort(rng.choice(g.n_pixels, 300, replace=False))
    pairs = [(int(a), int(b)) for a, b in zip(rng.integers(0, g.m, 24), rng.integers(0, g.m, 24))]
    rows = sorted({e for e, _ in pairs} | {r for _, r in pairs})
    m, n = g.m, g.n_pixels
    t_scale = 2.0 * g.ring_radius / g.c_background
    T = torch.empty((m, n), dtype=torch.float64, device=DEV)
    A = torch.empty((m, n), dtype=torch.float32, device=DEV)
    B = torch.empty((m, n), dtype=torch.float32, device=DEV)
    cols = {"T": np.empty((m, xs.size)), "A": np.empty((m, xs.size)), "B": np.empty((m, xs.size))}
    full = {}
    blk = 64
    for e0 in range(0, m, blk):
        r = np.random.default_rng(1000 + e0)
        t = r.uniform(0.05, 1.0, (blk, n)) * t_scale
        a = r.uniform(5.0, 50.0, (blk, n)).astype(np.float32)
        b = r.uniform(0.0, 0.2, (blk, n)).astype(np.float32)
        T[e0:e0 + blk] = torch.as_tensor(t, device=DEV)
        A[e0:e0 + blk] = torch.as_tensor(a, device=DEV)
        B[e0:e0 + blk] = torch.as_tensor(b, device=DEV)
        cols["T"][e0:e0 + blk] = t[:, xs]
        cols["A"][e0:e0 + blk] = a[:, xs]
        cols["B"][e0:e0 + blk] = b[:, xs]
        for e in rows:
            if e0 <= e < e0 + blk:
                full[e] = (t[e - e0].copy(), a[e - e0].astype(np.float64), b[e - e0].astype(np.float64))
    z64 = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    z32 = torch.zeros((m, m), dtype=torch.float32, device=DEV)
    tabs = {"T": T, "amp": A, "att": B, "T_rx": z64, "amp_rx": z32, "att_rx": z32}
    return g, freqs, xs, pairs, tabs, cols, full


def _green(rb, g, tabs, freqs, dtype):
    td = {"f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    Gr = torch.empty((len(freqs), g.m, g.n_pixels), dtype=td, device=DEV)
    Gi = torch.empty_like(Gr)
    sc = torch.empty(len(freqs), dtype=torch.float32, device=DEV)
    rb.build_green(g, tabs, freqs, 1.0, dtype, Gr, Gi, sc)
    return Gr, Gi, sc


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_large_backprojection_sampled_pixels(rb, case, dtype):
    g, freqs, xs, _, tabs, cols, _ = case
    nf = len(freqs)
    D = W.random_residual(nf, g.m, 302)
    mask = invert.receiver_mask(g.m).astype(np.float64)
    Wd = np.repeat(mask[None], nf, axis=0)
    _say(f"large backprojection {dtype} (1024 elements, 1100^2, random tables)")
    Gr, Gi, sc = _green(rb, g, tabs, freqs, dtype)
    grad = torch.zeros(g.n_pixels, dtype=torch.float64, device=DEV)
    dres = torch.as_tensor(np.stack([D.real, D.imag], -1), device=DEV)
    rb.born_adjoint_weighted(g, Gr, Gi, sc, dtype, freqs, dres, torch.as_tensor(Wd, device=DEV), grad, None)
    torch.cuda.synchronize()
    gg = grad[torch.as_tensor(xs, device=DEV)].cpu().numpy()
    del Gr, Gi
    torch.cuda.empty_cache()
    go = np.zeros(xs.size)
    for k, f in enumerate(freqs):
        G = born.green(cols["T"], cols["A"], cols["B"], f)
        go += born.born_adjoint(G, Wd[k] * D[k], f, g.h ** 2)
    close(gg, go, TOL[dtype], f"large backprojection {dtype} at {xs.size} pixels")


def test_large_forward_sampled_pairs_bf16(rb, case):
    g, freqs, _, pairs, tabs, _, full = case
    nf = len(freqs)
    delta = W.random_delta(g.n_pixels, 303)
    _say("large forward bf16 (1024 elements, 1100^2, random tables)")
    Gr, Gi, sc = _green(rb, g, tabs, freqs, "bf16")
    d = torch.empty((nf, g.m, g.m, 2), dtype=torch.float64, device=DEV)
    rb.born_forward(g, Gr, Gi, sc, "bf16", freqs, torch.as_tensor(delta, device=DEV), d)
    torch.cuda.synchronize()
    dg = d.cpu().numpy()
    del Gr, Gi
    torch.cuda.empty_cache()
    for k, f in enumerate(freqs):
        G = {e: born.green(t[None], a[None], b[None], f)[0] for e, (t, a, b) in full.items()}
        om2 = (2 * math.pi * f) ** 2 * g.h ** 2
        ref = np.array([om2 * np.sum(G[e] * G[r] * delta) for e, r in pairs])
        got = np.array([dg[k, e, r, 0] + 1j * dg[k, e, r, 1] for e, r in pairs])
        close(got, ref, TOL["bf16"], f"large forward bf16 f={f:.3e} at {len(pairs)} pairs")


def test_large_tables_sampled_emitters(rb):
    """Ray tables of the large instance's start model (1440 rays per element,
    emitters traced 128 at a time as bench.py does) at two sampled emitters
    against the oracle's tracer and rasteriser."""
    from oracle import rays
    prob = W.breast_ring1024(with_data=False)
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    _say("large trace, all 1024 emitters in batches of 128")
    tabs = rb.alloc_tables(g, DEV)
    ws = torch.empty(rb.trace_workspace_bytes(g, topts, 128), dtype=torch.uint8, device=DEV)
    s = torch.as_tensor(1.0 / prob.c_start.reshape(-1), device=DEV)
    a = torch.as_tensor(prob.alpha0.reshape(-1), device=DEV)
    rb.trace_rays(g, topts, s, a, tabs, ws=ws)
    torch.cuda.synchronize()
    del ws
    for e in (5, 700):
        T, A, B, Tr, Ar, Br = rays.tables(g, topts, 1.0 / prob.c_start, prob.alpha0, e, e + 1)
        Tg = tabs["T"][e].cpu().numpy()
        cg, co = np.isfinite(Tg), np.isfinite(T[0])
        both = cg & co
        ndiff = int((cg != co).sum())
        dT = float(np.max(np.abs(Tg[both] - T[0][both])))
        ag = tabs["amp"][e].cpu().numpy().astype(np.float64)
        da = float(np.max(np.abs(ag[both] - A[0][both]) / A[0][both]))
        bg = tabs["att"][e].cpu().numpy().astype(np.float64)
        dB = float(np.max(np.abs(bg[both] - B[0][both])))
        print(f"[large] tables emitter {e}: coverage differences {ndiff}, max |dT| {dT:.2e} s, "
              f"max rel da {da:.2e}, max |dB| {dB:.2e}", flush=True)
        assert ndiff <= 50 and both.sum() > 0.5 * Tg.size
        assert dT <= 1e-9 and da <= 2e-6 and dB <= 1e-6
        Trg = tabs["T_rx"][e].cpu().numpy()
        msk = invert.receiver_mask(g.m)[e]
        assert np.all(np.isfinite(Trg[msk])) and np.all(np.isfinite(Tr[0][msk]))
        assert np.max(np.abs(Trg[msk] - Tr[0][msk])) <= 1e-9


def test_large_frequency_set_fp32_and_bf16_against_fp64(rb):
    """One whole linearised frequency set of the large instance (set 0 of the
    breast phantom with straight-ray data, the launch configuration the bench
    times: 128 emitters per tracing batch): the FP32 and BF16 steps against
    the FP64 step, whose contractions run on the FP64 matrix cores and which
    matches the oracle at the smaller sizes (test_gpu_fullsize,
    test_gpu_parity).  The FP64 oracle itself would need about five minutes
    of 16 CPU threads for this set.  Bounds: the contraction types' image
    tolerances (FP32 rel-L2 1e-4 and max |dc| 0.01 m/s; BF16 1e-2 and
    1 m/s)."""
    prob = W.breast_ring1024(with_data=False)
    g = prob.geom
    fs = prob.freq_sets[0]
    _say("large frequency set: straight-ray data of set 0 (1024 elements, 1100^2)")
    pm = W.data_for_sets(g, prob.c_true, prob.alpha0, [fs])[0]
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    c_in = torch.as_tensor(prob.c_start.reshape(-1), dtype=torch.float64, device=DEV)
    al = torch.as_tensor(prob.alpha0.reshape(-1), dtype=torch.float64, device=DEV)
    pmt = torch.as_tensor(np.stack([pm.real, pm.imag], -1), dtype=torch.float64, device=DEV)
    dc = {}
    for dt in ("f64", "f32", "bf16"):
        _say(f"large frequency set {dt}")
        ws = torch.empty(rb.invert_workspace_bytes(g, topts, len(fs), dt, 128), dtype=torch.uint8, device=DEV)
        c_out = torch.empty_like(c_in)
        rb.invert_frequency_set(g, topts, prob.inv, dt, c_in, al, fs, pmt, c_out, ws=ws)
        dc[dt] = (c_out - c_in).cpu().numpy()
        del ws, c_out
        torch.cuda.empty_cache()
    ref = dc["f64"]
    assert np.all(np.isfinite(ref)) and np.linalg.norm(ref) > 0.0
    for dt, (rel_b, max_b) in (("f32", (1e-4, 0.01)), ("bf16", (1e-2, 1.0))):
        d = dc[dt] - ref
        rel = float(np.linalg.norm(d) / np.linalg.norm(ref))
        mx = float(np.abs(d).max())
        _say(f"large frequency set {dt} vs f64: rel-L2 {rel:.3e}, max |dc diff| {mx:.3e} m/s")
        assert rel <= rel_b and mx <= max_b, (dt, rel, mx)
