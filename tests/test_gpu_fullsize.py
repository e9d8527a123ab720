"""GPU parity at the bench workload's full size (256 elements, 480 x 480
grid, 720 rays per element, 3 frequencies per set), in the launch
configuration bench.py times.  The oracle checks sampled outputs it can
compute one by one (tables of sampled emitters, the backprojection at
sampled pixels, forward data at sampled pairs) and one whole frequency set.
"""
import math
import sys

import numpy as np
import pytest

import workload as W
from _parity import close
from oracle import born, invert, rays

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
    return W.breast_ring256()


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def test_fullsize_tables_sampled_emitters(rb, prob):
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    _say("full-size trace, all 256 emitters")
    tabs = rb.alloc_tables(g, DEV)
    rb.trace_rays(g, topts, _t(1.0 / prob.c_start.reshape(-1)), _t(prob.alpha0.reshape(-1)), tabs)
    torch.cuda.synchronize()
    for e in (0, 37, 128, 201):
        T, A, B, Tr, Ar, Br = rays.tables(g, topts, 1.0 / prob.c_start, prob.alpha0, e, e + 1)
        Tg = tabs["T"][e].cpu().numpy()
        cg, co = np.isfinite(Tg), np.isfinite(T[0])
        assert int((cg != co).sum()) <= 5
        both = cg & co
        assert both.sum() > 0.5 * Tg.size
        assert np.max(np.abs(Tg[both] - T[0][both])) <= 1e-9
        ag = tabs["amp"][e].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(ag[both] - A[0][both]) / A[0][both]) <= 2e-6
        bg = tabs["att"][e].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(bg[both] - B[0][both])) <= 1e-6
        Trg = tabs["T_rx"][e].cpu().numpy()
        msk = invert.receiver_mask(g.m)[e]
        assert np.all(np.isfinite(Trg[msk])) and np.all(np.isfinite(Tr[0][msk]))
        assert np.max(np.abs(Trg[msk] - Tr[0][msk])) <= 1e-9


def test_fullsize_backprojection_sampled_pixels(rb, prob):
    g = prob.geom
    nf = 3
    T, A, B, _, _, _ = W.random_tables(g, seed=77)
    freqs = list(prob.freq_sets[0])
    D = W.random_residual(nf, g.m, 78)
    mask = invert.receiver_mask(g.m).astype(np.float64)
    rng = np.random.default_rng(79)
    Wd = np.stack([mask * (rng.uniform(size=mask.shape) > 0.01) for _ in range(nf)])
    _say("full-size backprojection f32 (random tables)")
    tabs = {"T": _t(T), "amp": _t(A, torch.float32), "att": _t(B, torch.float32),
            "T_rx": _t(np.zeros((g.m, g.m))), "amp_rx": _t(np.zeros((g.m, g.m)), torch.float32),
            "att_rx": _t(np.zeros((g.m, g.m)), torch.float32)}
    Gr = torch.empty((nf, g.m, g.n_pixels), dtype=torch.float32, device=DEV)
    Gi = torch.empty_like(Gr)
    rb.build_green(g, tabs, freqs, 1.0, "f32", Gr, Gi, None)
    grad = torch.zeros(g.n_pixels, dtype=torch.float64, device=DEV)
    hd = torch.zeros_like(grad)
    rb.born_adjoint_weighted(g, Gr, Gi, None, "f32", freqs, _t(np.stack([D.real, D.imag], -1)), _t(Wd), grad, hd)
    torch.cuda.synchronize()
    gg, hg = grad.cpu().numpy(), hd.cpu().numpy()
    xs = rng.choice(g.n_pixels, 300, replace=False)
    go, ho = np.zeros(xs.size), np.zeros(xs.size)
    for k, f in enumerate(freqs):
        G = born.green(T[:, xs], A[:, xs].astype(np.float64), B[:, xs].astype(np.float64), f)
        go += born.born_adjoint(G, Wd[k] * D[k], f, g.h ** 2)
        ho += born.hessian_diag(G, Wd[k], f, g.h ** 2)
    close(gg[xs], go, 1e-5, "full-size grad, sampled pixels")
    close(hg[xs], ho, 1e-5, "full-size hdiag, sampled pixels")
    # the banded Hessian diagonal for the same weights (band + zeroed pairs)
    zl, nz = [], []
    for k in range(nf):
        z = np.flatnonzero((mask > 0) & (Wd[k] == 0))
        zl.append(np.stack([z // g.m, z % g.m], -1).astype(np.int32))
        nz.append(len(z))
    zcap = max(1, max(nz))
    za = np.zeros((nf, zcap, 2), np.int32)
    for k in range(nf):
        za[k, :nz[k]] = zl[k]
    dmin = int(math.ceil(0.25 * 0.5 * g.m - 1e-9))
    hb = torch.zeros(g.n_pixels, dtype=torch.float64, device=DEV)
    rb.born_hessian_banded(g, Gr, Gi, None, "f32", freqs, dmin, torch.as_tensor(za, device=DEV),
                           torch.as_tensor(np.array(nz, np.int32), device=DEV), hb)
    torch.cuda.synchronize()
    hbg = hb.cpu().numpy()
    close(hbg[xs], ho, 1e-5, "full-size banded hdiag, sampled pixels")
    close(hbg, hg, 2e-5, "full-size banded vs MFMA hdiag")


def test_fullsize_forward_sampled_pairs(rb, prob):
    g = prob.geom
    nf = 3
    T, A, B, _, _, _ = W.random_tables(g, seed=87)
    freqs = list(prob.freq_sets[-1])
    delta = W.random_delta(g.n_pixels, 88)
    _say("full-size forward f32 (random tables)")
    tabs = {"T": _t(T), "amp": _t(A, torch.float32), "att": _t(B, torch.float32),
            "T_rx": _t(np.zeros((g.m, g.m))), "amp_rx": _t(np.zeros((g.m, g.m)), torch.float32),
            "att_rx": _t(np.zeros((g.m, g.m)), torch.float32)}
    Gr = torch.empty((nf, g.m, g.n_pixels), dtype=torch.float32, device=DEV)
    Gi = torch.empty_like(Gr)
    rb.build_green(g, tabs, freqs, 1.0, "f32", Gr, Gi, None)
    d = torch.empty((nf, g.m, g.m, 2), dtype=torch.float64, device=DEV)
    rb.born_forward(g, Gr, Gi, None, "f32", freqs, _t(delta), d)
    torch.cuda.synchronize()
    dg = d.cpu().numpy()
    rng = np.random.default_rng(89)
    pairs = [(int(a), int(b)) for a, b in zip(rng.integers(0, g.m, 60), rng.integers(0, g.m, 60))]
    es = sorted({e for e, _ in pairs} | {r for _, r in pairs})
    for k, f in enumerate(freqs):
        G = dict(zip(es, born.green(T[es], A[es].astype(np.float64), B[es].astype(np.float64), f)))
        om2 = (2 * math.pi * f) ** 2 * g.h ** 2
        ref = np.array([om2 * np.sum(G[e] * G[r] * delta) for e, r in pairs])
        got = np.array([dg[k, e, r, 0] + 1j * dg[k, e, r, 1] for e, r in pairs])
        close(got, ref, 1e-5, f"full-size forward f{k}, sampled pairs")


def test_fullsize_one_frequency_set_end_to_end(rb, prob):
    """The first set of the bench sweep, f32 contractions, against the oracle."""
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    f = prob.freq_sets[0]
    _say("full-size invert_frequency_set f32, set 0 (oracle ~10-30 s on the host)")
    ref = invert.invert_frequency_set(g, topts, prob.inv, prob.c_start, prob.alpha0, f, prob.p_meas[0],
                                      return_parts=True)
    c_in = _t(prob.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    pm = _t(np.stack([prob.p_meas[0].real, prob.p_meas[0].imag], -1))
    l2 = rb.invert_frequency_set(g, topts, prob.inv, "f32", c_in, _t(prob.alpha0.reshape(-1)), f, pm, c_out)
    dc_g = c_out.cpu().numpy() - prob.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - prob.c_start.reshape(-1)
    rel = np.linalg.norm(dc_g - dc_o) / np.linalg.norm(dc_o)
    print(f"[gpu-case] full-size set 0: rel-L2 {rel:.3e}, max|dc diff| {np.abs(dc_g - dc_o).max():.3e} m/s, "
          f"norms {l2:.4f} vs {ref['dc_l2']:.4f}", flush=True)
    assert rel <= 1e-4
    assert np.abs(dc_g - dc_o).max() <= 0.01
    assert abs(l2 - ref["dc_l2"]) <= 1e-4 * ref["dc_l2"]


def test_fullsize_cg_three_iterations(rb, prob):
    """CG on the first set of the bench sweep (f32 contractions, three
    iterations) against the oracle's preconditioned CG."""
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    f = prob.freq_sets[0]
    _say("full-size invert_frequency_set_cg f32, set 0, 3 iterations (oracle ~20-40 s on the host)")
    ref = invert.invert_frequency_set_cg(g, topts, prob.inv, prob.c_start, prob.alpha0, f, prob.p_meas[0], 3,
                                         return_parts=True)
    c_in = _t(prob.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    pm = _t(np.stack([prob.p_meas[0].real, prob.p_meas[0].imag], -1))
    l2, alphas, rzs = rb.invert_frequency_set_cg(g, topts, prob.inv, "f32", c_in, _t(prob.alpha0.reshape(-1)), f,
                                                 pm, 3, c_out)
    dc_g = c_out.cpu().numpy() - prob.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - prob.c_start.reshape(-1)
    rel = np.linalg.norm(dc_g - dc_o) / np.linalg.norm(dc_o)
    ea = np.linalg.norm(np.asarray(alphas) - ref["alpha"]) / np.linalg.norm(ref["alpha"])
    print(f"[gpu-case] full-size cg: rel-L2 {rel:.3e}, rel alpha {ea:.3e}, max|dc diff| "
          f"{np.abs(dc_g - dc_o).max():.3e} m/s, norms {l2:.4f} vs {ref['dc_l2']:.4f}", flush=True)
    assert rel <= 1e-4 and ea <= 1e-4
    assert abs(l2 - ref["dc_l2"]) <= 1e-4 * ref["dc_l2"]


def test_fullsize_tof_start(rb, prob):
    """The ToF starting model at the bench workload's size, from water:
    before the first update every ray is straight, so the rms residual
    equals that of the straight-ray times chord / c (to the wavefront sag);
    the residual then falls at every iteration and the model moves toward
    the phantom."""
    g = prob.geom
    c0 = np.full((g.ny, g.nx), g.c_background)
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    T_meas = W.straight_ray_tof(g, prob.c_true)
    pos = g.element_positions()
    chord = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
    sel = invert.receiver_mask(g.m, prob.inv.recv_fraction)
    rms_water = math.sqrt(float(np.mean((T_meas - chord / g.c_background)[sel] ** 2)))
    _say("full-size ToF start, 3 iterations from water")
    c_in = _t(c0.reshape(-1))
    c_out = torch.empty_like(c_in)
    rms, betas = rb.tof_invert(g, topts, prob.inv, c_in, _t(T_meas), 3, c_out)
    c = c_out.cpu().numpy()
    print(f"[gpu-case] full-size ToF: rms {rms} (straight rays {rms_water:.4e}), beta {betas}", flush=True)
    assert abs(rms[0] / rms_water - 1.0) <= 1e-2
    assert rms[1] < rms[0] and rms[2] < rms[1]
    assert all(b > 0 for b in betas)
    ct = prob.c_true.reshape(-1)
    assert np.linalg.norm(c - ct) < 0.6 * np.linalg.norm(c0.reshape(-1) - ct)
    assert np.all(np.isfinite(c)) and c.min() > 1300.0 and c.max() < 1700.0


def test_fullsize_asymptotic_weights(rb, prob):
    """Set 0 of the bench sweep with the asymptotic weights (f32) against the oracle."""
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    f = prob.freq_sets[0]
    _say("full-size asymptotic weights f32, set 0")
    ref = invert.invert_frequency_set_asymptotic(g, topts, prob.inv, prob.c_start, prob.alpha0, f, prob.p_meas[0])
    c_in = _t(prob.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    pm = _t(np.stack([prob.p_meas[0].real, prob.p_meas[0].imag], -1))
    l2 = rb.invert_frequency_set_asymptotic(g, topts, prob.inv, "f32", c_in, _t(prob.alpha0.reshape(-1)), f, pm,
                                            c_out)
    dc_g = c_out.cpu().numpy() - prob.c_start.reshape(-1)
    dc_o = ref[0].reshape(-1) - prob.c_start.reshape(-1)
    rel = np.linalg.norm(dc_g - dc_o) / np.linalg.norm(dc_o)
    print(f"[gpu-case] full-size asymptotic: rel-L2 {rel:.3e}, max|dc diff| {np.abs(dc_g - dc_o).max():.3e} m/s, "
          f"norms {l2:.4f} vs {ref[1]:.4f}", flush=True)
    assert rel <= 1e-4
    assert np.abs(dc_g - dc_o).max() <= 0.01
    assert abs(l2 - ref[1]) <= 1e-4 * ref[1]
