"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Inputs come from the seeded generators in ``workload``; the oracle computes
its own results from the same inputs.  Sizes span several tiles with ragged
tails; tolerances are stated per quantity and dtype:

* travel time tables: |dT| <= 1e-9 s where both are covered;
* amplitude / absorption tables (FP32 storage): rel 2e-6 / abs 1e-6;
* contractions (same input tables): rel-L2 <= 1e-10 (f64), 1e-5 (f32),
  2e-3 (f16), 1e-2 (bf16);
* one inversion step: rel-L2 of the update <= 1e-4 (f32/f64 path).
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


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _tables_gpu(rb, geom, topts, c, alpha):
    tabs = rb.alloc_tables(geom, DEV)
    s = _t(1.0 / c.reshape(-1))
    al = None if alpha is None else _t(alpha.reshape(-1))
    rb.trace_rays(geom, topts, s, al, tabs)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in tabs.items()}


def _compare_tables(gpu, ora, T_tol=1e-9):
    for key_T, key_a, key_b in (("T", "amp", "att"), ("T_rx", "amp_rx", "att_rx")):
        Tg, To = gpu[key_T], ora[key_T]
        cg, co = np.isfinite(Tg), np.isfinite(To)
        mismatch = int((cg != co).sum())
        assert mismatch <= max(2, int(1e-5 * cg.size)), f"{key_T}: coverage differs at {mismatch} points"
        both = cg & co
        assert both.sum() > 0.3 * cg.size
        assert np.max(np.abs(Tg[both] - To[both])) <= T_tol
        ag, ao = gpu[key_a][both], ora[key_a][both]
        assert np.max(np.abs(ag - ao) / np.maximum(np.abs(ao), 1e-30)) <= 2e-6
        bg, bo = gpu[key_b][both], ora[key_b][both]
        assert np.max(np.abs(bg - bo)) <= 1e-6 * max(1.0, np.abs(bo).max())
        assert np.all(gpu[key_a][~cg] == 0) and np.all(gpu[key_b][~cg] == 0)


def _oracle_tables(geom, topts, c, alpha, e0=0, e1=None):
    T, A, B, Tr, Ar, Br = rays.tables(geom, topts, 1.0 / c, alpha, e0, e1)
    return {"T": T, "amp": A, "att": B, "T_rx": Tr, "amp_rx": Ar, "att_rx": Br}


# ----------------------------------------------------------------------------- tracing

@pytest.mark.parametrize("case", ["ring64_grid128", "ragged_45x45_m12", "ring_outside_grid", "ring64_caustic_lens"])
def test_trace_tables_match_oracle(rb, case):
    if case == "ring64_caustic_lens":
        # a strong slow lens in front of element 0 folds the wavefronts of the
        # nearby elements: where two branches overlap, both sides must keep the
        # earlier one (their amplitudes differ severalfold)
        geom = W.centred_grid(128, 0.5e-3, 64, 30e-3, 1500.0)
        c, al = W.lens_medium(geom, (25e-3, 0.0), 1.5e-3, -400.0)
        topts = W.resolve_trace_opts(geom, c, 360)
    elif case == "ring64_grid128":
        p = W.small_ring(with_data=False)
        geom, c, al = p.geom, p.c_true, p.alpha0
        topts = W.resolve_trace_opts(geom, c, 360)
    elif case == "ragged_45x45_m12":
        p = W.custom(45, 0.5e-3, 12, 10e-3, 90, [[3e5]], seed=4, with_data=False)
        geom, c, al = p.geom, p.c_true, p.alpha0
        topts = W.resolve_trace_opts(geom, c, 90)
    else:   # ring radius beyond the grid half-width; no absorption map
        p = W.custom(40, 0.5e-3, 16, 12e-3, 120, [[3e5]], seed=5, with_data=False)
        geom, c, al = p.geom, p.c_true, None
        topts = W.resolve_trace_opts(geom, c, 120)
    _say(f"trace {case} m={geom.m} N={geom.n_pixels} rays={topts.n_rays}")
    gpu = _tables_gpu(rb, geom, topts, c, al)
    ora = _oracle_tables(geom, topts, c, al)
    _compare_tables(gpu, ora)


def test_trace_batched_workspace_matches_single_batch(rb):
    p = W.custom(41, 0.5e-3, 10, 9e-3, 64, [[3e5]], seed=6, with_data=False)
    geom, c, al = p.geom, p.c_true, p.alpha0
    topts = W.resolve_trace_opts(geom, c, 64)
    _say("trace batched workspace (3 emitters per batch)")
    s, alt = _t(1.0 / c.reshape(-1)), _t(al.reshape(-1))
    full = rb.alloc_tables(geom, DEV)
    rb.trace_rays(geom, topts, s, alt, full)
    small = rb.alloc_tables(geom, DEV)
    ws = torch.empty(rb.trace_workspace_bytes(geom, topts, 3), dtype=torch.uint8, device=DEV)
    rb.trace_rays(geom, topts, s, alt, small, ws=ws)
    torch.cuda.synchronize()
    for k in full:
        a, b = full[k].cpu().numpy(), small[k].cpu().numpy()
        assert np.array_equal(np.isnan(a), np.isnan(b))
        assert np.array_equal(np.nan_to_num(a), np.nan_to_num(b)), k


# ----------------------------------------------------------------------------- Green's functions

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_build_green_matches_oracle(rb, dtype):
    geom = W.centred_grid(33, 0.5e-3, 20, 10e-3, 1500.0)
    T, A, B, Tr, Ar, Br = W.random_tables(geom, seed=11)
    freqs = [2.5e5, 7.3e5, 1.9e6]
    _say(f"build_green dtype={dtype}")
    tabs = {"T": _t(T), "amp": _t(A, torch.float32), "att": _t(B, torch.float32),
            "T_rx": _t(Tr), "amp_rx": _t(Ar, torch.float32), "att_rx": _t(Br, torch.float32)}
    td = rb._binding.TORCH_DTYPES[rb.DTYPES[dtype]]
    Gr = torch.empty((3, geom.m, geom.n_pixels), dtype=td, device=DEV)
    Gi = torch.empty_like(Gr)
    sc = torch.empty(3, dtype=torch.float32, device=DEV)
    rb.build_green(geom, tabs, freqs, 1.0, dtype, Gr, Gi, sc)
    torch.cuda.synchronize()
    scale = sc.cpu().numpy().astype(np.float64)
    tol = {"f64": 1e-14, "f32": 1e-7, "bf16": 8e-3, "f16": 1e-3}[dtype]
    for k, f in enumerate(freqs):
        Go = born.green(T, A.astype(np.float64), B.astype(np.float64), f)
        Gg = (Gr[k].double().cpu().numpy() + 1j * Gi[k].double().cpu().numpy()) * scale[k]
        err = np.abs(Gg - Go).max() / np.abs(Go).max()
        assert err <= tol, (k, err)
        assert np.all(Gg[np.isnan(T)] == 0)


# ----------------------------------------------------------------------------- contractions

def _contraction_inputs(geom, nf, seed):
    T, A, B, _, _, _ = W.random_tables(geom, seed=seed)
    freqs = list(np.linspace(3e5, 9e5, nf))
    D = W.random_residual(nf, geom.m, seed + 1)
    mask = invert.receiver_mask(geom.m, 0.75).astype(np.float64)
    rng = np.random.default_rng(seed + 2)
    Wd = np.stack([mask * (rng.uniform(size=mask.shape) > 0.02) for _ in range(nf)])
    delta = W.random_delta(geom.n_pixels, seed + 3)
    return T, A, B, freqs, D, Wd, delta


def _gpu_green(rb, geom, T, A, B, freqs, dtype):
    tabs = {"T": _t(T), "amp": _t(A, torch.float32), "att": _t(B, torch.float32),
            "T_rx": _t(np.zeros((geom.m, geom.m))), "amp_rx": _t(np.zeros((geom.m, geom.m)), torch.float32),
            "att_rx": _t(np.zeros((geom.m, geom.m)), torch.float32)}
    td = rb._binding.TORCH_DTYPES[rb.DTYPES[dtype]]
    Gr = torch.empty((len(freqs), geom.m, geom.n_pixels), dtype=td, device=DEV)
    Gi = torch.empty_like(Gr)
    sc = torch.empty(len(freqs), dtype=torch.float32, device=DEV)
    rb.build_green(geom, tabs, freqs, 1.0, dtype, Gr, Gi, sc)
    return Gr, Gi, sc


CONTRACTION_TOL = {"f64": 1e-10, "f32": 1e-5, "f16": 2e-3, "bf16": 1e-2}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("shape", [(37, 29, 40), (64, 64, 64), (21, 50, 97), (30, 30, 48), (24, 23, 300),
                                   (26, 19, 90)])
def test_adjoint_and_hessian_match_oracle(rb, dtype, shape):
    nx, ny, m = shape
    geom = W.centred_grid(nx, 0.5e-3, m, 12e-3, 1500.0)
    import dataclasses
    geom = dataclasses.replace(geom, ny=ny, y0=-0.5 * (ny - 1) * 0.5e-3)
    nf = 2
    T, A, B, freqs, D, Wd, _ = _contraction_inputs(geom, nf, 21)
    _say(f"adjoint dtype={dtype} nx={nx} ny={ny} m={m}")
    Gr, Gi, sc = _gpu_green(rb, geom, T, A, B, freqs, dtype)
    grad = torch.zeros(geom.n_pixels, dtype=torch.float64, device=DEV)
    hd = torch.zeros_like(grad)
    dres = _t(np.stack([D.real, D.imag], axis=-1))
    rb.born_adjoint_weighted(geom, Gr, Gi, sc, dtype, freqs, dres, _t(Wd), grad, hd)
    grad_only = torch.zeros_like(grad)
    rb.born_adjoint_weighted(geom, Gr, Gi, sc, dtype, freqs, dres, _t(Wd), grad_only, None)
    torch.cuda.synchronize()
    g_o = np.zeros(geom.n_pixels)
    h_o = np.zeros(geom.n_pixels)
    for k, f in enumerate(freqs):
        G = born.green(T, A.astype(np.float64), B.astype(np.float64), f)
        g_o += born.born_adjoint(G, Wd[k] * D[k], f, geom.h ** 2)
        h_o += born.hessian_diag(G, Wd[k], f, geom.h ** 2)
    tol = CONTRACTION_TOL[dtype]
    close(grad.cpu().numpy(), g_o, tol, f"grad {dtype} {shape}")
    close(hd.cpu().numpy(), h_o, tol, f"hdiag {dtype} {shape}")
    close(grad_only.cpu().numpy(), g_o, tol, f"grad-only {dtype} {shape}")   # the gradient-only kernel


def _banded_weights(m, nf, dmin, nzero_each, seed):
    """Band-selection weights with `nzero_each` selected pairs zeroed per
    frequency, and the (e, r) list of those pairs."""
    e = np.arange(m)[:, None]
    r = np.arange(m)[None, :]
    d = np.minimum(np.abs(e - r), m - np.abs(e - r))
    sel = d >= dmin
    rng = np.random.default_rng(seed)
    Wd, lists = [], []
    for _ in range(nf):
        w = sel.astype(np.float64)
        idx = np.flatnonzero(sel)
        z = np.sort(rng.choice(idx, size=min(nzero_each, idx.size), replace=False)) if idx.size else idx
        w.reshape(-1)[z] = 0.0
        Wd.append(w)
        lists.append(np.stack([z // m, z % m], axis=-1).astype(np.int32))
    return np.stack(Wd), lists


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("shape", [(37, 29, 40, 5, 6), (64, 64, 64, 8, 40), (21, 50, 97, 12, 0),
                                   (30, 30, 33, 0, 9), (30, 30, 16, 9, 0), (24, 23, 300, 38, 70),
                                   (10, 11, 1024, 128, 300), (12, 12, 1024, 128, 300),
                                   (37, 29, 40, 5, 700), (24, 23, 300, 38, 5000), (12, 12, 1024, 128, 9000)])
def test_hessian_banded_matches_oracle(rb, dtype, shape):
    """The banded Hessian diagonal against the oracle's dense sum with the same
    weights, and against the backprojection's Hessian diagonal (dmin = 0: no
    band; dmin = 9 at m = 16: the band covers the ring, so hd = 0; the last
    three shapes pass their zeroed pairs through LDS in two to five chunks)."""
    nx, ny, m, dmin, nz = shape
    geom = W.centred_grid(nx, 0.5e-3, m, 12e-3, 1500.0)
    import dataclasses
    geom = dataclasses.replace(geom, ny=ny, y0=-0.5 * (ny - 1) * 0.5e-3)
    nf = 2
    T, A, B, freqs, D, _, _ = _contraction_inputs(geom, nf, 41)
    Wd, lists = _banded_weights(m, nf, dmin, nz, 42)
    _say(f"hessian_banded dtype={dtype} nx={nx} ny={ny} m={m} dmin={dmin} zeroed={nz}")
    Gr, Gi, sc = _gpu_green(rb, geom, T, A, B, freqs, dtype)
    zcap = max(1, max(len(q) for q in lists))
    zl = np.zeros((nf, zcap, 2), np.int32)
    for k, q in enumerate(lists):
        zl[k, :len(q)] = q
    nzero = torch.as_tensor(np.array([len(q) for q in lists], np.int32), device=DEV)
    hd = torch.zeros(geom.n_pixels, dtype=torch.float64, device=DEV)
    rb.born_hessian_banded(geom, Gr, Gi, sc, dtype, freqs, dmin, torch.as_tensor(zl, device=DEV), nzero, hd)
    grad = torch.zeros_like(hd)
    hd_mfma = torch.zeros_like(hd)
    rb.born_adjoint_weighted(geom, Gr, Gi, sc, dtype, freqs, _t(np.stack([D.real, D.imag], -1)), _t(Wd), grad,
                             hd_mfma)
    torch.cuda.synchronize()
    h_o = np.zeros(geom.n_pixels)
    for k, f in enumerate(freqs):
        G = born.green(T, A.astype(np.float64), B.astype(np.float64), f)
        h_o += born.hessian_diag(G, Wd[k], f, geom.h ** 2)
    hg = hd.cpu().numpy()
    if not np.any(Wd):
        assert np.all(hg == 0.0) and np.all(h_o == 0.0)
        return
    tol = CONTRACTION_TOL[dtype]
    close(hg, h_o, tol, f"banded hdiag {dtype} {shape}")
    close(hg, hd_mfma.cpu().numpy(), 2 * tol, f"banded vs MFMA hdiag {dtype} {shape}")


def test_hessian_banded_ignores_bad_pairs_and_is_deterministic(rb):
    geom = W.centred_grid(24, 0.5e-3, 32, 8e-3, 1500.0)
    T, A, B, freqs, _, _, _ = _contraction_inputs(geom, 1, 51)
    Wd, lists = _banded_weights(32, 1, 4, 10, 52)
    Gr, Gi, sc = _gpu_green(rb, geom, T, A, B, freqs, "f32")
    zl = np.zeros((1, 12, 2), np.int32)
    zl[0, :10] = lists[0]
    zl[0, 10] = (-1, 3)        # out of range: ignored
    zl[0, 11] = (5, 32)        # out of range: ignored
    zdev = torch.as_tensor(zl, device=DEV)
    outs = []
    for n in (12, 12):
        hd = torch.zeros(geom.n_pixels, dtype=torch.float64, device=DEV)
        rb.born_hessian_banded(geom, Gr, Gi, sc, "f32", freqs, 4, zdev,
                               torch.tensor([n], dtype=torch.int32, device=DEV), hd)
        outs.append(hd.cpu().numpy())
    G = born.green(T, A.astype(np.float64), B.astype(np.float64), freqs[0])
    h_o = born.hessian_diag(G, Wd[0], freqs[0], geom.h ** 2)
    assert np.array_equal(outs[0], outs[1])
    close(outs[0], h_o, 1e-5, "banded hdiag, out-of-range pairs")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("shape", [(37, 29, 40), (50, 50, 130), (24, 20, 1030), (22, 20, 1100)])
def test_forward_matches_oracle(rb, dtype, shape):
    """The last two shapes take the 128 x 128-tile 16-bit kernel (m >= 1024,
    N a multiple of 8): whole and partial last pixel chunks, m not a
    multiple of the tile."""
    nx, ny, m = shape
    geom = W.centred_grid(nx, 0.5e-3, m, 12e-3, 1500.0)
    import dataclasses
    geom = dataclasses.replace(geom, ny=ny, y0=-0.5 * (ny - 1) * 0.5e-3)
    nf = 2
    T, A, B, freqs, _, _, delta = _contraction_inputs(geom, nf, 31)
    _say(f"forward dtype={dtype} nx={nx} ny={ny} m={m}")
    Gr, Gi, sc = _gpu_green(rb, geom, T, A, B, freqs, dtype)
    d = torch.empty((nf, m, m, 2), dtype=torch.float64, device=DEV)
    rb.born_forward(geom, Gr, Gi, sc, dtype, freqs, _t(delta), d)
    torch.cuda.synchronize()
    dg = d.cpu().numpy()
    dg = dg[..., 0] + 1j * dg[..., 1]
    tol = CONTRACTION_TOL[dtype]
    for k, f in enumerate(freqs):
        G = born.green(T, A.astype(np.float64), B.astype(np.float64), f)
        do = born.born_forward(G, delta, f, geom.h ** 2)
        close(dg[k], do, tol, f"forward {dtype} {shape} f{k}")
        assert np.array_equal(dg[k], dg[k].T)


def test_adjoint_is_deterministic_and_accumulates(rb):
    geom = W.centred_grid(48, 0.5e-3, 64, 12e-3, 1500.0)
    T, A, B, freqs, D, Wd, _ = _contraction_inputs(geom, 3, 41)
    _say("adjoint determinism")
    Gr, Gi, sc = _gpu_green(rb, geom, T, A, B, freqs, "f32")
    dres = _t(np.stack([D.real, D.imag], axis=-1))
    outs = []
    for _ in range(2):
        grad = torch.zeros(geom.n_pixels, dtype=torch.float64, device=DEV)
        rb.born_adjoint_weighted(geom, Gr, Gi, sc, "f32", freqs, dres, _t(Wd), grad, None)
        outs.append(grad.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    grad = torch.zeros(geom.n_pixels, dtype=torch.float64, device=DEV)
    for _ in range(2):
        rb.born_adjoint_weighted(geom, Gr, Gi, sc, "f32", freqs, dres, _t(Wd), grad, None)
    assert np.allclose(grad.cpu().numpy(), 2 * outs[0], rtol=1e-15, atol=0)


def test_gpu_dot_product_adjoint(rb):
    geom = W.centred_grid(40, 0.5e-3, 32, 12e-3, 1500.0)
    T, A, B, freqs, D, _, delta = _contraction_inputs(geom, 1, 51)
    Wd = np.ones((1, geom.m, geom.m))
    _say("gpu dot-product test f64")
    Gr, Gi, sc = _gpu_green(rb, geom, T, A, B, freqs, "f64")
    d = torch.empty((1, geom.m, geom.m, 2), dtype=torch.float64, device=DEV)
    rb.born_forward(geom, Gr, Gi, sc, "f64", freqs, _t(delta), d)
    grad = torch.zeros(geom.n_pixels, dtype=torch.float64, device=DEV)
    rb.born_adjoint_weighted(geom, Gr, Gi, sc, "f64", freqs, _t(np.stack([D.real, D.imag], -1)), _t(Wd), grad,
                             None)
    torch.cuda.synchronize()
    dj = d.cpu().numpy()
    lhs = float(np.sum(dj[0, ..., 0] * D[0].real + dj[0, ..., 1] * D[0].imag))
    rhs = float(np.dot(delta, grad.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


# ----------------------------------------------------------------------------- one inversion step

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_invert_frequency_set_matches_oracle(rb, dtype):
    p = W.small_ring()
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    _say(f"invert ring64_grid128 dtype={dtype}")
    ref = invert.invert_frequency_set(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0],
                                      return_parts=True)
    pm = _t(np.stack([p.p_meas[0].real, p.p_meas[0].imag], -1))
    c_in = _t(p.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    dl2 = rb.invert_frequency_set(p.geom, topts, p.inv, dtype, c_in, _t(p.alpha0.reshape(-1)), f, pm, c_out)
    dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref["c_new"].reshape(-1) - p.c_start.reshape(-1)
    assert _rel(dc_g, dc_o) <= 1e-4
    assert np.max(np.abs(dc_g - dc_o)) <= 0.01
    assert abs(dl2 - ref["dc_l2"]) <= 1e-4 * ref["dc_l2"]
    assert np.array_equal(c_in.cpu().numpy(), p.c_start.reshape(-1))


def test_invert_outlier_ties_split_by_flat_index(rb):
    """The outlier threshold falls inside a group of exactly equal |p|^2:
    of 3k tied pairs the k with the smallest flat index are zeroed (the
    oracle's lexicographic order), which only the ranked-tie path decides."""
    p = W.small_ring()
    topts = W.resolve_trace_opts(p.geom, p.c_start, 360)
    f = p.freq_sets[0]
    m = p.geom.m
    mask = invert.receiver_mask(m, p.inv.recv_fraction)
    sel = np.flatnonzero(mask.reshape(-1))
    kz = int(np.floor(p.inv.outlier_fraction * sel.size))
    assert kz >= 1
    pm = p.p_meas[0].copy()
    rng = np.random.default_rng(77)
    for k in range(pm.shape[0]):
        big = 2.0 * np.abs(pm[k]).max()
        tied = np.sort(rng.choice(sel, size=3 * kz, replace=False))
        pm[k].reshape(-1)[tied] = big * np.exp(0.3j)
    _say("invert ring64_grid128 f64 with tied outliers")
    ref = invert.invert_frequency_set(p.geom, topts, p.inv, p.c_start, p.alpha0, f, pm)
    c_in = _t(p.c_start.reshape(-1))
    c_out = torch.empty_like(c_in)
    rb.invert_frequency_set(p.geom, topts, p.inv, "f64", c_in, _t(p.alpha0.reshape(-1)), f,
                            _t(np.stack([pm.real, pm.imag], -1)), c_out)
    dc_g = c_out.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref[0].reshape(-1) - p.c_start.reshape(-1)
    assert _rel(dc_g, dc_o) <= 1e-6


def test_invert_in_place_and_ragged(rb):
    p = W.custom(47, 0.5e-3, 24, 11e-3, 150, [[2.4e5, 3.1e5, 3.7e5]], seed=13)
    topts = W.resolve_trace_opts(p.geom, p.c_start, 150)
    f = p.freq_sets[0]
    _say("invert ragged 47x47 m=24 in place")
    ref = invert.invert_frequency_set(p.geom, topts, p.inv, p.c_start, p.alpha0, f, p.p_meas[0])
    c = _t(p.c_start.reshape(-1))
    rb.invert_frequency_set(p.geom, topts, p.inv, "f32", c, _t(p.alpha0.reshape(-1)), f,
                            _t(np.stack([p.p_meas[0].real, p.p_meas[0].imag], -1)), c)
    dc_g = c.cpu().numpy() - p.c_start.reshape(-1)
    dc_o = ref[0].reshape(-1) - p.c_start.reshape(-1)
    assert _rel(dc_g, dc_o) <= 1e-4


def test_invert_refuses_nonpositive_update(rb):
    """A point perturbation of -2/c^2 drives 1/c^2 negative: RB_ENUMERIC and
    the model is left unchanged (oracle raises too)."""
    g = W.centred_grid(33, 0.5e-3, 24, 12e-3, 1500.0)
    import dataclasses
    g = dataclasses.replace(g, support_margin=12e-3 - 0.25e-3)
    X, Y = g.pixel_centres()
    c = 1500.0 + 12.0 * np.exp(-((X - 2e-3) ** 2 + (Y + 1e-3) ** 2) / (2 * (3e-3) ** 2))
    al = np.full_like(c, 2.0)
    topts = W.resolve_trace_opts(g, c, 240)
    freqs = [2.5e5]
    T, A, B, Tr, Ar, Br = rays.tables(g, topts, 1.0 / c, al)
    G = born.green(T, A, B, freqs[0])
    p_model = born.green(Tr, Ar, Br, freqs[0])
    ic = (g.ny // 2) * g.nx + g.nx // 2
    e_c = np.zeros(g.n_pixels)
    e_c[ic] = -2.0 / c.reshape(-1)[ic] ** 2
    pm = p_model + born.born_forward(G, e_c, freqs[0], g.h ** 2)
    with pytest.raises(invert.NumericError):
        invert.invert_frequency_set(g, topts, W.InvertOpts(), c, al, freqs, pm[None])
    _say("invert numeric refusal")
    cin = _t(c.reshape(-1))
    cout = _t(np.zeros(g.n_pixels))
    with pytest.raises(rb.NumericError):
        rb.invert_frequency_set(g, topts, W.InvertOpts(), "f64", cin, _t(al.reshape(-1)), freqs,
                                _t(np.stack([pm.real, pm.imag], -1)[None]), cout)
    assert np.array_equal(cout.cpu().numpy(), c.reshape(-1))
