"""The no-allocation backprojection (rb_born_adjoint_weighted_noalloc): the
library's fixed per-GPU scratch in place of a caller workspace.

GPU: two calls in a row through the C ABI, the second on a smaller problem
(so it runs on the first call's leftover scratch), each bitwise equal to
rb_born_adjoint_weighted with a workspace on the same inputs.  CPU: a
problem whose workspace exceeds the fixed scratch is refused before any
work is enqueued."""
import ctypes
import dataclasses

import numpy as np
import pytest

import workload as W
from oracle import invert

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _geom(nx, ny, m):
    g = W.centred_grid(nx, 0.5e-3, m, 12e-3, 1500.0)
    return dataclasses.replace(g, ny=ny, y0=-0.5 * (ny - 1) * 0.5e-3)


def _inputs(rb, geom, nf, dtype, seed):
    T, A, B, _, _, _ = W.random_tables(geom, seed=seed)
    freqs = list(np.linspace(3e5, 9e5, nf))
    D = W.random_residual(nf, geom.m, seed + 1)
    mask = invert.receiver_mask(geom.m, 0.75).astype(np.float64)
    rng = np.random.default_rng(seed + 2)
    Wd = np.stack([mask * (rng.uniform(size=mask.shape) > 0.02) for _ in range(nf)])
    t = lambda a, d=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device=DEV)
    tabs = {"T": t(T), "amp": t(A, torch.float32), "att": t(B, torch.float32),
            "T_rx": t(np.zeros((geom.m, geom.m))), "amp_rx": t(np.zeros((geom.m, geom.m)), torch.float32),
            "att_rx": t(np.zeros((geom.m, geom.m)), torch.float32)}
    td = rb._binding.TORCH_DTYPES[rb.DTYPES[dtype]]
    Gr = torch.empty((nf, geom.m, geom.n_pixels), dtype=td, device=DEV)
    Gi = torch.empty_like(Gr)
    sc = torch.empty(nf, dtype=torch.float32, device=DEV)
    rb.build_green(geom, tabs, freqs, 1.0, dtype, Gr, Gi, sc)
    return Gr, Gi, sc, freqs, t(np.stack([D.real, D.imag], -1)), t(Wd)


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_point_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_16633_amd as rb
    rb.lib()
    cases = [((50, 21, 97), 2, "f32", True), ((37, 29, 40), 1, "bf16", False)]
    for (nx, ny, m), nf, dtype, with_h in cases:
        geom = _geom(nx, ny, m)
        print(f"[gpu-case] noalloc adjoint {dtype} nx={nx} ny={ny} m={m} nf={nf} hdiag={with_h}", flush=True)
        assert rb.adjoint_workspace_bytes(geom, nf, dtype) <= rb._binding.NOALLOC_SCRATCH_BYTES
        Gr, Gi, sc, freqs, dres, Wd = _inputs(rb, geom, nf, dtype, 500 + m)
        g_ref = torch.full((geom.n_pixels,), 0.25, dtype=torch.float64, device=DEV)
        h_ref = torch.full_like(g_ref, 0.5) if with_h else None
        g_na = g_ref.clone()
        h_na = None if h_ref is None else h_ref.clone()
        rb.born_adjoint_weighted(geom, Gr, Gi, sc, dtype, freqs, dres, Wd, g_ref, h_ref)
        rb.born_adjoint_weighted_noalloc(geom, Gr, Gi, sc, dtype, freqs, dres, Wd, g_na, h_na)
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_na.cpu().numpy()
        assert np.any(a != 0.25)
        assert np.array_equal(a, b), f"grad differs: max {np.abs(a - b).max():.3e}"
        if with_h:
            assert np.array_equal(h_ref.cpu().numpy(), h_na.cpu().numpy())


def test_noalloc_refuses_a_problem_beyond_its_scratch():
    """Host-side refusal (RB_ENOMEM, no GPU work): 1024 elements over 1100^2
    pixels and four frequencies need far more than the fixed scratch."""
    import paper_2511_16633_amd as rb
    from paper_2511_16633_amd import _binding as Bd
    geom = W.centred_grid(1100, 0.2e-3, 1024, 0.11, 1500.0)
    L = rb.lib()
    fa = (ctypes.c_double * 4)(3e5, 4e5, 5e5, 6e5)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: the call is refused first
    rc = L.rb_born_adjoint_weighted_noalloc(ctypes.byref(Bd.geometry_struct(geom)), fake, fake, fake, 2, fa, 4,
                                            fake, fake, fake, None, None)
    assert rc == -2   # RB_ENOMEM
    assert b"scratch" in L.rb_last_error()
