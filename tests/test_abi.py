"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before touching a GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rayborn.h")

rb = pytest.importorskip("paper_2511_16633_amd")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 13
    L = rb.lib()
    for n in names:
        assert hasattr(L, n), n
    assert rb.version().startswith("rayborn")


def _declared_arity():
    """Parameter count of every entry point declared in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(rb_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", text):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_declares_every_symbol_with_its_arity():
    """The binding gives every declared entry point a restype and argtypes
    with as many arguments as the header declares (ctypes would otherwise
    pass untyped integers and pointers)."""
    L = rb.lib()
    arity = _declared_arity()
    assert set(arity) == set(_declared())
    sig = L.rb_signatures
    for name, n in arity.items():
        assert name in sig, f"{name} has no signature in the binding"
        assert len(sig[name][1]) == n, (name, len(sig[name][1]), n)
        assert getattr(L, name).argtypes is not None


def test_status_strings():
    L = rb.lib()
    assert L.rb_status_string(0) == b"ok"
    assert L.rb_status_string(-1) == b"invalid argument"
    assert L.rb_status_string(-5).startswith(b"non-positive")


def _geom(**kw):
    g = W.centred_grid(16, 1e-3, 8, 6e-3, 1500.0)
    import dataclasses
    return dataclasses.replace(g, **kw)


def test_workspace_sizes_are_positive_and_monotone():
    g = _geom()
    t = W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=2e-5, j_min=0.0)
    a = rb.trace_workspace_bytes(g, t, 1)
    b = rb.trace_workspace_bytes(g, t, 8)
    assert 0 < a < b
    assert rb.invert_workspace_bytes(g, t, 2, "f32") > b
    assert rb.adjoint_workspace_bytes(g, 2, "bf16") > 0
    assert rb.forward_workspace_bytes(g, 2, "f64") > 0
    bad = W.TraceOpts(n_rays=2, dtau=1e-7, tau_max=2e-5)
    assert rb.trace_workspace_bytes(g, bad, 1) == 0
    assert rb.invert_workspace_bytes(_geom(m=2), t, 2, "f32") == 0


def _call_trace(g, t, ws_bytes=1 << 20):
    L = rb.lib()
    from paper_2511_16633_amd._binding import RbTables, geometry_struct, trace_opts_struct
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: checks fail first
    tabs = RbTables(*(0x1000 for _ in range(6)))
    return L.rb_trace_rays(ctypes.byref(geometry_struct(g)), ctypes.byref(trace_opts_struct(t)), fake, None,
                           ctypes.byref(tabs), fake, ws_bytes, None)


@pytest.mark.parametrize("kw", [{"nx": 0}, {"h": -1.0}, {"m": 3}, {"ring_radius": 0.0}, {"c_background": 0.0}])
def test_invalid_geometry_is_rejected_on_host(kw):
    t = W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=2e-5)
    assert _call_trace(_geom(**kw), t) == -1
    assert len(rb.lib().rb_last_error()) > 0


@pytest.mark.parametrize("t", [W.TraceOpts(n_rays=2, dtau=1e-7, tau_max=2e-5),
                               W.TraceOpts(n_rays=30, dtau=0.0, tau_max=2e-5),
                               W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=1e-8)])
def test_invalid_trace_options_are_rejected_on_host(t):
    assert _call_trace(_geom(), t) == -1


def test_too_small_workspace_is_enomem():
    t = W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=2e-5)
    assert _call_trace(_geom(), t, ws_bytes=64) == -2
    assert b"too small" in rb.lib().rb_last_error()


def test_binding_raises_with_message():
    with pytest.raises(rb.RayBornError) as ei:
        rb._binding._check(-1)
    assert "invalid argument" in str(ei.value)
    with pytest.raises(rb.NumericError):
        rb._binding._check(-5)


@pytest.mark.parametrize("n_iter", [0, -3, 65])
def test_cg_iteration_count_is_checked_on_host(n_iter):
    g = _geom()
    t = W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=2e-5)
    L = rb.lib()
    from paper_2511_16633_amd._binding import _freqs, geometry_struct, invert_opts_struct, trace_opts_struct
    fa, nf = _freqs([2e5, 3e5])
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: checks fail first
    hist = (ctypes.c_double * 4)()
    out = ctypes.c_double(0.0)
    rc = L.rb_invert_frequency_set_cg(ctypes.byref(geometry_struct(g)), ctypes.byref(trace_opts_struct(t)),
                                      ctypes.byref(invert_opts_struct(W.InvertOpts(), "f32")), fake, None, fa,
                                      nf, fake, n_iter, fake, ctypes.byref(out), hist, fake, 1 << 30, None)
    assert rc == -1
    assert b"n_iter" in L.rb_last_error()


def test_cg_workspace_holds_the_single_step_workspace():
    g = _geom()
    t = W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=2e-5)
    a = rb.invert_workspace_bytes(g, t, 2, "bf16")
    b = rb.invert_cg_workspace_bytes(g, t, 2, "bf16")
    assert b >= a + 5 * 8 * g.nx * g.ny


def test_asymptotic_weights_refuse_16bit_on_host():
    g = _geom()
    t = W.TraceOpts(n_rays=30, dtau=1e-7, tau_max=2e-5)
    L = rb.lib()
    from paper_2511_16633_amd._binding import _freqs, geometry_struct, invert_opts_struct, trace_opts_struct
    fa, nf = _freqs([2e5])
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: checks fail first
    out = ctypes.c_double(0.0)
    rc = L.rb_invert_frequency_set_asymptotic(ctypes.byref(geometry_struct(g)), ctypes.byref(trace_opts_struct(t)),
                                              ctypes.byref(invert_opts_struct(W.InvertOpts(), "bf16")), fake, None,
                                              fa, nf, fake, fake, ctypes.byref(out), fake, 1 << 30, None)
    assert rc == -4
    assert rb.invert_asymptotic_workspace_bytes(g, t, 1, "bf16") == 0
    assert rb.invert_asymptotic_workspace_bytes(g, t, 1, "f32") > rb.invert_workspace_bytes(g, t, 1, "f32")


def test_misaligned_green_tables_are_rejected_on_host():
    g = _geom()
    L = rb.lib()
    from paper_2511_16633_amd._binding import _freqs, geometry_struct
    fa, nf = _freqs([2e5])
    ok, bad = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1008)   # never dereferenced: checks fail first
    rc = L.rb_born_forward(ctypes.byref(geometry_struct(g)), bad, ok, ok, 1, fa, nf, ok, ok, ok, 1 << 30, None)
    assert rc == -1 and "16-byte" in L.rb_last_error().decode()
    rc = L.rb_born_adjoint_weighted(ctypes.byref(geometry_struct(g)), ok, bad, ok, 1, fa, nf, ok, ok, ok, None,
                                    ok, 1 << 30, None)
    assert rc == -1 and "16-byte" in L.rb_last_error().decode()


def test_grouped_step_refuses_bad_counts():
    """rb_invert_frequency_sets_grouped: no jobs, or too many, is RB_EINVAL
    before any work (no GPU needed)."""
    from paper_2511_16633_amd import _binding as Bd
    L = rb.lib()
    arr = (Bd.RbSetJob * 1)()
    assert L.rb_invert_frequency_sets_grouped(arr, 0, None) == -1
    assert L.rb_invert_frequency_sets_grouped(None, 1, None) == -1
    assert L.rb_invert_frequency_sets_grouped(arr, 100000, None) == -1
    # a job with NULL geometry is refused by the per-job checks
    assert L.rb_invert_frequency_sets_grouped(arr, 1, None) == -1
