"""Shared comparison for the GPU parity tests (no GPU code here).

``close(got, ref, tol)`` asserts both a relative L2 bound and a
per-element bound: rel-L2 <= tol and max |got - ref| <= c tol max |ref|,
so one wrong element (a ragged-tail pixel, a pair at a tile edge) cannot
hide inside a small L2 norm over many correct ones.
"""
import numpy as np

PER_ELEMENT_FACTOR = 5.0


def close(got, ref, tol, what="", c=PER_ELEMENT_FACTOR):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    scale = float(np.max(np.abs(ref)))
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    mx = float(np.max(np.abs(got - ref))) / scale
    print(f"[parity] {what}: rel-L2 {rel:.3e}, max|d|/max|ref| {mx:.3e} (bounds {tol:.1e}, {c * tol:.1e})",
          flush=True)
    assert rel <= tol, f"{what}: rel-L2 {rel:.3e} > {tol:.1e}"
    assert mx <= c * tol, f"{what}: max|d|/max|ref| {mx:.3e} > {c * tol:.1e}"
    return rel, mx
