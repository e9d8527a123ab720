"""Host-side figures bench.py reports (no GPU): the selected-pair count and
the matrix-core work the backprojection kernels issue, against brute-force
loops."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("m", [64, 70, 256])
def test_selected_pairs_counts_the_weights(bench, m):
    w = bench.selection_weights(m, 0.75, 2)
    assert bench.selected_pairs(m, 0.75) == int((w[0] != 0).sum())
    assert (w[0] == w[1]).all() and (w[0] == w[0].T).all()


@pytest.mark.parametrize("m", [64, 70])
def test_issued_mfma_flop_brute_force(bench, m):
    rng = np.random.default_rng(3)
    w = bench.selection_weights(m, 0.75, 2)
    w[1][rng.random((m, m)) < 0.6] = 0.0   # a sparser second frequency
    n_pixels = 50
    for products in (3, 4):
        blocks = 0
        for k in range(2):
            for e0 in range(0, m, 32):
                for r0 in range(0, m, 32):
                    blocks += bool((w[k, e0:e0 + 32, r0:r0 + 32] != 0).any())
        expect = blocks * 32 * 32 * n_pixels * 2 * products
        assert bench.issued_mfma_flop(w, n_pixels, products) == expect
