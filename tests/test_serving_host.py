"""Host-side pieces of the serving loop: the sequential baseline queue and
the workspace plan (no GPU needed)."""
import math

import numpy as np
import pytest

import workload as W

torch = pytest.importorskip("torch")


def _job(S, jid, arrival, cls=0, seed=2201, radius=0.1):
    p = W.serving_job(cls, seed, radius, with_data=False)
    topts = W.resolve_trace_opts(p.geom, p.c_start, p.trace.n_rays)
    return S.Job(jid=jid, arrival=arrival, geom=p.geom, topts=topts, inv=p.inv, dtype="f32", c_start=p.c_start,
                 alpha0=p.alpha0, freq_sets=p.freq_sets, p_meas=[], size_class=cls)


def test_sequential_baseline_is_a_fifo_queue():
    from paper_2511_16633_amd import serving as S
    jobs = [_job(S, i, a) for i, a in enumerate([0.0, 0.5, 0.6, 5.0])]
    out = S.sequential_baseline(jobs, [1.0, 1.0, 1.0, 0.5])
    # finish times 1.0, 2.0, 3.0, 5.5 -> latencies 1.0, 1.5, 2.4, 0.5
    lat = np.array([1.0, 1.5, 2.4, 0.5])
    assert math.isclose(out["p50_latency_s"], float(np.percentile(lat, 50)))
    assert math.isclose(out["makespan_s"], 5.5)


def test_plan_shrinks_the_emitter_batch_to_fit():
    pytest.importorskip("paper_2511_16633_amd")
    from paper_2511_16633_amd import serving as S
    import paper_2511_16633_amd as rb
    try:
        rb.lib()
    except Exception:
        pytest.skip("library not built")
    j = _job(S, 0, 0.0, cls=1)
    full = rb.invert_workspace_bytes(j.geom, j.topts, 3, "f32", 0)
    S.plan(j, full // 3)
    assert 0 < j.emitter_batch < j.geom.m
    assert j.ws_bytes <= full // 3
    assert j.footprint > j.ws_bytes
    assert j.units == 480 * 480 * 256 * (3 * 256 // 4 + 1) * 24
