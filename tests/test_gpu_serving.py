"""Serving loop on the GPU: jobs of different ring sizes and contraction
types are served together - the small rings in grouped rounds of the batch
lanes (their backprojections in shared launches), the large ring on its own
stream - and every result is bit-for-bit the one the job gives alone, with
one batch lane and with four.  The mix holds a 16-bit job of the
large-ring class (1040 elements around a small grid, BF16 contractions with
the 128 x 128-tile forward), whose served image is also checked against the
FP64 oracle at equal accuracy (rel-L2 <= 1e-2, max |dc| <= 1 m/s)."""
import copy

import numpy as np
import pytest

import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def serving():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_16633_amd as rbm
    from paper_2511_16633_amd import serving as S
    rbm.lib()
    return S


_RING1040 = None


def _ring1040():
    """A large ring on a small grid (the 1024+-element class, cheap to check)."""
    global _RING1040
    if _RING1040 is None:
        _RING1040 = W.custom(44, 0.5e-3, 1040, 20e-3, 360, [[200e3, 250e3]], seed=9)
    return _RING1040


def _jobs(S):
    specs = [(0, 2101, 0.085), (0, 2102, 0.11), (1, 2103, 0.1), (0, 2104, 0.095), (0, 2105, 0.12), (0, 2106, 0.03),
             (2, None, None)]
    jobs = []
    for i, (cls, seed, radius) in enumerate(specs):
        p = W.serving_job(cls, seed, radius) if seed is not None else _ring1040()
        dtype = "f32" if seed is not None else "bf16"
        topts = W.resolve_trace_opts(p.geom, p.c_start, p.trace.n_rays)
        jobs.append(S.Job(jid=i, arrival=0.05 * i, geom=p.geom, topts=topts, inv=p.inv, dtype=dtype,
                          c_start=p.c_start, alpha0=p.alpha0, freq_sets=p.freq_sets, p_meas=p.p_meas,
                          size_class=cls))
    return jobs


def test_mixed_results_equal_alone(serving):
    S = serving
    print("[gpu-case] serving: 7 jobs alone, then mixed", flush=True)
    alone = _jobs(S)
    srv = S.Server(DEV, max_running=4, lanes=1, group_max_m=256)   # one batch lane: 64- and 256-element rings share rounds
    for j in alone:
        S.plan(j, srv.budget // 2)
        S.run_job(j, DEV)
    mixed = _jobs(S)
    stats = srv.run(mixed, realtime=False)
    assert stats["errors"] == 0, [j.error for j in mixed]
    print(f"[gpu-case] serving: {stats['grouped_rounds']} grouped rounds, up to {stats['max_jobs_per_round']} "
          f"jobs per round", flush=True)
    assert stats["grouped_rounds"] >= 8 and stats["max_jobs_per_round"] >= 2
    assert stats["max_ring_sizes_per_round"] >= 2   # 64- and 256-element rings in one grouped launch
    for a, b in zip(alone, mixed):
        assert a.result is not None and b.result is not None
        assert np.array_equal(a.result, b.result), f"job {a.jid} differs alone and mixed"
        assert a.norms == b.norms
        assert not np.array_equal(b.result, b.c_start.reshape(-1))   # the model was updated
    # the same stream with four batch lanes: still bitwise the jobs' alone results
    print("[gpu-case] serving: mixed, four batch lanes", flush=True)
    mixed4 = _jobs(S)
    stats4 = S.Server(DEV, max_running=4, lanes=4, group_max_m=256).run(mixed4, realtime=False)
    assert stats4["errors"] == 0, [j.error for j in mixed4]
    for a, b in zip(alone, mixed4):
        assert np.array_equal(a.result, b.result), f"job {a.jid} differs alone and with four lanes"
    # several jobs were on the device at once
    spans = sorted((j.t_admit, j.t_done) for j in mixed)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    # the served bf16 job against the FP64 oracle, at equal accuracy
    from oracle import invert
    j = mixed[-1]
    assert j.dtype == "bf16" and j.geom.m == 1040
    ref_c, _ = invert.invert_frequency_set(j.geom, j.topts, j.inv, j.c_start, j.alpha0, j.freq_sets[0], j.p_meas[0])
    dc_g = j.result - j.c_start.reshape(-1)
    dc_o = ref_c.reshape(-1) - j.c_start.reshape(-1)
    rel = float(np.linalg.norm(dc_g - dc_o) / np.linalg.norm(dc_o))
    mx = float(np.abs(dc_g - dc_o).max())
    print(f"[gpu-case] served bf16 ring1040 vs oracle: rel-L2 {rel:.3e}, max|dc diff| {mx:.3e} m/s", flush=True)
    assert rel <= 1e-2 and mx <= 1.0


def test_admission_respects_the_budget(serving):
    """A budget that holds one large-ish job at a time still serves every job,
    and jobs never overlap beyond the budget."""
    S = serving
    print("[gpu-case] serving: tight budget", flush=True)
    jobs = _jobs(S)
    for j in jobs:
        S.plan(j, 1 << 62)
    budget = max(j.footprint for j in jobs)
    srv = S.Server(DEV, budget_bytes=budget, max_running=8)
    stats = srv.run(jobs, realtime=False)
    assert stats["errors"] == 0
    events = sorted([(j.t_admit, j.footprint) for j in jobs] + [(j.t_done, -j.footprint) for j in jobs])
    used = 0
    for _, d in events:
        used += d
        assert used <= budget
