"""Throughput of the ray-Born single-step inversion on one MI355X.

One step = the whole hot path over the 256-element / 480x480 workload: for
each of the 8 frequency sets (3 frequencies each, 0.3-1.25 MHz, low to
high) trace rays in the current model, build the ray tables and Green's
functions, form residual and data weights, run the weighted backprojection
with the Hessian diagonal, the forward operator for the step length, and
update the model.  Inputs are synthetic and resident in HBM before timing.

Metric: Born backprojection throughput in Gpixel.pair.freq/s =
N * P * F / t_step / 1e9 (N pixels, P selected emitter-receiver pairs,
F frequencies).  The roofline entry is for the dominant kernel, the fused
complex MFMA backprojection as the step runs it (gradient only; the step
takes the Hessian diagonal from band sums), at 8 flop per (pixel, pair,
frequency).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0}   # dense MFMA TFLOP/s
# HBM traffic of the backprojection kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a copy of known size.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_k_adjoint_f32_ring256_grid480.md")
ADJOINT_SOURCES = ["adjoint.hip", "mma.h", "born.h", "common.h"]
COPY_BYTES = 256 << 20   # calibration copy: reads and writes this many bytes once
METRIC = "Born backprojection Gpixel·pair·freq/s + recon latency p50/p99 vs plain"


def selected_pairs(m: int, recv_fraction: float) -> int:
    dmin = int(math.ceil((1.0 - recv_fraction) * 0.5 * m - 1e-9))
    return m * sum(1 for r in range(m) if min(r, m - r) >= dmin)


def selection_weights(m: int, recv_fraction: float, nf: int) -> np.ndarray:
    """Receiver-selection weights [nf][m][m] (timing input for the adjoint)."""
    dmin = int(math.ceil((1.0 - recv_fraction) * 0.5 * m - 1e-9))
    e = np.arange(m)[:, None]
    r = np.arange(m)[None, :]
    d = np.minimum(np.abs(e - r), m - np.abs(e - r))
    return np.repeat((d >= dmin).astype(np.float64)[None], nf, axis=0)


def adjoint_source_hash() -> str:
    h = hashlib.sha256()
    for name in ADJOINT_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_16633_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def issued_mfma_flop(w: np.ndarray, n_pixels: int, products: int) -> float:
    """Matrix-core flop one backprojection launch issues: the kernels skip a
    wave's 32 x 32 (emitter, receiver) block whose weights are all zero and
    compute the others whole, `products` real products of 2 flop per
    complex multiply-add."""
    nf, m, _ = w.shape
    mp = (m + 31) // 32 * 32
    wp = np.zeros((nf, mp, mp), bool)
    wp[:, :m, :m] = w != 0
    on = wp.reshape(nf, mp // 32, 32, mp // 32, 32).any(axis=(2, 4))
    return float(on.sum()) * 32 * 32 * n_pixels * 2 * products


def measured_traffic(dtype: str, workload: str):
    """HBM bytes per backprojection launch from the committed counter summary,
    or None when it is missing, for another dtype or workload, or the
    kernel's sources have changed since the counters were taken."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            kv = dict(line[2:].split(": ", 1) for line in f.read().splitlines() if line.startswith("- ") and ": " in line)
    except OSError:
        return None
    if (kv.get("source_sha256", "").strip() != adjoint_source_hash() or kv.get("dtype", "").strip() != dtype
            or kv.get("workload", "").strip() != workload):
        return None
    try:
        return int(kv["hbm_bytes_per_launch"].split()[0])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-reps", type=int, default=20)
    ap.add_argument("--workload", default="ring256_grid480", choices=["ring256_grid480", "ring1024_grid1100"],
                    help="ring256_grid480 (default, the measured workload) or the large instance")
    ap.add_argument("--emitter-batch", type=int, default=0, help="emitters traced per batch (0: all that fit)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop latency measurement")
    ap.add_argument("--serving-jobs", type=int, default=24)
    ap.add_argument("--cg-iters", type=int, default=10,
                    help="CG iterations for the CG-solved set timing (0: skip)")
    ap.add_argument("--tof-iters", type=int, default=3,
                    help="iterations of the ToF starting-model timing (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2511_16633_amd as rb
    import workload as W

    dev = "cuda:0"
    t0 = time.time()
    large = args.workload == "ring1024_grid1100"
    prob = W.breast_ring1024(dtype=args.dtype) if large else W.breast_ring256(dtype=args.dtype)
    batch = args.emitter_batch or (128 if large else 0)
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    print(f"[bench] inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    c_start = torch.as_tensor(prob.c_start.reshape(-1), device=dev)
    alpha = torch.as_tensor(prob.alpha0.reshape(-1), device=dev)
    pms = [torch.as_tensor(np.stack([p.real, p.imag], -1), device=dev) for p in prob.p_meas]
    nf_max = max(len(f) for f in prob.freq_sets)
    ws = torch.empty(rb.invert_workspace_bytes(g, topts, nf_max, args.dtype, batch), dtype=torch.uint8, device=dev)
    c = torch.empty_like(c_start)
    stream = torch.cuda.current_stream()

    def step():
        c.copy_(c_start)
        hist = []
        for fs, pm in zip(prob.freq_sets, pms):
            hist.append(rb.invert_frequency_set(g, topts, prob.inv, args.dtype, c, alpha, fs, pm, c, ws=ws,
                                                stream=stream))
        return hist

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        hist = step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    N, P = g.n_pixels, selected_pairs(g.m, prob.inv.recv_fraction)
    F = sum(len(f) for f in prob.freq_sets)
    units = N * P * F
    value = units / (ms_per_step * 1e-3) / 1e9
    print(f"[bench] {ms_per_step:.1f} ms/step, update norms {['%.2f' % h for h in hist]}", file=sys.stderr,
          flush=True)

    # ---- dominant kernel: the weighted backprojection, timed per launch with
    # events on the stream the library launches on.
    fs = prob.freq_sets[0]
    nf = len(fs)
    tabs = rb.alloc_tables(g, dev)
    s = (1.0 / c_start).contiguous()
    del ws   # the sweep's workspace; the stage timings below use their own
    tws = torch.empty(rb.trace_workspace_bytes(g, topts, batch), dtype=torch.uint8, device=dev)
    rb.trace_rays(g, topts, s, alpha, tabs, ws=tws, stream=stream)
    td = rb._binding.TORCH_DTYPES[rb.DTYPES[args.dtype]]
    Gr = torch.empty((nf, g.m, N), dtype=td, device=dev)
    Gi = torch.empty_like(Gr)
    sc = torch.empty(nf, dtype=torch.float32, device=dev)
    rb.build_green(g, tabs, fs, prob.inv.y_pow, args.dtype, Gr, Gi, sc, stream=stream)
    Wd = torch.as_tensor(selection_weights(g.m, prob.inv.recv_fraction, nf), device=dev)
    grad = torch.zeros(N, dtype=torch.float64, device=dev)
    hd = torch.zeros(N, dtype=torch.float64, device=dev)
    aws = torch.empty(rb.adjoint_workspace_bytes(g, nf, args.dtype), dtype=torch.uint8, device=dev)
    for _ in range(3):
        rb.born_adjoint_weighted(g, Gr, Gi, sc, args.dtype, fs, pms[0], Wd, grad, None, ws=aws, stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.adjoint_reps):
        rb.born_adjoint_weighted(g, Gr, Gi, sc, args.dtype, fs, pms[0], Wd, grad, None, ws=aws, stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    adj_ms = ev0.elapsed_time(ev1) / args.adjoint_reps
    flops = 8.0 * N * P * nf
    achieved = flops / (adj_ms * 1e-3) / 1e12
    esize = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[args.dtype]
    alg_bytes = 2 * nf * g.m * N * esize + nf * N * 8   # G (re, im) once + per-frequency gradient partials
    issued = issued_mfma_flop(Wd.cpu().numpy(), N, 3 if args.dtype == "f32" else 4) if args.dtype != "f64" else None
    kname = {"f32": "k_adjoint_f32", "bf16": "k_adjoint16_lds", "f16": "k_adjoint16_lds", "f64": "k_adjoint"}[args.dtype]
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[args.dtype], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK[args.dtype], 4), "traffic": measured_traffic(args.dtype, args.workload),
                "kernel": kname + " (fused complex backprojection, gradient as the step runs it)",
                "launch_ms": round(adj_ms, 4), "algorithmic_flop_per_launch": flops,
                "algorithmic_bytes_per_launch": alg_bytes,
                "mfma_issued": None if issued is None else {
                                "flop_per_launch": issued,
                                "frac": round(issued / (adj_ms * 1e-3) / 1e12 / PEAK[args.dtype], 4),
                                "what": "real matrix-core work the kernel issues: 32-emitter x 32-receiver blocks "
                                        "with a nonzero weight (unselected pairs inside them carry weight 0), "
                                        "3 real products per complex MAC in FP32, 4 in 16-bit"}}

    # ---- calibration copy for the traffic counters (outside every timed region)
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst

    # ---- stage times for one set (events, same stream)
    def timed(fn, reps=3):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / reps

    dmin = int(math.ceil((1.0 - prob.inv.recv_fraction) * 0.5 * g.m - 1e-9))
    fws = torch.empty(rb.forward_workspace_bytes(g, nf, args.dtype), dtype=torch.uint8, device=dev)
    dout = torch.empty((nf, g.m, g.m, 2), dtype=torch.float64, device=dev)
    stages = {
        "trace_rays": timed(lambda: rb.trace_rays(g, topts, s, alpha, tabs, ws=tws, stream=stream)),
        "build_green": timed(lambda: rb.build_green(g, tabs, fs, prob.inv.y_pow, args.dtype, Gr, Gi, sc,
                                                    stream=stream)),
        "born_adjoint_weighted": adj_ms,
        "born_adjoint_weighted+hdiag": timed(lambda: rb.born_adjoint_weighted(g, Gr, Gi, sc, args.dtype, fs, pms[0],
                                                                              Wd, grad, hd, ws=aws, stream=stream)),
        "born_hessian_banded": timed(lambda: rb.born_hessian_banded(g, Gr, Gi, sc, args.dtype, fs, dmin, None, None,
                                                                    hd, stream=stream)),
        "born_forward": timed(lambda: rb.born_forward(g, Gr, Gi, sc, args.dtype, fs, grad, dout, ws=fws,
                                                      stream=stream)),
    }
    stages = {k: round(v, 3) for k, v in stages.items()}

    # ---- the linear subproblem of set 0 solved by CG instead of the single
    # step: whole set (trace, tables, CG) for 1 and for K iterations
    cg = None
    if args.cg_iters > 0 and not large:
        del fws
        cws = torch.empty(rb.invert_cg_workspace_bytes(g, topts, nf, args.dtype, batch), dtype=torch.uint8,
                          device=dev)
        ccg = torch.empty_like(c_start)

        def cg_set(k):
            ccg.copy_(c_start)
            return rb.invert_frequency_set_cg(g, topts, prob.inv, args.dtype, ccg, alpha, fs, pms[0], k, ccg,
                                              ws=cws, stream=stream)

        def one_set():
            ccg.copy_(c_start)
            return rb.invert_frequency_set(g, topts, prob.inv, args.dtype, ccg, alpha, fs, pms[0], ccg, ws=cws,
                                           stream=stream)

        t_one = timed(one_set)
        t_1 = timed(lambda: cg_set(1))
        t_k = timed(lambda: cg_set(args.cg_iters))
        _, alphas, rzs = cg_set(args.cg_iters)
        # algorithmic work of one extra iteration: the weighted adjoint
        # (8 flop per pixel, selected pair, frequency) and the forward over the
        # selected pairs, symmetric in e and r (4 flop per unit)
        t_it = (t_k - t_1) / max(args.cg_iters - 1, 1)
        it_flop = 12.0 * N * P * nf
        cg = {"iters": args.cg_iters, "ms_per_set": round(t_k, 3), "ms_per_set_one_iteration": round(t_1, 3),
              "ms_per_set_single_step": round(t_one, 3),
              "ms_per_extra_iteration": round(t_it, 3),
              "iteration_tflops": round(it_flop / (t_it * 1e-3) / 1e12, 3),
              "iteration_frac": round(it_flop / (t_it * 1e-3) / 1e12 / PEAK[args.dtype], 4),
              "rz_first_last": [rzs[0], rzs[-1]]}
        print(f"[bench] CG set 0: {args.cg_iters} iterations {t_k:.2f} ms, 1 iteration {t_1:.2f} ms, "
              f"single step {t_one:.2f} ms", file=sys.stderr, flush=True)
        del cws
        # the same set with the asymptotic (amplitude-normalised) weights
        if args.dtype in ("f32", "f64"):
            asws = torch.empty(rb.invert_asymptotic_workspace_bytes(g, topts, nf, args.dtype, batch),
                               dtype=torch.uint8, device=dev)

            def asym_set():
                ccg.copy_(c_start)
                return rb.invert_frequency_set_asymptotic(g, topts, prob.inv, args.dtype, ccg, alpha, fs, pms[0],
                                                          ccg, ws=asws, stream=stream)

            t_as = timed(asym_set)
            cg["asymptotic_weights_ms_per_set"] = round(t_as, 3)
            print(f"[bench] asymptotic weights set 0: {t_as:.2f} ms", file=sys.stderr, flush=True)
            del asws
        del ccg
        fws = None

    # ---- the ToF starting model: bent-ray ToF inversion from water against
    # straight-chord ToFs of the true phantom (the stand-in for picked ToFs)
    tof = None
    # (the large instance's fans, all resident at once, would not fit)
    if args.tof_iters > 0 and not large:
        T_meas = torch.as_tensor(W.straight_ray_tof(g, prob.c_true), device=dev)
        c_w = torch.full_like(c_start, g.c_background)
        c_t = torch.empty_like(c_start)
        tws_tof = torch.empty(rb.tof_workspace_bytes(g, topts), dtype=torch.uint8, device=dev)
        rb.tof_invert(g, topts, prob.inv, c_w, T_meas, 1, c_t, ws=tws_tof, stream=stream)   # warm-up
        t_tof = timed(lambda: rb.tof_invert(g, topts, prob.inv, c_w, T_meas, args.tof_iters, c_t, ws=tws_tof,
                                            stream=stream), reps=2)
        rms, betas = rb.tof_invert(g, topts, prob.inv, c_w, T_meas, args.tof_iters, c_t, ws=tws_tof, stream=stream)
        ct = torch.as_tensor(prob.c_true.reshape(-1), device=dev)
        err0 = float(torch.linalg.vector_norm(c_w - ct)) / math.sqrt(N)
        err1 = float(torch.linalg.vector_norm(c_t - ct)) / math.sqrt(N)
        tof = {"iters": args.tof_iters, "ms": round(t_tof, 3), "ms_per_iteration": round(t_tof / args.tof_iters, 3),
               "rms_tof_residual_s": [float("%.4g" % r) for r in rms],
               "rms_speed_error_m_s": [round(err0, 3), round(err1, 3)]}
        # the whole reconstruction: ToF start, then the 8-set sweep from it,
        # next to the sweep from the smoothed-truth start the step is timed on
        del tws_tof
        sws = torch.empty(rb.invert_workspace_bytes(g, topts, nf_max, args.dtype, batch), dtype=torch.uint8,
                          device=dev)
        c_s = torch.empty_like(c_start)

        def sweep(c0):
            c_s.copy_(c0)
            for fs_k, pm_k in zip(prob.freq_sets, pms):
                rb.invert_frequency_set(g, topts, prob.inv, args.dtype, c_s, alpha, fs_k, pm_k, c_s, ws=sws,
                                        stream=stream)
            return float(torch.linalg.vector_norm(c_s - ct)) / math.sqrt(N)

        try:
            t0p = time.perf_counter()
            tws_tof = torch.empty(rb.tof_workspace_bytes(g, topts), dtype=torch.uint8, device=dev)
            rb.tof_invert(g, topts, prob.inv, c_w, T_meas, args.tof_iters, c_t, ws=tws_tof, stream=stream)
            del tws_tof
            e_tof = sweep(c_t)
            torch.cuda.synchronize()
            t_pipe = (time.perf_counter() - t0p) * 1e3
            e_ref = sweep(c_start)
            tof["pipeline"] = {"ms": round(t_pipe, 1),
                               "what": "ToF start from water, then the 8-set sweep (workspace allocation included)",
                               "rms_speed_error_m_s": {"after_sweep_from_tof_start": round(e_tof, 3),
                                                       "after_sweep_from_smoothed_truth": round(e_ref, 3)}}
            print(f"[bench] pipeline ToF + sweep {t_pipe:.1f} ms; speed error after the sweep {e_tof:.2f} m/s "
                  f"(smoothed-truth start: {e_ref:.2f})", file=sys.stderr, flush=True)
        except rb.RayBornError as exc:   # reported, the measured line still prints
            tof["pipeline"] = {"error": str(exc)}
        del sws, c_s
        print(f"[bench] ToF start: {args.tof_iters} iterations {t_tof:.2f} ms, rms residual "
              f"{rms[0]:.3g} -> {rms[-1]:.3g} s, speed error {err0:.2f} -> {err1:.2f} m/s", file=sys.stderr,
              flush=True)
        del T_meas, c_w, c_t, ct

    out = {"metric": METRIC, "value": round(value, 3), "unit": "Gpixel·pair·freq/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
           "data": "synthetic (seeded breast phantom, straight-ray measured-data stand-in)",
           "config": {"workload": (("ring1024_grid1100: 1024-element ring R=110 mm, 1100x1100 grid at 0.2 mm, "
                                   "12 sets x 4 frequencies 0.3-2.0 MHz low to high, 1440 rays/emitter, ")
                                  if large else
                                  ("ring256_grid480: 256-element ring R=110 mm, 480x480 grid at 0.5 mm, "
                                   "8 sets x 3 frequencies 0.3-1.25 MHz low to high, 720 rays/emitter, "))
                                 + "FP64 rays/phase, " + args.dtype + " contractions",
                      "pixels": N, "selected_pairs": P, "frequencies": F, "pixel_pair_freq_per_step": units},
           "roofline": roofline, "stages_ms_per_set": stages}
    if cg is not None:
        out["cg"] = cg
    if tof is not None:
        out["tof"] = tof

    if large:
        out["config"]["emitter_batch"] = batch
    if not args.no_serving and not large:
        del tabs, Gr, Gi, sc, Wd, grad, hd, aws, tws, fws, dout, pms, c, c_start, alpha
        torch.cuda.empty_cache()
        try:
            out["serving"] = serving_report(dev, args.serving_jobs)
        except Exception as exc:   # reported, the measured line still prints
            out["serving"] = {"error": f"{type(exc).__name__}: {exc}"}
    if not args.no_cpu_baseline and not large:
        out["cpu_baseline"] = cpu_baseline(prob, topts, P)
    print(json.dumps(out), flush=True)


# Contraction type per serving size class: FP32 for the 64- and 256-element
# jobs, BF16 (FP32 accumulation, FP64 phase) for the 1024-element jobs, as
# the large instance is specified.
SERVING_DTYPES = ("f32", "f32", "bf16")


def serving_report(dev, n_jobs):
    """Latency of the serving loop on a Poisson stream (0.5 jobs/s, sizes
    64/256/1024 elements in the ratio 5:4:1; contraction type per class as
    in SERVING_DTYPES), against the same jobs run one at a time in plain
    FP32 (sequential baseline)."""
    import copy
    import torch
    import workload as W
    from paper_2511_16633_amd import serving as S
    t = time.time()
    specs = W.serving_stream(n_jobs)
    jobs = []
    for sp in specs:
        p = W.serving_job(sp["size_class"], sp["seed"], sp["ring_radius"])
        topts = W.resolve_trace_opts(p.geom, p.c_start, p.trace.n_rays)
        jobs.append(S.Job(jid=sp["job"], arrival=sp["arrival_s"], geom=p.geom, topts=topts, inv=p.inv,
                          dtype=SERVING_DTYPES[sp["size_class"]], c_start=p.c_start, alpha0=p.alpha0,
                          freq_sets=p.freq_sets, p_meas=p.p_meas, size_class=sp["size_class"]))
    print(f"[bench] serving: {n_jobs} jobs generated in {time.time() - t:.1f} s", file=sys.stderr, flush=True)
    srv = S.Server(dev, max_running=4)
    mixed = srv.run(jobs, realtime=True)
    print(f"[bench] serving: stream served, p50 {mixed['p50_latency_s']:.3f} s, p99 {mixed['p99_latency_s']:.3f} s",
          file=sys.stderr, flush=True)
    service, same = [], True
    for j in jobs:
        # alone, as served (bitwise check), then alone in plain FP32 (baseline)
        a = copy.copy(j)
        a.result = None
        torch.cuda.synchronize()
        t = time.perf_counter()
        S.run_job(a, dev)
        t_alone = time.perf_counter() - t
        same = same and a.result is not None and j.result is not None and bool(np.array_equal(a.result, j.result))
        if j.dtype != "f32":
            a = copy.copy(j)
            a.result = None
            a.dtype = "f32"
            S.plan(a, srv.budget // 2)
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.run_job(a, dev)
            t_alone = time.perf_counter() - t
        service.append(t_alone)
    seq = S.sequential_baseline(jobs, service)
    counts = [sum(1 for j in jobs if j.size_class == c) for c in range(3)]
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    return {"stream": f"Poisson 0.5 jobs/s, {n_jobs} jobs, seed 42; ring64_grid128 / ring256_grid480 / "
                      f"ring1024_grid1100 = {counts[0]} / {counts[1]} / {counts[2]}; ring radius 80-120 mm; "
                      f"served in {' / '.join(SERVING_DTYPES)}, baseline plain f32 one job at a time",
            "budget_gib": round(srv.budget / 2**30, 1), "max_running": srv.max_running,
            "served": rnd(mixed), "sequential_plain": rnd(seq), "same_alone_and_mixed": same}


def cpu_baseline(prob, topts, P):
    """The FP64 oracle, as it stands, on the first two frequency sets of the
    same workload (the second starts from the first's image, as in the
    sweep)."""
    from oracle import invert
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas = 1
    omp = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t = time.perf_counter()
    c = prob.c_start
    nfreq = 0
    for s in range(2):
        c, _ = invert.invert_frequency_set(prob.geom, topts, prob.inv, c, prob.alpha0, prob.freq_sets[s],
                                           prob.p_meas[s])
        nfreq += len(prob.freq_sets[s])
    dt = time.perf_counter() - t
    units = prob.geom.n_pixels * P * nfreq
    return {"value": round(units / dt / 1e9, 4), "unit": "Gpixel·pair·freq/s",
            "cores": max(blas, omp), "kind": "oracle",
            "sample": f"the first two frequency sets ({nfreq} of 24 frequencies) of the same workload, "
                      f"full grid and ring; {dt:.1f} s"}


if __name__ == "__main__":
    main()
