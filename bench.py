"""Throughput of the ray-Born single-step inversion on one MI355X.

Workload (default): the large instance, ring1024_grid1100 - a 1024-element
ring of radius 110 mm around a 1100 x 1100 grid at 0.2 mm, breast phantom
with microcalcifications, 12 frequency sets of 4 frequencies (0.3-2.0 MHz),
1440 rays per element, FP32 contractions with FP64 travel times and phase.

One step = one linearised frequency set, the hot path's unit: trace rays in
the current model, build the ray tables and Green's functions, form residual
and data weights, run the weighted backprojection and the Hessian diagonal,
the forward operator for the step length, and update the model.  Steps take
the sets in sweep order, low to high frequency, each starting from the
previous set's model (after the last set the sweep restarts from the start
model).  Inputs are synthetic and resident in HBM before timing.

Metric: Born backprojection throughput in Gpixel.pair.freq/s =
N * P * F / t_step / 1e9 (N pixels, P selected emitter-receiver pairs, F
frequencies of the set).  The roofline entry is for the dominant kernel,
the fused complex MFMA backprojection as the step runs it (gradient only;
the step takes the Hessian diagonal from band sums), at 8 flop per (pixel,
pair, frequency).

Extra legs (keys beside the headline): the same workload with BF16
contractions; the 256-element / 480 x 480 workload's whole 8-set sweep; the
CG-solved set, the asymptotic weights and the ToF starting model on that
workload; the serving loop on a Poisson stream of mixed jobs.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload ...]
                       [--no-cpu-baseline] [--no-serving] [--no-extras]
"""
from __future__ import annotations

import argparse
import copy
import hashlib
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0}   # dense MFMA TFLOP/s
# HBM traffic of the backprojection kernel per workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a copy
# of known size.
TRAFFIC_SUMMARIES = {
    "ring1024_grid1100": os.path.join(ROOT, "profiles", "hbm_traffic_k_adjoint_f32_ring1024_grid1100.md"),
    "ring256_grid480": os.path.join(ROOT, "profiles", "hbm_traffic_k_adjoint_f32_ring256_grid480.md"),
}
ADJOINT_SOURCES = ["adjoint.hip", "mma.h", "born.h", "common.h"]
COPY_BYTES = 256 << 20   # calibration copy: reads and writes this many bytes once
METRIC = "Born backprojection Gpixel·pair·freq/s + recon latency p50/p99 vs plain"
UNIT = "Gpixel·pair·freq/s"
WORKLOADS = {
    "ring1024_grid1100": ("1024-element ring R=110 mm, 1100x1100 grid at 0.2 mm, breast phantom with "
                          "microcalcifications, 12 sets x 4 frequencies 0.3-2.0 MHz, 1440 rays/emitter"),
    "ring256_grid480": ("256-element ring R=110 mm, 480x480 grid at 0.5 mm, breast phantom, "
                        "8 sets x 3 frequencies 0.3-1.25 MHz, 720 rays/emitter"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def zeroed_pairs(m: int, recv_fraction: float, outlier_fraction: float, nf: int, seed: int = 3):
    """Per frequency, floor(outlier_fraction x selected pairs) seeded random
    selected (e, r) pairs: the zeroed-pair list of the step's Hessian
    diagonal in shape and count (timing input), [nf][zcap][2] and [nf]."""
    dmin = int(math.ceil((1.0 - recv_fraction) * 0.5 * m - 1e-9))
    e = np.arange(m)[:, None]
    r = np.arange(m)[None, :]
    d = np.minimum(np.abs(e - r), m - np.abs(e - r))
    idx = np.flatnonzero(d >= dmin)
    nz = int(math.floor(outlier_fraction * idx.size))
    rng = np.random.default_rng(seed)
    zl = np.zeros((nf, max(nz, 1), 2), np.int32)
    for k in range(nf):
        z = np.sort(rng.choice(idx, size=nz, replace=False))
        zl[k, :nz, 0] = z // m
        zl[k, :nz, 1] = z % m
    return zl, np.full(nf, nz, np.int32)


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
    path = TRAFFIC_SUMMARIES.get(workload)
    try:
        with open(path) as f:
            kv = dict(line[2:].split(": ", 1) for line in f.read().splitlines() if line.startswith("- ") and ": " in line)
    except (OSError, TypeError):
        return None
    if (kv.get("source_sha256", "").strip() != adjoint_source_hash() or kv.get("dtype", "").strip() != dtype
            or kv.get("workload", "").strip() != workload):
        return None
    try:
        return int(kv["hbm_bytes_per_launch"].split()[0])
    except (KeyError, ValueError):
        return None


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle uses: OpenMP in the C tracer, BLAS in NumPy."""
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas = 1
    omp = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return max(blas, omp)


def load_problem(workload: str, dtype: str):
    import workload as W
    return W.breast_ring1024(dtype=dtype) if workload == "ring1024_grid1100" else W.breast_ring256(dtype=dtype)


class Sweep:
    """Device-resident inputs of one workload and its frequency-set steps."""

    def __init__(self, prob, dtype, batch, dev):
        import torch
        import paper_2511_16633_amd as rb
        import workload as W
        self.rb, self.torch = rb, torch
        self.prob, self.dtype, self.batch = prob, dtype, batch
        self.g = prob.geom
        self.topts = W.resolve_trace_opts(self.g, prob.c_start, prob.trace.n_rays)
        self.c_start = torch.as_tensor(prob.c_start.reshape(-1), device=dev)
        self.alpha = torch.as_tensor(prob.alpha0.reshape(-1), device=dev)
        self.pms = [torch.as_tensor(np.stack([p.real, p.imag], -1), device=dev) for p in prob.p_meas]
        nf_max = max(len(f) for f in prob.freq_sets)
        self.ws = torch.empty(rb.invert_workspace_bytes(self.g, self.topts, nf_max, dtype, batch),
                              dtype=torch.uint8, device=dev)
        self.c = self.c_start.clone()
        self.stream = torch.cuda.current_stream()
        self.next_set = 0
        self.norms = []

    def set_step(self):
        """One frequency set in sweep order (the model carried between sets)."""
        k = self.next_set
        if k == 0:
            self.c.copy_(self.c_start)
        fs = self.prob.freq_sets[k]
        n = self.rb.invert_frequency_set(self.g, self.topts, self.prob.inv, self.dtype, self.c, self.alpha, fs,
                                         self.pms[k], self.c, ws=self.ws, stream=self.stream)
        self.norms.append(n)
        self.next_set = (k + 1) % len(self.prob.freq_sets)
        return n

    def sweep(self):
        """The whole sweep from the start model."""
        self.next_set = 0
        for _ in self.prob.freq_sets:
            self.set_step()

    def release_workspace(self):
        """Frees the step's workspace (the stage timings bring their own)."""
        self.ws = None
        self.torch.cuda.empty_cache()

    def release(self):
        del self.ws, self.pms, self.c, self.c_start, self.alpha


def timed_events(torch, stream, fn, reps=3, warm=1):
    for _ in range(warm):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def backprojection_roofline(sw: Sweep, reps: int, workload: str, stages: bool):
    """Average duration of the step's backprojection launch (gradient only,
    set 0's frequencies) with HIP events on the launch stream, its roofline
    entry, and optionally the other entry points' times for one set."""
    rb, torch = sw.rb, sw.torch
    g, prob, dtype, stream = sw.g, sw.prob, sw.dtype, sw.stream
    dev = sw.c.device
    fs = prob.freq_sets[0]
    nf = len(fs)
    N, P = g.n_pixels, selected_pairs(g.m, prob.inv.recv_fraction)
    tabs = rb.alloc_tables(g, dev)
    s = (1.0 / sw.c_start).contiguous()
    tws = torch.empty(rb.trace_workspace_bytes(g, sw.topts, sw.batch), dtype=torch.uint8, device=dev)
    rb.trace_rays(g, sw.topts, s, sw.alpha, tabs, ws=tws, stream=stream)
    td = rb._binding.TORCH_DTYPES[rb.DTYPES[dtype]]
    Gr = torch.empty((nf, g.m, N), dtype=td, device=dev)
    Gi = torch.empty_like(Gr)
    sc = torch.empty(nf, dtype=torch.float32, device=dev)
    rb.build_green(g, tabs, fs, prob.inv.y_pow, dtype, Gr, Gi, sc, stream=stream)
    Wd = torch.as_tensor(selection_weights(g.m, prob.inv.recv_fraction, nf), device=dev)
    grad = torch.zeros(N, dtype=torch.float64, device=dev)
    hd = torch.zeros(N, dtype=torch.float64, device=dev)
    aws = torch.empty(rb.adjoint_workspace_bytes(g, nf, dtype), dtype=torch.uint8, device=dev)
    adj = lambda: rb.born_adjoint_weighted(g, Gr, Gi, sc, dtype, fs, sw.pms[0], Wd, grad, None, ws=aws,
                                           stream=stream)
    adj_ms = timed_events(torch, stream, adj, reps=reps, warm=2)
    flops = 8.0 * N * P * nf
    achieved = flops / (adj_ms * 1e-3) / 1e12
    esize = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[dtype]
    alg_bytes = 2 * nf * g.m * N * esize + nf * N * 8   # G (re, im) once + per-frequency gradient partials
    issued = issued_mfma_flop(Wd.cpu().numpy(), N, 3 if dtype == "f32" else 4) if dtype != "f64" else None
    kname = {"f32": "k_adjoint_f32", "bf16": "k_adjoint16_tr", "f16": "k_adjoint16_tr", "f64": "k_adjoint"}[dtype]
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[dtype], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[dtype], 4), "traffic": measured_traffic(dtype, workload),
            "kernel": kname + " (fused complex backprojection, gradient as the step runs it)",
            "launch_ms": round(adj_ms, 4), "launches_timed": reps,
            "algorithmic_flop_per_launch": flops, "algorithmic_bytes_per_launch": alg_bytes,
            "unit_of_work": f"{N} pixels x {P} selected pairs x {nf} frequencies, 8 flop each",
            "mfma_issued": None if issued is None else {
                "flop_per_launch": issued,
                "frac": round(issued / (adj_ms * 1e-3) / 1e12 / PEAK[dtype], 4),
                "what": "real matrix-core work the kernel issues: 32-emitter x 32-receiver blocks with a nonzero "
                        "weight (unselected pairs inside them carry weight 0), 3 real products per complex MAC "
                        "in FP32, 4 in 16-bit"}}
    st = None
    if stages:
        dmin = int(math.ceil((1.0 - prob.inv.recv_fraction) * 0.5 * g.m - 1e-9))
        zl, nzero = zeroed_pairs(g.m, prob.inv.recv_fraction, prob.inv.outlier_fraction, nf)
        zl, nzero = torch.as_tensor(zl, device=dev), torch.as_tensor(nzero, device=dev)
        fws = torch.empty(rb.forward_workspace_bytes(g, nf, dtype), dtype=torch.uint8, device=dev)
        dout = torch.empty((nf, g.m, g.m, 2), dtype=torch.float64, device=dev)
        st = {
            "trace_rays": timed_events(torch, stream, lambda: rb.trace_rays(g, sw.topts, s, sw.alpha, tabs, ws=tws,
                                                                            stream=stream)),
            "build_green": timed_events(torch, stream, lambda: rb.build_green(g, tabs, fs, prob.inv.y_pow, dtype,
                                                                              Gr, Gi, sc, stream=stream)),
            "born_adjoint_weighted": adj_ms,
            "born_adjoint_weighted+hdiag": timed_events(torch, stream, lambda: rb.born_adjoint_weighted(
                g, Gr, Gi, sc, dtype, fs, sw.pms[0], Wd, grad, hd, ws=aws, stream=stream), reps=2),
            "born_hessian_banded": timed_events(torch, stream, lambda: rb.born_hessian_banded(
                g, Gr, Gi, sc, dtype, fs, dmin, zl, nzero, hd, stream=stream)),
            "born_forward": timed_events(torch, stream, lambda: rb.born_forward(g, Gr, Gi, sc, dtype, fs, grad, dout,
                                                                                ws=fws, stream=stream), reps=2),
        }
        st = {k: round(v, 3) for k, v in st.items()}
        del fws, dout, zl, nzero
    del tabs, tws, Gr, Gi, sc, Wd, grad, hd, aws
    torch.cuda.empty_cache()
    return roof, st


def calibration_copy(torch, dev):
    """Copy of known size for scaling the traffic counters (outside every
    timed region)."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def headline(args, dev):
    import torch
    t0 = time.time()
    prob = load_problem(args.workload, args.dtype)
    large = args.workload == "ring1024_grid1100"
    # the headline step traces 512 emitters per batch (98.5 GiB of its
    # workspace; 128 per batch: 24.6 GiB, trace_rays about 5 ms slower)
    batch = args.emitter_batch or (512 if large else 0)
    log(f"{args.workload}: inputs generated in {time.time() - t0:.1f} s")
    sw = Sweep(prob, args.dtype, batch, dev)
    for _ in range(args.warmup):
        sw.set_step()
    torch.cuda.synchronize()
    log("warmup done")
    first = sw.next_set
    t1 = time.perf_counter()
    for _ in range(args.steps):
        sw.set_step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    g = sw.g
    N, P = g.n_pixels, selected_pairs(g.m, prob.inv.recv_fraction)
    nsets = len(prob.freq_sets)
    timed_sets = [(first + i) % nsets for i in range(args.steps)]
    F_timed = sum(len(prob.freq_sets[k]) for k in timed_sets)
    units = N * P * F_timed / args.steps
    value = units / (ms_per_step * 1e-3) / 1e9
    log(f"{ms_per_step:.1f} ms/step (one frequency set), {value:.1f} {UNIT}")
    sw.release_workspace()   # the stage timings allocate their own buffers
    roof, stages = backprojection_roofline(sw, args.adjoint_reps, args.workload, stages=True)
    calibration_copy(torch, dev)
    sw.release()
    del sw
    torch.cuda.empty_cache()
    out = {"metric": METRIC, "value": round(value, 3), "unit": UNIT, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
           "data": "synthetic (seeded breast phantom, straight-ray measured-data stand-in)",
           "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}; FP64 rays/phase, {args.dtype} "
                                  f"contractions; one step = one linearised frequency set, sets taken in sweep "
                                  f"order (model carried from set to set, the sweep restarting from the start "
                                  f"model after its last set)",
                      "pixels": N, "selected_pairs": P, "frequencies_per_step": F_timed / args.steps,
                      "pixel_pair_freq_per_step": units, "sets_timed": timed_sets,
                      "ms_per_sweep_estimate": round(ms_per_step * nsets, 1)},
           "roofline": roof, "stages_ms_per_set": stages}
    if large:
        out["config"]["emitter_batch"] = batch
    return out, prob


def dtype_leg(args, dev, dtype, prob_f32):
    """The headline workload with another contraction type: per-set time over
    one sweep, the backprojection launch, and the image of set 0 against the
    headline type's image of set 0."""
    import torch
    prob = copy.copy(prob_f32)
    prob.dtype = dtype
    large = args.workload == "ring1024_grid1100"
    batch = args.emitter_batch or (512 if large else 0)   # as the headline step
    res = {}
    c_hi = None
    if args.dtype != dtype:
        # set 0 in the headline type first, so that only one workspace of the
        # large instance is held at a time
        ref = Sweep(prob, args.dtype, batch, dev)
        ref.set_step()
        c_hi = ref.c.cpu().numpy()
        ref.release()
        del ref
        torch.cuda.empty_cache()
    sw = Sweep(prob, dtype, batch, dev)
    c0 = sw.c_start.cpu().numpy()
    sw.set_step()
    c_lo = sw.c.cpu().numpy()
    if c_hi is not None:
        d_lo, d_hi = c_lo - c0, c_hi - c0
        res["set0_image_vs_" + args.dtype] = {
            "rel_l2_dc": float("%.4g" % (np.linalg.norm(d_lo - d_hi) / np.linalg.norm(d_hi))),
            "max_abs_dc_diff_m_s": float("%.4g" % np.abs(d_lo - d_hi).max())}
    sw.next_set = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    sw.sweep()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / len(prob.freq_sets)
    g = sw.g
    N, P = g.n_pixels, selected_pairs(g.m, prob.inv.recv_fraction)
    F = sum(len(f) for f in prob.freq_sets) / len(prob.freq_sets)
    res.update({"ms_per_set": round(ms, 3), "value": round(N * P * F / (ms * 1e-3) / 1e9, 3), "unit": UNIT})
    sw.release_workspace()
    roof, _ = backprojection_roofline(sw, max(3, args.adjoint_reps // 2), args.workload, stages=False)
    res["backprojection"] = {k: roof[k] for k in ("kernel", "launch_ms", "achieved", "peak", "frac")}
    res["backprojection"]["mfma_issued_frac"] = roof["mfma_issued"]["frac"] if roof["mfma_issued"] else None
    sw.release()
    del sw
    torch.cuda.empty_cache()
    log(f"{dtype} leg: {ms:.1f} ms per set, backprojection {roof['launch_ms']:.2f} ms ({roof['frac']:.3f} of peak)")
    return res


def ring256_leg(args, dev):
    """The 256-element workload: its whole 8-set sweep, the CG-solved set, the
    asymptotic weights and the ToF starting model."""
    import torch
    import paper_2511_16633_amd as rb
    import workload as W
    prob = W.breast_ring256(dtype="f32")
    sw = Sweep(prob, "f32", 0, dev)
    stream = sw.stream
    g, topts = sw.g, sw.topts
    sw.sweep()
    torch.cuda.synchronize()
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        sw.sweep()
    torch.cuda.synchronize()
    ms_sweep = (time.perf_counter() - t) * 1e3 / reps
    N, P = g.n_pixels, selected_pairs(g.m, prob.inv.recv_fraction)
    F = sum(len(f) for f in prob.freq_sets)
    out = {"workload": "ring256_grid480: " + WORKLOADS["ring256_grid480"] + "; f32 contractions; one 8-set sweep",
           "ms_per_sweep": round(ms_sweep, 3), "value": round(N * P * F / (ms_sweep * 1e-3) / 1e9, 3), "unit": UNIT,
           "update_norms_m_s": [round(x, 2) for x in sw.norms[-len(prob.freq_sets):]]}
    roof, stages = backprojection_roofline(sw, 20, "ring256_grid480", stages=True)
    out["roofline"] = roof
    out["stages_ms_per_set"] = stages
    log(f"ring256 sweep {ms_sweep:.1f} ms, backprojection {roof['launch_ms']:.3f} ms ({roof['frac']:.3f})")
    fs, pm0, c_start, alpha = prob.freq_sets[0], sw.pms[0], sw.c_start, sw.alpha
    nf = len(fs)
    ws_bytes = sw.ws.numel()
    sw.ws = None
    torch.cuda.empty_cache()

    if args.cg_iters > 0:   # --cg-iters 0 skips the CG and asymptotic-weight measurements
        # the linear subproblem of set 0 solved by CG instead of the single step
        cws = torch.empty(max(rb.invert_cg_workspace_bytes(g, topts, nf, "f32", 0), ws_bytes), dtype=torch.uint8,
                          device=dev)
        ccg = torch.empty_like(c_start)

        def cg_set(k):
            ccg.copy_(c_start)
            return rb.invert_frequency_set_cg(g, topts, prob.inv, "f32", ccg, alpha, fs, pm0, k, ccg, ws=cws,
                                              stream=stream)

        def one_set():
            ccg.copy_(c_start)
            return rb.invert_frequency_set(g, topts, prob.inv, "f32", ccg, alpha, fs, pm0, ccg, ws=cws, stream=stream)

        t_one = timed_events(torch, stream, one_set)
        t_1 = timed_events(torch, stream, lambda: cg_set(1))
        t_k = timed_events(torch, stream, lambda: cg_set(args.cg_iters))
        _, alphas, rzs = cg_set(args.cg_iters)
        t_it = (t_k - t_1) / max(args.cg_iters - 1, 1)
        it_flop = 12.0 * N * P * nf
        cg = {"iters": args.cg_iters, "ms_per_set": round(t_k, 3), "ms_per_set_one_iteration": round(t_1, 3),
              "ms_per_set_single_step": round(t_one, 3), "ms_per_extra_iteration": round(t_it, 3),
              "iteration_tflops": round(it_flop / (t_it * 1e-3) / 1e12, 3),
              "iteration_frac": round(it_flop / (t_it * 1e-3) / 1e12 / PEAK["f32"], 4),
              "rz_first_last": [rzs[0], rzs[-1]]}
        del cws
        asws = torch.empty(rb.invert_asymptotic_workspace_bytes(g, topts, nf, "f32", 0), dtype=torch.uint8, device=dev)

        def asym_set():
            ccg.copy_(c_start)
            return rb.invert_frequency_set_asymptotic(g, topts, prob.inv, "f32", ccg, alpha, fs, pm0, ccg, ws=asws,
                                                      stream=stream)

        cg["asymptotic_weights_ms_per_set"] = round(timed_events(torch, stream, asym_set), 3)
        del asws, ccg
        out["cg"] = cg
        log(f"CG set 0: {args.cg_iters} iterations {t_k:.2f} ms, single step {t_one:.2f} ms")

    # the ToF starting model from water against straight-chord ToFs of the phantom
    T_meas = torch.as_tensor(W.straight_ray_tof(g, prob.c_true), device=dev)
    c_w = torch.full_like(c_start, g.c_background)
    c_t = torch.empty_like(c_start)
    tws = torch.empty(rb.tof_workspace_bytes(g, topts), dtype=torch.uint8, device=dev)
    t_tof = timed_events(torch, stream, lambda: rb.tof_invert(g, topts, prob.inv, c_w, T_meas, args.tof_iters, c_t,
                                                             ws=tws, stream=stream), reps=2)
    rms, _ = rb.tof_invert(g, topts, prob.inv, c_w, T_meas, args.tof_iters, c_t, ws=tws, stream=stream)
    del tws
    ct = torch.as_tensor(prob.c_true.reshape(-1), device=dev)
    err0 = float(torch.linalg.vector_norm(c_w - ct)) / math.sqrt(N)
    err1 = float(torch.linalg.vector_norm(c_t - ct)) / math.sqrt(N)
    sw.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def sweep_from(c0):
        sw.c_start = c0
        sw.sweep()
        return float(torch.linalg.vector_norm(sw.c - ct)) / math.sqrt(N)

    e_tof = sweep_from(c_t.clone())
    e_ref = sweep_from(c_start)
    out["tof"] = {"iters": args.tof_iters, "ms": round(t_tof, 3), "ms_per_iteration": round(t_tof / args.tof_iters, 3),
                  "rms_tof_residual_s": [float("%.4g" % r) for r in rms],
                  "rms_speed_error_m_s": {"water": round(err0, 3), "after_tof": round(err1, 3),
                                          "after_sweep_from_tof_start": round(e_tof, 3),
                                          "after_sweep_from_smoothed_truth": round(e_ref, 3)}}
    log(f"ToF start: {args.tof_iters} iterations {t_tof:.2f} ms")
    sw.release()
    del sw, T_meas, c_w, c_t, ct
    torch.cuda.empty_cache()
    return out


# Contraction type per serving size class in the precision-form mix: FP32 for
# the 64- and 256-element jobs, BF16 (FP32 accumulation, FP64 phase) for the
# 1024-element jobs, as the large instance is specified.
MIXED_DTYPES = ("f32", "f32", "bf16")
PLAIN_DTYPES = ("f32", "f32", "f32")


def serving_report(dev, n_jobs):
    """The serving loop on a Poisson stream (0.5 jobs/s, sizes 64/256/1024
    elements in the ratio 5:4:1), twice: every job in plain FP32, and the
    precision form (BF16 contractions for the 1024-element jobs).  Each
    served run is quoted against the same jobs in the same contraction types
    served one job at a time (a single-server FIFO queue over the jobs'
    measured alone times, one run per job), and every served result is
    compared bitwise with that job's alone result."""
    import torch
    import workload as W
    from paper_2511_16633_amd import serving as S
    t = time.time()
    specs = W.serving_stream(n_jobs)
    probs = []
    for sp in specs:
        p = W.serving_job(sp["size_class"], sp["seed"], sp["ring_radius"])
        probs.append((sp, p, W.resolve_trace_opts(p.geom, p.c_start, p.trace.n_rays)))
    log(f"serving: {n_jobs} jobs generated in {time.time() - t:.1f} s")
    counts = [sum(1 for sp, _, _ in probs if sp["size_class"] == c) for c in range(3)]
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    out = {"stream": f"Poisson 0.5 jobs/s, {n_jobs} jobs, seed 42; ring64_grid128 / ring256_grid480 / "
                     f"ring1024_grid1100 = {counts[0]} / {counts[1]} / {counts[2]}; ring radius 80-120 mm",
           "baseline": "the same jobs in the same contraction types one at a time: a single-server FIFO queue "
                       "over the arrivals whose service times are the jobs' measured alone times (each job run "
                       "alone once, after the served run)"}
    for name, dtypes in (("plain_f32", PLAIN_DTYPES), ("precision_form", MIXED_DTYPES)):
        jobs = [S.Job(jid=sp["job"], arrival=sp["arrival_s"], geom=p.geom, topts=to, inv=p.inv,
                      dtype=dtypes[sp["size_class"]], c_start=p.c_start, alpha0=p.alpha0, freq_sets=p.freq_sets,
                      p_meas=p.p_meas, size_class=sp["size_class"]) for sp, p, to in probs]
        torch.cuda.empty_cache()
        srv = S.Server(dev, max_running=4)
        srv.prewarm(jobs)
        served = srv.run(jobs, realtime=True)
        log(f"serving {name}: p50 {served['p50_latency_s']:.3f} s, p99 {served['p99_latency_s']:.3f} s")
        service, same = [], True
        for j in jobs:
            a = copy.copy(j)
            a.result = None
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.run_job(a, dev, srv.pool)   # the served run's workspaces, reused as the server reuses them
            service.append(time.perf_counter() - t)
            same = same and a.result is not None and j.result is not None and bool(np.array_equal(a.result, j.result))
        srv.pool.release()
        torch.cuda.empty_cache()
        seq = S.sequential_baseline(jobs, service)
        out[name] = {"dtypes": "/".join(dtypes), "budget_gib": round(srv.budget / 2**30, 1),
                     "max_running": srv.max_running, "served": rnd(served), "one_at_a_time": rnd(seq),
                     "same_alone_and_served": same}
        if name == "precision_form":
            # the precision form's large jobs against their plain-FP32 results
            big = [(j, x) for j, x in zip(jobs, out_plain_results) if j.dtype != "f32"]
            if big:
                rel = [float(np.linalg.norm((j.result - j.c_start.reshape(-1)) - (x - j.c_start.reshape(-1)))
                             / np.linalg.norm(x - j.c_start.reshape(-1))) for j, x in big]
                mx = [float(np.abs(j.result - x).max()) for j, x in big]
                out[name]["bf16_jobs_vs_plain_f32_after_whole_sweep"] = {"max_rel_l2_dc": float("%.4g" % max(rel)),
                                                       "max_abs_dc_diff_m_s": float("%.4g" % max(mx))}
        else:
            out_plain_results = [j.result for j in jobs]
        del jobs
        torch.cuda.empty_cache()
    out["burst"] = serving_burst(dev)
    return out


def serving_burst(dev, n_jobs=40):
    """A burst of small and medium jobs (64- and 256-element rings, FP32),
    all present at the start: served as the server does by default (the
    64-element rings in four batch lanes of grouped rounds, the 256-element
    rings on streams of their own), with every job in one lane of grouped
    rounds, with one stream per job and no grouping, and one at a time."""
    import torch
    import workload as W
    from paper_2511_16633_amd import serving as S
    specs = [sp for sp in W.serving_stream(4 * n_jobs, seed=7) if sp["size_class"] < 2][:n_jobs]
    probs = []
    for sp in specs:
        p = W.serving_job(sp["size_class"], sp["seed"], sp["ring_radius"])
        probs.append((sp, p, W.resolve_trace_opts(p.geom, p.c_start, p.trace.n_rays)))

    def jobs():
        return [S.Job(jid=i, arrival=0.0, geom=p.geom, topts=to, inv=p.inv, dtype="f32", c_start=p.c_start,
                      alpha0=p.alpha0, freq_sets=p.freq_sets, p_meas=p.p_meas, size_class=sp["size_class"])
                for i, (sp, p, to) in enumerate(probs)]

    res = {"jobs": f"{n_jobs} jobs all present at the start, ring64_grid128 / ring256_grid480 = "
                   f"{sum(1 for sp, _, _ in probs if sp['size_class'] == 0)} / "
                   f"{sum(1 for sp, _, _ in probs if sp['size_class'] == 1)}, f32"}
    ref = None
    for name, kw in (("served", {}), ("grouped_up_to_256", dict(group_max_m=256, lanes=1)),
                     ("streams", dict(grouped=False))):
        js = jobs()
        torch.cuda.empty_cache()   # every run starts from the same free memory
        srv = S.Server(dev, max_running=8, lane_max=64, **kw)
        srv.run(js, realtime=False)   # warm-up run
        js = jobs()
        st = srv.run(js, realtime=False)
        srv.pool.release()
        res[name] = {"makespan_s": round(st["makespan_s"], 4), "p50_latency_s": round(st["p50_latency_s"], 4),
                     "p99_latency_s": round(st["p99_latency_s"], 4), "errors": st["errors"],
                     "first_error": st["first_error"],
                     "grouped_rounds": st["grouped_rounds"], "max_jobs_per_round": st["max_jobs_per_round"]}
        if ref is None:
            ref = [j.result for j in js]
        else:
            res["same_in_every_mode"] = (res.get("same_in_every_mode", True) and
                                               all(np.array_equal(a, j.result) for a, j in zip(ref, js)))
    alone = jobs()
    torch.cuda.empty_cache()
    srv = S.Server(dev)
    srv.prewarm(alone)   # one workspace of each size, as the served runs had
    torch.cuda.synchronize()
    t = time.perf_counter()
    for j in alone:
        S.run_job(j, dev, srv.pool)
    res["one_at_a_time_s"] = round(time.perf_counter() - t, 4)
    srv.pool.release()
    res["same_alone_and_grouped"] = all(np.array_equal(a, j.result) for a, j in zip(ref, alone))
    log(f"burst: served {res['served']['makespan_s']:.3f} s (p50 {res['served']['p50_latency_s']:.3f} s), "
        f"all grouped {res['grouped_up_to_256']['makespan_s']:.3f} s, streams {res['streams']['makespan_s']:.3f} s "
        f"(p50 {res['streams']['p50_latency_s']:.3f} s), one at a time {res['one_at_a_time_s']:.3f} s")
    torch.cuda.empty_cache()
    return res


def cpu_baseline_large(prob, P, reps=3):
    """The FP64 oracle, as it stands, on a labelled subset of one frequency
    set of the large instance, extrapolated linearly to the whole set:

    * rays and tables (oracle.rays.tables) of 16 of the 1024 emitters on the
      full grid, in the start model: x 64;
    * the set's per-frequency oracle work - Green's functions on the tables
      and at the receivers, outlier weights, backprojection, Hessian
      diagonal, then the forward operator of the step length - for all 1024
      elements and the set's 4 frequencies on a 110 x 110-pixel patch (1/100
      of the pixels) with seeded tables of the same shape: x 100.
    Median of `reps` runs of each part."""
    import workload as W
    from oracle import born, invert, rays
    g = prob.geom
    topts = W.resolve_trace_opts(g, prob.c_start, prob.trace.n_rays)
    s = 1.0 / prob.c_start
    ne = 16
    tt = []
    for _ in range(reps):
        t = time.perf_counter()
        rays.tables(g, topts, s, prob.alpha0, 0, ne)
        tt.append(time.perf_counter() - t)
    patch = W.centred_grid(110, g.h, g.m, g.ring_radius, g.c_background)
    T, A, B, Tr, Ar, Br = W.random_tables(patch, seed=5)
    A, B, Ar, Br = (x.astype(np.float64) for x in (A, B, Ar, Br))
    fs = prob.freq_sets[0]
    mask = invert.receiver_mask(g.m, prob.inv.recv_fraction)
    dA = g.h * g.h
    v = W.random_delta(patch.n_pixels, 6)
    tc = []
    for _ in range(reps):
        t = time.perf_counter()
        Gs = []
        for k, f in enumerate(fs):
            G = born.green(T, A, B, f, prob.inv.y_pow)
            p = born.green(Tr, Ar, Br, f, prob.inv.y_pow)
            D = prob.p_meas[0][k] - p
            Wk = invert.outlier_weights(prob.p_meas[0][k], mask, prob.inv.outlier_fraction)
            born.born_adjoint(G, Wk * D, f, dA)
            born.hessian_diag(G, Wk, f, dA)
            Gs.append(G)
        for k, f in enumerate(fs):
            born.born_forward(Gs[k], v, f, dA)
        del Gs
        tc.append(time.perf_counter() - t)
    t_trace = statistics.median(tt) * (g.m / ne)
    t_contr = statistics.median(tc) * (g.n_pixels / patch.n_pixels)
    t_set = t_trace + t_contr
    units = g.n_pixels * P * len(fs)
    return {"value": round(units / t_set / 1e9, 5), "unit": UNIT, "cores": host_threads(), "kind": "oracle",
            "cpu": host_cpu(), "extrapolated": True,
            "sample": (f"one frequency set of the same workload (4 frequencies), extrapolated linearly from a "
                       f"labelled subset, median of {reps} runs each: rays and tables of {ne} of {g.m} emitters "
                       f"on the full grid ({statistics.median(tt):.1f} s, x {g.m // ne}) and the per-frequency "
                       f"Green's functions, backprojection, Hessian diagonal and forward for all {g.m} elements "
                       f"on a 110x110-pixel patch with seeded tables ({statistics.median(tc):.1f} s, "
                       f"x {g.n_pixels / patch.n_pixels:.0f}); estimated {t_set:.0f} s per set"),
            "seconds_per_set_estimate": round(t_set, 1)}


def cpu_baseline_ring256(prob, P, reps=3):
    """The FP64 oracle, as it stands, on the first frequency set of the
    256-element workload (full grid and ring), median of `reps` runs."""
    import workload as W
    from oracle import invert
    topts = W.resolve_trace_opts(prob.geom, prob.c_start, prob.trace.n_rays)
    tt = []
    for _ in range(reps):
        t = time.perf_counter()
        invert.invert_frequency_set(prob.geom, topts, prob.inv, prob.c_start, prob.alpha0, prob.freq_sets[0],
                                    prob.p_meas[0])
        tt.append(time.perf_counter() - t)
    dt = statistics.median(tt)
    units = prob.geom.n_pixels * P * len(prob.freq_sets[0])
    return {"value": round(units / dt / 1e9, 4), "unit": UNIT, "cores": host_threads(), "kind": "oracle",
            "cpu": host_cpu(), "extrapolated": False,
            "sample": f"the first frequency set (3 frequencies) of the same workload, full grid and ring, median of "
                      f"{reps} runs: {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16", "f16"])
    ap.add_argument("--workload", default="ring1024_grid1100", choices=list(WORKLOADS),
                    help="headline workload (default: the large instance)")
    ap.add_argument("--emitter-batch", type=int, default=0, help="emitters traced per batch (0: default)")
    ap.add_argument("--adjoint-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop latency measurement")
    ap.add_argument("--no-extras", action="store_true", help="headline only (no bf16 / 256-element legs)")
    ap.add_argument("--serving-jobs", type=int, default=24)
    ap.add_argument("--cg-iters", type=int, default=10)
    ap.add_argument("--tof-iters", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    dev = "cuda:0"
    out, prob = headline(args, dev)
    extra = []
    if not args.no_extras:
        other = "bf16" if args.dtype != "bf16" else "f32"
        out[other + "_contractions"] = dtype_leg(args, dev, other, prob)
        extra.append(other + "_contractions")
        if args.workload != "ring256_grid480":
            out["ring256_grid480"] = ring256_leg(args, dev)
            extra.append("ring256_grid480")
    if not args.no_serving:
        torch.cuda.empty_cache()
        try:
            out["serving"] = serving_report(dev, args.serving_jobs)
        except Exception as exc:   # reported, the measured line still prints
            out["serving"] = {"error": f"{type(exc).__name__}: {exc}"}
        extra.append("serving")
    if not args.no_cpu_baseline:
        P = out["config"]["selected_pairs"]
        t = time.time()
        out["cpu_baseline"] = (cpu_baseline_large(prob, P) if args.workload == "ring1024_grid1100"
                               else cpu_baseline_ring256(prob, P))
        log(f"cpu baseline {out['cpu_baseline']['value']} {UNIT} ({time.time() - t:.1f} s)")
    out["extra_keys"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
