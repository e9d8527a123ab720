"""Serving loop for reconstruction jobs (continuous batching on one GPU).

Jobs of different ring sizes and grids arrive over time.  A job is admitted
as soon as its device-memory footprint (the library workspace for its
largest frequency set plus its inputs and outputs) fits the budget and a
slot is free; admission is first-come first-served with backfill, so a small
job may start while a large one waits for memory.  Every admitted job runs
its frequency sets low to high, its workspace (ray tables, Green's
functions) resident on the device from admission to completion.

Two lanes share the budget:

* the batch lane (rings of up to `group_max_m` elements): one host thread
  and one HIP stream run rounds; a round takes the next frequency set of
  every job in the lane and runs them in one call of the library's grouped
  single step, whose backprojection contractions share launches - a flat
  grid of (job, frequency, pixel tile) work items - so that small problems
  fill the GPU together.  Jobs join the lane between rounds as they are
  admitted and leave it when their last set is done (iteration-level
  batching);
* large rings, which fill the GPU alone, run on a HIP stream and host
  thread of their own each, overlapping with the batch lane and with each
  other on the device.

A job's result depends only on its own inputs (private workspace; the
grouped launches compute each work item as the single-job launch does, and
every reduction has a fixed order), so it is bitwise the same alone and in
any mix.

Only argument marshalling and bookkeeping happen here; every step of a
reconstruction runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
import math
import threading
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _binding as B


@dataclasses.dataclass
class Job:
    jid: int
    arrival: float                 # seconds after the stream starts
    geom: object
    topts: object
    inv: object
    dtype: str
    c_start: np.ndarray
    alpha0: Optional[np.ndarray]
    freq_sets: Sequence[np.ndarray]
    p_meas: Sequence[np.ndarray]
    size_class: int = 0
    emitter_batch: int = 0
    footprint: int = 0
    ws_bytes: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    result: Optional[np.ndarray] = None
    norms: Optional[List[float]] = None
    error: Optional[str] = None

    @property
    def units(self) -> int:
        """pixel x selected pair x frequency of the whole job"""
        m = self.geom.m
        dmin = int(math.ceil((1.0 - self.inv.recv_fraction) * 0.5 * m - 1e-9))
        per_e = sum(1 for r in range(m) if min(r, m - r) >= dmin)
        return self.geom.nx * self.geom.ny * m * per_e * sum(len(f) for f in self.freq_sets)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def plan(job: Job, cap_bytes: int) -> None:
    """Emitter batch and footprint: the largest batch whose workspace fits
    `cap_bytes` (all emitters if they fit)."""
    nf = max(len(f) for f in job.freq_sets)
    m = job.geom.m
    batch = 0
    ws = B.invert_workspace_bytes(job.geom, job.topts, nf, job.dtype, 0)
    b = m
    while ws > cap_bytes and b > 1:
        b = max(1, b // 2)
        batch = b
        ws = B.invert_workspace_bytes(job.geom, job.topts, nf, job.dtype, b)
    N = job.geom.nx * job.geom.ny
    io = 8 * N * 3 + sum(16 * len(f) * m * m for f in job.freq_sets)
    job.emitter_batch = batch
    job.ws_bytes = ws
    job.footprint = ws + io + (64 << 20)


def run_job(job: Job, device: str) -> None:
    """The whole sweep of one job on a stream of its own (blocking)."""
    st = torch.cuda.Stream(device=device)   # default priority
    with torch.cuda.stream(st):
        c = torch.as_tensor(job.c_start.reshape(-1), dtype=torch.float64).to(device, non_blocking=False)
        al = None if job.alpha0 is None else torch.as_tensor(job.alpha0.reshape(-1), dtype=torch.float64).to(device)
        pms = [torch.as_tensor(np.stack([p.real, p.imag], -1), dtype=torch.float64).to(device) for p in job.p_meas]
        ws = torch.empty(max(job.ws_bytes, 256), dtype=torch.uint8, device=device)
        norms = []
        for fs, pm in zip(job.freq_sets, pms):
            norms.append(B.invert_frequency_set(job.geom, job.topts, job.inv, job.dtype, c, al, fs, pm, c, ws=ws,
                                                stream=st))
        job.result = c.cpu().numpy()
        job.norms = norms
        del ws, pms, c, al
    st.synchronize()


class _LaneJob:
    """A job in the batch lane: its device inputs and next frequency set."""

    def __init__(self, job: Job, device: str):
        self.job = job
        self.c = torch.as_tensor(job.c_start.reshape(-1), dtype=torch.float64).to(device)
        self.al = (None if job.alpha0 is None
                   else torch.as_tensor(job.alpha0.reshape(-1), dtype=torch.float64).to(device))
        self.pms = [torch.as_tensor(np.stack([p.real, p.imag], -1), dtype=torch.float64).to(device)
                    for p in job.p_meas]
        self.ws = torch.empty(max(job.ws_bytes, 256), dtype=torch.uint8, device=device)
        self.k = 0
        self.norms: List[float] = []

    def call(self) -> dict:
        j = self.job
        return {"g": j.geom, "t": j.topts, "o": j.inv, "dtype": j.dtype, "c_in": self.c, "alpha0": self.al,
                "freqs": j.freq_sets[self.k], "p_meas": self.pms[self.k], "c_out": self.c, "ws": self.ws}


class Server:
    """Admission by device-memory footprint; the batch lane for small rings
    (grouped rounds on one stream), one stream and host thread per large
    running job."""

    def __init__(self, device: str = "cuda:0", budget_bytes: Optional[int] = None, max_running: int = 4,
                 grouped: bool = True, group_max_m: int = 256, lane_max: int = 16):
        self.device = device
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(torch.device(device))
            budget_bytes = int(0.75 * free)
        self.budget = int(budget_bytes)
        self.max_running = int(max_running)
        self.grouped = bool(grouped)
        self.group_max_m = int(group_max_m)
        self.lane_max = int(lane_max)
        self.rounds = 0            # grouped calls made by the last run
        self.round_sizes: List[int] = []
        self.round_rings: List[int] = []   # distinct ring sizes per round

    def in_lane(self, job: Job) -> bool:
        return self.grouped and job.geom.m <= self.group_max_m

    def run(self, jobs: List[Job], realtime: bool = True) -> dict:
        """Serve `jobs` (arrival times relative to the start).  With
        realtime=False every job is present at the start."""
        B.lib()
        for j in jobs:
            if not j.footprint:
                plan(j, self.budget // 2)   # two of the largest jobs can run side by side
            if j.footprint > self.budget:
                raise ValueError(f"job {j.jid} needs {j.footprint} bytes, budget {self.budget}")
        pending = sorted(jobs, key=lambda j: (j.arrival, j.jid))
        waiting: List[Job] = []
        running = {}
        lane_new: List[Job] = []   # admitted to the batch lane, not yet in a round
        lane_count = 0
        used = 0
        stop = False
        cond = threading.Condition()
        t0 = time.perf_counter()
        self.rounds = 0
        self.round_sizes = []
        self.round_rings = []

        def now() -> float:
            return time.perf_counter() - t0

        def finish(job: Job):
            nonlocal used, lane_count
            with cond:
                job.t_done = now()
                used -= job.footprint
                if self.in_lane(job):
                    lane_count -= 1
                running.pop(job.jid, None)
                cond.notify_all()

        def batcher():
            """Rounds of the batch lane: the next set of every job in it, in
            one grouped call on the lane's stream."""
            st = torch.cuda.Stream(device=self.device)   # default priority
            active: List[_LaneJob] = []
            with torch.cuda.stream(st):
                while True:
                    with cond:
                        while not lane_new and not active and not stop:
                            cond.wait()
                        if not lane_new and not active and stop:
                            return
                        fresh = list(lane_new)
                        lane_new.clear()
                    for job in fresh:
                        try:
                            active.append(_LaneJob(job, self.device))
                        except Exception as exc:  # recorded; the stream goes on
                            job.error = f"{type(exc).__name__}: {exc}"
                            finish(job)
                    if not active:
                        continue
                    self.rounds += 1
                    self.round_sizes.append(len(active))
                    self.round_rings.append(len({a.job.geom.m for a in active}))
                    try:
                        norms = B.invert_frequency_sets_grouped([a.call() for a in active], stream=st)
                        err = None
                    except Exception as exc:
                        norms, err = None, f"{type(exc).__name__}: {exc}"
                    done = []
                    for i, a in enumerate(active):
                        if err is not None:
                            a.job.error = err
                            done.append(a)
                            continue
                        a.norms.append(norms[i])
                        a.k += 1
                        if a.k == len(a.job.freq_sets):
                            done.append(a)
                    for a in done:
                        active.remove(a)
                        if a.job.error is None:
                            a.job.result = a.c.cpu().numpy()
                            a.job.norms = a.norms
                        del a.ws, a.pms, a.c, a.al
                        finish(a.job)

        def worker(job: Job):
            try:
                run_job(job, self.device)
            except Exception as exc:  # recorded; the stream goes on
                job.error = f"{type(exc).__name__}: {exc}"
            finish(job)

        threads = []
        lane = threading.Thread(target=batcher, daemon=True)
        lane.start()
        with cond:
            while pending or waiting or running:
                t = now()
                while pending and (not realtime or pending[0].arrival <= t):
                    waiting.append(pending.pop(0))
                # first come, first served, with backfill
                for job in list(waiting):
                    lane_job = self.in_lane(job)
                    if lane_job and lane_count >= self.lane_max:
                        continue
                    if not lane_job and len(running) - lane_count >= self.max_running:
                        continue
                    if used + job.footprint <= self.budget:
                        waiting.remove(job)
                        used += job.footprint
                        job.t_admit = now()
                        running[job.jid] = job
                        if lane_job:
                            lane_count += 1
                            lane_new.append(job)
                            cond.notify_all()
                        else:
                            th = threading.Thread(target=worker, args=(job,), daemon=True)
                            threads.append(th)
                            th.start()
                timeout = None
                if pending and realtime:
                    timeout = max(0.0, pending[0].arrival - now())
                if pending or waiting or running:
                    cond.wait(timeout=timeout if timeout is not None else 1.0)
            stop = True
            cond.notify_all()
        lane.join()
        for th in threads:
            th.join()
        out = summarize(jobs, now())
        out["grouped_rounds"] = self.rounds
        out["max_jobs_per_round"] = max(self.round_sizes) if self.round_sizes else 0
        out["max_ring_sizes_per_round"] = max(self.round_rings) if self.round_rings else 0
        return out


def summarize(jobs: List[Job], makespan: float) -> dict:
    lat = np.array([j.latency for j in jobs])
    units = sum(j.units for j in jobs)
    return {"jobs": len(jobs), "errors": sum(1 for j in jobs if j.error),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "makespan_s": float(makespan),
            "jobs_per_s": len(jobs) / makespan, "gpixel_pair_freq_per_s": units / makespan / 1e9}


def sequential_baseline(jobs: List[Job], service_s: Sequence[float]) -> dict:
    """The same arrivals served one job at a time, each taking its measured
    alone time: a single-server first-come first-served queue."""
    order = sorted(range(len(jobs)), key=lambda i: (jobs[i].arrival, jobs[i].jid))
    t = 0.0
    lat = np.zeros(len(jobs))
    for i in order:
        start = max(t, jobs[i].arrival)
        t = start + service_s[i]
        lat[i] = t - jobs[i].arrival
    units = sum(j.units for j in jobs)
    return {"p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "makespan_s": float(t),
            "jobs_per_s": len(jobs) / t, "gpixel_pair_freq_per_s": units / t / 1e9}
