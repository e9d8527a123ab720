"""Serving loop for reconstruction jobs (continuous batching on one GPU).

Jobs of different ring sizes and grids arrive over time.  A job is admitted
as soon as its device-memory footprint (the library workspace for its
largest frequency set plus its inputs and outputs) fits the budget and a
slot is free; admission is first-come first-served with backfill, so a small
job may start while a large one waits for memory.  Every admitted job runs
its frequency sets low to high, its workspace (ray tables, Green's
functions) resident on the device from admission to completion.

Two kinds of lanes share the budget:

* the batch lanes (rings of up to `group_max_m` elements, 64 by default:
  larger rings fill the GPU well enough alone that overlapping them on
  streams of their own serves a burst faster than grouping them): each of
  `lanes` lanes has a host thread and a HIP stream of its own and runs
  rounds; a round takes the next frequency set of every job in the lane and runs them
  in one call of the library's grouped single step, whose backprojection
  contractions share launches - a flat grid of (job, frequency, pixel tile)
  work items - so that small problems fill the GPU together, while the
  lanes' other kernels (tracing, forward, update) overlap on the device.
  An admitted job joins the lane with the fewest jobs between rounds and
  leaves it when its last set is done (iteration-level batching);
* larger rings run on a HIP stream and host thread of their own each,
  overlapping with the batch lanes and with each other on the device.

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


def round_workspace(nbytes: int) -> int:
    """A workspace size rounded up to a multiple of 1/8 of its power of two
    (at least 64 MiB): jobs of one size class then ask for the same few
    sizes, so PyTorch's caching allocator hands a finished job's block to
    the next job instead of allocating and mapping gigabytes anew."""
    g = max(64 << 20, 1 << max(0, int(nbytes).bit_length() - 4))
    return -(-int(nbytes) // g) * g


def plan(job: Job, cap_bytes: int) -> None:
    """Emitter batch and footprint: the largest batch whose workspace fits
    `cap_bytes` (all emitters if they fit); the workspace size is rounded
    (round_workspace)."""
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
    job.ws_bytes = round_workspace(ws)
    ws = job.ws_bytes
    job.footprint = ws + io + (64 << 20)


class WorkspacePool:
    """Device workspaces kept from job to job.  A job takes the smallest idle
    buffer that holds its (rounded) workspace and is at most 1/4 larger -
    the library uses what it needs of a larger one - or a new buffer, and
    gives it back when it finishes.  The pool's buffers, in use or idle, stay within
    `limit_bytes`: a new buffer that would pass it first frees idle ones
    (smallest first) back to the device.  So the blocks of large jobs are
    reused whole instead of being split by small jobs' allocations in
    PyTorch's caching allocator, and a new allocation does not find the
    device filled with idle blocks (which makes the allocator free its whole
    cache and retry, a few hundred milliseconds each time)."""

    def __init__(self, device: str, limit_bytes: int):
        self.device = device
        self.limit = int(limit_bytes)
        self.total = 0        # bytes of the pool's buffers, in use or idle
        self.idle_bytes = 0
        self._idle: List[torch.Tensor] = []
        self._lock = threading.Lock()

    def take(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        freed = False
        with self._lock:
            # at most 1/4 larger than asked: admission counts the job's own
            # workspace size, so a small job must not hold a large block
            fits = [i for i, b in enumerate(self._idle) if nbytes <= b.numel() <= nbytes + nbytes // 4]
            if fits:
                i = min(fits, key=lambda i: self._idle[i].numel())
                buf = self._idle.pop(i)
                self.idle_bytes -= buf.numel()
                return buf
            self._idle.sort(key=lambda b: b.numel())
            while self._idle and self.total + nbytes > self.limit:
                n = self._idle.pop(0).numel()
                self.idle_bytes -= n
                self.total -= n
                freed = True
            self.total += nbytes
        try:
            if freed:
                torch.cuda.empty_cache()   # the freed buffers go back to the device
            return torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        except torch.cuda.OutOfMemoryError:
            self.release()
            torch.cuda.empty_cache()
            try:
                return torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            except torch.cuda.OutOfMemoryError:
                with self._lock:
                    self.total -= nbytes
                raise

    def give(self, buf: torch.Tensor) -> None:
        with self._lock:
            self._idle.append(buf)
            self.idle_bytes += buf.numel()

    def release(self) -> None:
        """Drop every idle buffer (PyTorch's cache keeps their blocks)."""
        with self._lock:
            self.total -= self.idle_bytes
            self._idle.clear()
            self.idle_bytes = 0


def run_job(job: Job, device: str, pool: Optional[WorkspacePool] = None) -> None:
    """The whole sweep of one job on a stream of its own (blocking); the
    workspace comes from `pool` when one is given."""
    st = torch.cuda.Stream(device=device)   # default priority
    with torch.cuda.stream(st):
        c = torch.as_tensor(job.c_start.reshape(-1), dtype=torch.float64).to(device, non_blocking=False)
        al = None if job.alpha0 is None else torch.as_tensor(job.alpha0.reshape(-1), dtype=torch.float64).to(device)
        pms = [torch.as_tensor(np.stack([p.real, p.imag], -1), dtype=torch.float64).to(device) for p in job.p_meas]
        ws = pool.take(job.ws_bytes) if pool is not None else torch.empty(max(job.ws_bytes, 256),
                                                                          dtype=torch.uint8, device=device)
        norms = []
        for fs, pm in zip(job.freq_sets, pms):
            norms.append(B.invert_frequency_set(job.geom, job.topts, job.inv, job.dtype, c, al, fs, pm, c, ws=ws,
                                                stream=st))
        job.result = c.cpu().numpy()
        job.norms = norms
        st.synchronize()   # the workspace is free for the next job
        if pool is not None:
            pool.give(ws)
        del ws, pms, c, al


class _LaneJob:
    """A job in the batch lane: its device inputs and next frequency set."""

    def __init__(self, job: Job, device: str, pool: WorkspacePool):
        self.job = job
        self.c = torch.as_tensor(job.c_start.reshape(-1), dtype=torch.float64).to(device)
        self.al = (None if job.alpha0 is None
                   else torch.as_tensor(job.alpha0.reshape(-1), dtype=torch.float64).to(device))
        self.pms = [torch.as_tensor(np.stack([p.real, p.imag], -1), dtype=torch.float64).to(device)
                    for p in job.p_meas]
        self.ws = pool.take(job.ws_bytes)
        self.k = 0
        self.norms: List[float] = []

    def call(self) -> dict:
        j = self.job
        return {"g": j.geom, "t": j.topts, "o": j.inv, "dtype": j.dtype, "c_in": self.c, "alpha0": self.al,
                "freqs": j.freq_sets[self.k], "p_meas": self.pms[self.k], "c_out": self.c, "ws": self.ws}


class Server:
    """Admission by device-memory footprint; batch lanes for small rings
    (grouped rounds, one stream each), one stream and host thread per large
    running job."""

    def __init__(self, device: str = "cuda:0", budget_bytes: Optional[int] = None, max_running: int = 4,
                 grouped: bool = True, group_max_m: int = 64, lane_max: int = 16, lanes: int = 4):
        self.device = device
        if budget_bytes is None:
            # free device memory, counting blocks PyTorch holds cached but unused
            dev = torch.device(device)
            free, _ = torch.cuda.mem_get_info(dev)
            cached = torch.cuda.memory_reserved(dev) - torch.cuda.memory_allocated(dev)
            budget_bytes = int(0.75 * (free + cached))
        self.budget = int(budget_bytes)
        self.max_running = int(max_running)
        self.grouped = bool(grouped)
        self.group_max_m = int(group_max_m)
        self.lane_max = int(lane_max)   # jobs in all batch lanes together
        self.lanes = max(1, int(lanes))
        # workspaces kept between jobs, within the budget
        self.pool = WorkspacePool(device, self.budget)
        self.rounds = 0            # grouped calls made by the last run
        self.round_sizes: List[int] = []
        self.round_rings: List[int] = []   # distinct ring sizes per round

    def prewarm(self, jobs: List[Job]) -> None:
        """Plan `jobs` and allocate one idle workspace of each of their sizes
        (a server started ahead of its traffic)."""
        for j in jobs:
            if not j.footprint:
                plan(j, self.budget // 2)
        for n in sorted({j.ws_bytes for j in jobs}):
            self.pool.give(self.pool.take(n))

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
        lane_new: List[List[Job]] = [[] for _ in range(self.lanes)]   # admitted, not yet in a round
        lane_jobs = [0] * self.lanes   # jobs in each lane
        lane_of = {}
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
                if job.jid in lane_of:
                    lane_count -= 1
                    lane_jobs[lane_of.pop(job.jid)] -= 1
                running.pop(job.jid, None)
                cond.notify_all()

        def batcher(li: int):
            """Rounds of batch lane li: the next set of every job in it, in
            one grouped call on the lane's stream."""
            st = torch.cuda.Stream(device=self.device)   # default priority
            active: List[_LaneJob] = []
            with torch.cuda.stream(st):
                while True:
                    with cond:
                        while not lane_new[li] and not active and not stop:
                            cond.wait()
                        if not lane_new[li] and not active and stop:
                            return
                        fresh = list(lane_new[li])
                        lane_new[li].clear()
                    for job in fresh:
                        try:
                            active.append(_LaneJob(job, self.device, self.pool))
                        except Exception as exc:  # recorded; the stream goes on
                            job.error = f"{type(exc).__name__}: {exc}"
                            finish(job)
                    if not active:
                        continue
                    with cond:
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
                            a.job.result = a.c.cpu().numpy()   # synchronises the lane's stream
                            a.job.norms = a.norms
                        else:
                            st.synchronize()
                        self.pool.give(a.ws)
                        del a.ws, a.pms, a.c, a.al
                        finish(a.job)

        def worker(job: Job):
            try:
                run_job(job, self.device, self.pool)
            except Exception as exc:  # recorded; the stream goes on
                job.error = f"{type(exc).__name__}: {exc}"
            finish(job)

        threads = []
        lane_threads = [threading.Thread(target=batcher, args=(li,), daemon=True) for li in range(self.lanes)]
        for th in lane_threads:
            th.start()
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
                            li = min(range(self.lanes), key=lambda i: (lane_jobs[i], i))
                            lane_jobs[li] += 1
                            lane_of[job.jid] = li
                            lane_new[li].append(job)
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
        for th in lane_threads:
            th.join()
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
    errs = [f"job {j.jid}: {j.error}" for j in jobs if j.error]
    return {"jobs": len(jobs), "errors": len(errs), "first_error": errs[0] if errs else None,
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
