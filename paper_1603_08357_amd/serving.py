"""Continuous-batching labeling server on one GPU.

Requests (an edge list, an occupancy mask and a site count) arrive over time.
The scheduler admits them in arrival order whenever a slot is free and their
device bytes fit the HBM budget; an admitted job's copies and its labeling are
enqueued on a stream of its own, so jobs admitted while others are still on
the GPU run alongside them.  A completion event per job frees its slot and its
budget share, which immediately lets the next waiting request in.

The scheduler knows nothing about GPUs: it drives an executor with
``launch(job) -> handle``, ``done(handle) -> bool`` and ``finish(handle)``.
``GpuExecutor`` runs jobs through the C ABI (``ccl_label``) on HIP streams;
tests drive the scheduler with a fake executor and a fake clock.

Latency is arrival -> completion observed by the scheduler (labels back in
host memory).  A malformed request (ids out of range, mismatched lengths) is
rejected at submission and does not touch the GPU or other requests.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


def job_device_bytes(n_sites: int, n_bonds: int) -> int:
    """Device bytes one job holds: src, dst (int32), occ (uint8), labels (int32),
    each rounded up to the allocator's 512-byte granule."""
    up = lambda x: (x + 511) // 512 * 512
    return 2 * up(4 * n_bonds) + up(n_bonds) + up(4 * n_sites)


@dataclass
class Job:
    rid: int
    arrival: float
    n_sites: int
    src: np.ndarray
    dst: np.ndarray
    occ: np.ndarray | None = None
    # filled in by the scheduler
    status: str = "new"  # new | queued | running | done | rejected
    reason: str = ""
    t_admit: float = float("nan")
    t_done: float = float("nan")
    labels: np.ndarray | None = None
    # optional pinned host copies of (src, dst, occ) for asynchronous uploads
    pinned: tuple | None = None
    # ids already checked (e.g. graphs from a validated pool): skip the O(B) scan
    validated: bool = False

    @property
    def n_bonds(self) -> int:
        return int(len(self.src))

    @property
    def bytes(self) -> int:
        return job_device_bytes(self.n_sites, self.n_bonds)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def check_request(job: Job) -> str:
    """Empty string when the request is well formed, else the reason."""
    if job.n_sites < 0 or job.n_sites > 2**31 - 1:
        return "n_sites out of range"
    for name, a, dt in (("src", job.src, np.int32), ("dst", job.dst, np.int32)):
        if a.dtype != dt or a.ndim != 1:
            return f"{name} must be a 1-D {dt.__name__} array"
    if len(job.dst) != len(job.src) or (job.occ is not None and len(job.occ) != len(job.src)):
        return "src, dst and occ lengths differ"
    if job.occ is not None and job.occ.dtype != np.uint8:
        return "occ must be uint8"
    if len(job.src) and job.n_sites == 0:
        return "bonds on an empty graph"
    if len(job.src) and not job.validated:
        lo = min(int(job.src.min()), int(job.dst.min()))
        hi = max(int(job.src.max()), int(job.dst.max()))
        if lo < 0 or hi >= job.n_sites:
            return "site id outside [0, n_sites)"
    return ""


class Scheduler:
    """Admission by HBM budget and slots, FIFO, continuous (no batch barrier)."""

    def __init__(self, executor, budget_bytes: int, max_slots: int, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock
        self.pending: collections.deque[Job] = collections.deque()
        self.running: dict[int, tuple[Job, object]] = {}
        self.finished: list[Job] = []
        self.used = 0
        self.peak_used = 0
        self.peak_running = 0

    def submit(self, job: Job) -> None:
        why = check_request(job)
        if not why and job.bytes > self.budget:
            why = "larger than the HBM budget"
        if why:
            job.status, job.reason = "rejected", why
            job.t_done = self.clock()
            self.finished.append(job)
            return
        job.status = "queued"
        self.pending.append(job)

    def poll(self) -> int:
        """Retire finished jobs, then admit waiting ones; returns #retired."""
        retired = 0
        for rid in list(self.running):
            job, h = self.running[rid]
            if self.ex.done(h):
                job.labels = self.ex.finish(h)
                job.t_done = self.clock()
                job.status = "done"
                self.used -= job.bytes
                del self.running[rid]
                self.finished.append(job)
                retired += 1
        while (self.pending and len(self.running) < self.max_slots
               and self.used + self.pending[0].bytes <= self.budget):
            job = self.pending.popleft()
            self.used += job.bytes
            self.peak_used = max(self.peak_used, self.used)
            job.t_admit = self.clock()
            job.status = "running"
            self.running[job.rid] = (job, self.ex.launch(job))
            self.peak_running = max(self.peak_running, len(self.running))
        return retired

    @property
    def idle(self) -> bool:
        return not self.pending and not self.running

    def serve(self, jobs, t0: float | None = None, idle_wait: float = 0.0):
        """Replay `jobs` (sorted by `arrival`, seconds after t0): submit each
        when its arrival time passes, keep polling, return when all finished.
        Arrival times are rewritten to absolute clock values."""
        t0 = self.clock() if t0 is None else t0
        i = 0
        while i < len(jobs) or not self.idle:
            now = self.clock()
            while i < len(jobs) and t0 + jobs[i].arrival <= now:
                jobs[i].arrival = t0 + jobs[i].arrival
                self.submit(jobs[i])
                i += 1
            self.poll()
            if idle_wait and self.idle and i < len(jobs):
                time.sleep(min(idle_wait, max(0.0, t0 + jobs[i].arrival - self.clock())))
        return self.finished


class GpuExecutor:
    """Runs each job on its own HIP stream: H2D copies, ccl_label, D2H copy of
    the labels into pinned memory, then a completion event."""

    def __init__(self, n_streams: int = 4, device=None, max_sites: int = 1 << 24):
        import torch
        import paper_1603_08357_amd as ccl
        self.torch, self.ccl = torch, ccl
        self.device = torch.device(device if device is not None else "cuda")
        self.free_streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.pinned = [torch.empty(max_sites, dtype=torch.int32, pin_memory=True)
                       for _ in range(n_streams)]
        self.max_sites = max_sites

    def launch(self, job: Job):
        torch = self.torch
        if not self.free_streams:
            raise RuntimeError("more jobs in flight than streams")
        if job.n_sites > self.max_sites:
            raise ValueError("job larger than the executor's pinned buffers")
        s = self.free_streams.pop()
        pin = self.pinned.pop()
        with torch.cuda.stream(s):
            def h2d(a):
                t = a if isinstance(a, torch.Tensor) else torch.from_numpy(a)
                if not t.is_pinned():
                    t = t.pin_memory()
                return t.to(self.device, non_blocking=True)
            hs, hd, ho = job.pinned if job.pinned is not None else (job.src, job.dst, job.occ)
            src, dst = h2d(hs), h2d(hd)
            occ = h2d(ho) if ho is not None else None
            out = torch.empty(job.n_sites, dtype=torch.int32, device=self.device)
            self.ccl.label(src, dst, job.n_sites, occ, out=out, stream=s)
            host = pin[:job.n_sites]
            host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (s, pin, ev, (src, dst, occ, out), host)

    def done(self, h) -> bool:
        return h[2].query()

    def finish(self, h):
        s, pin, ev, tensors, host = h
        ev.synchronize()
        labels = host.numpy().copy()
        del tensors  # allocated on s and used only on s
        self.free_streams.append(s)
        self.pinned.append(pin)
        return labels


def latency_summary(jobs, t_start: float, t_end: float) -> dict:
    done = [j for j in jobs if j.status == "done"]
    lat = np.array([j.latency for j in done]) * 1e3
    sites = sum(j.n_sites for j in done)
    span = max(t_end - t_start, 1e-9)
    return {
        "requests": len(jobs), "completed": len(done),
        "rejected": sum(j.status == "rejected" for j in jobs),
        "throughput_req_s": round(len(done) / span, 2),
        "throughput_Gsites_s": round(sites / span / 1e9, 4),
        "p50_ms": round(float(np.percentile(lat, 50)), 4) if len(lat) else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 4) if len(lat) else None,
        "mean_ms": round(float(lat.mean()), 4) if len(lat) else None,
    }
