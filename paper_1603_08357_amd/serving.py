"""Continuous-batching labeling server on one GPU.

Requests (an edge list, an occupancy mask and a site count) arrive over time.
The scheduler admits them in arrival order whenever their device bytes fit
the HBM budget (and fewer than `max_slots` launches are in flight); an
admitted job's copies and its labeling are enqueued at once on one of the
executor's streams, so jobs admitted while others are still on the GPU run
alongside them, and the budget -- not a slot count -- is what bounds the work
held on the device.  Small requests that wait together are admitted as one
tick: their edge lists are copied side by side into one batch and labelled by
a single ccl_label_batched launch of a capacity plan (ccl_plan_set_layout per
tick, no allocation or device synchronization), instead of three kernel
launches and four copies each.  A completion event per launch retires its
jobs, which frees their budget share and lets the next waiting requests in.

The scheduler knows nothing about GPUs: it drives an executor with
``launch(job) -> handle``, ``done(handle) -> bool`` and ``finish(handle)``,
plus ``launch_batch(jobs)`` and ``tick_limits`` when the executor groups
small jobs.  ``GpuExecutor`` runs jobs through the C ABI on HIP streams;
tests drive the scheduler with a fake executor and a fake clock.

Latency is arrival -> completion observed by the scheduler (labels back in
host memory).  The GPU executor also records, per launch, the device time of
the host-to-device copies, of the labeling kernels and of the copy back (HIP
events on the launch's stream), so a latency splits into the wait for
admission, those three device phases, and the rest (the stream's earlier
work and the host's polling).  A malformed request (ids out of range,
mismatched lengths) is rejected at submission and does not touch the GPU or
other requests.
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
    # device phases of the job's launch in ms (a tick's jobs share their launch's)
    t_h2d_ms: float = float("nan")
    t_kernel_ms: float = float("nan")
    t_d2h_ms: float = float("nan")
    batched: int = 0  # jobs in the launch that carried this one

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
    """Admission by HBM budget, FIFO, continuous (no batch barrier).

    `max_slots` bounds the launches in flight (a tick counts once).  When the
    executor offers `launch_batch` and the job at the head of the queue is
    small (at most `tick_limits["sites"]` sites), the small jobs among the
    first `tick_window` waiting ones are admitted with it as one launch,
    within the tick's job, site and bond limits and the budget; they may pass
    larger jobs that wait behind the head, never the head itself.  An
    executor with `lane(handle)` (the stream a launch runs on) has its
    launches retired in order per lane: only each lane's oldest launch is
    polled."""

    def __init__(self, executor, budget_bytes: int, max_slots: int, clock=time.perf_counter,
                 tick_window: int = 4096):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock
        self.pending: collections.deque[Job] = collections.deque()
        self.running: dict[int, tuple[list, object]] = {}
        self.lanes: dict[object, collections.deque[int]] = {}
        self.finished: list[Job] = []
        self.used = 0
        self.peak_used = 0
        self.peak_running = 0
        self.in_flight_jobs = 0
        self.launches = 0
        self.ticks = 0
        self._next = 0
        lim = getattr(executor, "tick_limits", None)
        self.tick = dict(lim) if lim and hasattr(executor, "launch_batch") else None
        self.tick_window = int(tick_window)

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

    def _take_tick(self) -> list:
        """The head of the queue (a small job) and the small jobs among the
        next waiting ones that one tick can carry, in arrival order."""
        lim = self.tick
        group, keep, extra, sites, bonds = [], [], 0, 0, 0
        scanned = 0
        while self.pending and scanned < self.tick_window and len(group) < lim["jobs"]:
            j = self.pending.popleft()
            scanned += 1
            if (j.n_sites <= lim["sites"] and self.used + extra + j.bytes <= self.budget
                    and sites + j.n_sites <= lim["total_sites"] and bonds + j.n_bonds <= lim["total_bonds"]):
                group.append(j)
                extra += j.bytes
                sites += j.n_sites
                bonds += j.n_bonds
            else:
                keep.append(j)
        self.pending.extendleft(reversed(keep))
        return group

    def _retire(self, key) -> int:
        jobs, h = self.running.pop(key)
        out = self.ex.finish(h)
        labels = out if len(jobs) > 1 else [out]
        now = self.clock()
        for job, lab in zip(jobs, labels):
            job.labels = lab
            job.t_done = now
            job.status = "done"
            self.used -= job.bytes
            self.finished.append(job)
        self.in_flight_jobs -= len(jobs)
        return len(jobs)

    def poll(self) -> int:
        """Retire finished launches, then admit waiting jobs; returns #retired jobs."""
        retired = 0
        if hasattr(self.ex, "lane"):
            for q in self.lanes.values():
                while q and self.ex.done(self.running[q[0]][1]):
                    retired += self._retire(q.popleft())
        else:
            for key in list(self.running):
                if self.ex.done(self.running[key][1]):
                    retired += self._retire(key)
        while (self.pending and len(self.running) < self.max_slots
               and self.used + self.pending[0].bytes <= self.budget):
            group = self._take_tick() if self.tick and self.pending[0].n_sites <= self.tick["sites"] else []
            if len(group) <= 1:
                group = group or [self.pending.popleft()]
            now = self.clock()
            for job in group:
                self.used += job.bytes
                job.t_admit = now
                job.status = "running"
                job.batched = len(group)
            self.peak_used = max(self.peak_used, self.used)
            h = self.ex.launch_batch(group) if len(group) > 1 else self.ex.launch(group[0])
            self.running[self._next] = (group, h)
            if hasattr(self.ex, "lane"):
                self.lanes.setdefault(self.ex.lane(h), collections.deque()).append(self._next)
            self._next += 1
            self.launches += 1
            self.ticks += len(group) > 1
            self.in_flight_jobs += len(group)
            self.peak_running = max(self.peak_running, self.in_flight_jobs)
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
            if not self.poll() and self.running:
                time.sleep(0)  # lets the executor's copy threads take the interpreter lock
            if idle_wait and self.idle and i < len(jobs):
                time.sleep(min(idle_wait, max(0.0, t0 + jobs[i].arrival - self.clock())))
        return self.finished


class _Done:
    """An already finished copy (the Future interface the executor uses)."""

    def __init__(self, value):
        self.value = value

    def done(self) -> bool:
        return True

    def result(self):
        return self.value


class GpuExecutor:
    """Runs launches on a fixed set of HIP streams, taken in turn: a job's
    H2D copies, ccl_label and the D2H copy of its labels into pinned memory;
    a tick's jobs copied side by side into one batch and labelled by one
    ccl_label_batched launch of the stream's capacity plan.  HIP events
    bracket the three device phases of every launch."""

    def __init__(self, n_streams: int = 4, device=None, max_sites: int = 1 << 24,
                 tick_sites: int = 1 << 17, tick_jobs: int = 512, tick_total_sites: int = 1 << 23,
                 tick_total_bonds: int = 1 << 25, tuning=None, copy_threads: int = 8,
                 inline_copy_sites: int = 1 << 20):
        import torch
        import paper_1603_08357_amd as ccl
        self.torch, self.ccl = torch, ccl
        d = torch.device(device if device is not None else "cuda")
        self.device = d if d.index is not None else torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self._turn = 0
        self.max_sites = max_sites
        self.tick_limits = {"sites": tick_sites, "jobs": tick_jobs, "total_sites": tick_total_sites,
                            "total_bonds": tick_total_bonds}
        self.tuning = tuning
        self.plans = {}  # stream index -> capacity plan (a plan runs on one stream)
        self._pinned = collections.defaultdict(list)  # size class -> free pinned label buffers
        # labels leave the pinned buffers on host threads (a copy into fresh
        # pageable memory runs at a few GB/s per core), so the scheduler's
        # loop keeps admitting while they are copied
        import concurrent.futures as cf
        self._copiers = cf.ThreadPoolExecutor(max_workers=copy_threads)
        self.inline_copy_sites = inline_copy_sites
        if tick_sites > 0:  # the capacity plans up front: creating one synchronizes the device
            for i in range(n_streams):
                self._plan(i)

    def _plan(self, i: int):
        plan = self.plans.get(i)
        if plan is None:
            lim = self.tick_limits
            with self.torch.cuda.device(self.device):
                plan = self.ccl.Plan.with_capacity(lim["jobs"], lim["total_sites"], lim["total_bonds"],
                                                   self.tuning, device=self.device)
            self.plans[i] = plan
        return plan

    def _stream(self):
        i = self._turn
        self._turn = (i + 1) % len(self.streams)
        return i, self.streams[i]

    def _pinned_labels(self, n: int):
        """A pinned host buffer for n labels from a pool of power-of-two
        size classes (pinned allocations are slow; buffers are reused)."""
        c = max(12, (max(n, 1) - 1).bit_length())
        free = self._pinned[c]
        buf = free.pop() if free else self.torch.empty(1 << c, dtype=self.torch.int32, pin_memory=True)
        return c, buf

    def lane(self, h):
        return h[5]

    def _events(self):
        return [self.torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def _h2d(self, a):
        torch = self.torch
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(a)
        if not t.is_pinned():
            t = t.pin_memory()
        return t

    def launch(self, job: Job):
        torch = self.torch
        if job.n_sites > self.max_sites:
            raise ValueError("job larger than the executor's limit")
        lane, s = self._stream()
        ev = self._events()
        with torch.cuda.stream(s):
            ev[0].record(s)
            hs, hd, ho = job.pinned if job.pinned is not None else (job.src, job.dst, job.occ)
            src = self._h2d(hs).to(self.device, non_blocking=True)
            dst = self._h2d(hd).to(self.device, non_blocking=True)
            occ = self._h2d(ho).to(self.device, non_blocking=True) if ho is not None else None
            ev[1].record(s)
            out = torch.empty(job.n_sites, dtype=torch.int32, device=self.device)
            self.ccl.label(src, dst, job.n_sites, occ, out=out, stream=s)
            ev[2].record(s)
            pin = self._pinned_labels(job.n_sites)
            host = pin[1][:job.n_sites]
            host.copy_(out, non_blocking=True)
            ev[3].record(s)
        return ([job], ev, (src, dst, occ, out), (pin, host), None, lane, {"copy": None})

    def launch_batch(self, jobs):
        torch = self.torch
        i, s = self._stream()
        plan = self._plan(i)
        site_off = np.zeros(len(jobs) + 1, np.int64)
        bond_off = np.zeros(len(jobs) + 1, np.int64)
        site_off[1:] = np.cumsum([j.n_sites for j in jobs])
        bond_off[1:] = np.cumsum([j.n_bonds for j in jobs])
        n, m = int(site_off[-1]), int(bond_off[-1])
        ev = self._events()
        with torch.cuda.stream(s):
            ev[0].record(s)
            src = torch.empty(m, dtype=torch.int32, device=self.device)
            dst = torch.empty(m, dtype=torch.int32, device=self.device)
            occ = torch.empty(m, dtype=torch.uint8, device=self.device)
            for k, j in enumerate(jobs):
                a, b = int(bond_off[k]), int(bond_off[k + 1])
                if a == b:
                    continue
                hs, hd, ho = j.pinned if j.pinned is not None else (j.src, j.dst, j.occ)
                src[a:b].copy_(self._h2d(hs), non_blocking=True)
                dst[a:b].copy_(self._h2d(hd), non_blocking=True)
                if ho is not None:
                    occ[a:b].copy_(self._h2d(ho), non_blocking=True)
                else:
                    occ[a:b].fill_(1)
            ev[1].record(s)
            plan.set_layout(site_off, bond_off, stream=s)
            out = torch.empty(n, dtype=torch.int32, device=self.device)
            plan.label(src, dst, occ, out=out, stream=s)
            ev[2].record(s)
            pin = self._pinned_labels(n)
            host = pin[1][:n]
            host.copy_(out, non_blocking=True)
            ev[3].record(s)
        return (list(jobs), ev, (src, dst, occ, out), (pin, host), site_off, i, {"copy": None})

    def _copy_out(self, host, site_off, n_jobs):
        labels = host.numpy()
        if site_off is None:
            return labels.copy()
        return [labels[int(site_off[k]):int(site_off[k + 1])].copy() for k in range(n_jobs)]

    def done(self, h) -> bool:
        """True once the launch's labels are in host memory: when its last
        event has completed, labels of up to `inline_copy_sites` sites are
        copied out of the pinned buffer at once, larger ones on a host thread,
        and the launch is done when that copy is."""
        st = h[6]
        if st["copy"] is None:
            if not h[1][3].query():
                return False
            jobs, (pin, host), site_off = h[0], h[3], h[4]
            if host.numel() <= self.inline_copy_sites:
                st["copy"] = _Done(self._copy_out(host, site_off, len(jobs)))
            else:
                st["copy"] = self._copiers.submit(self._copy_out, host, site_off, len(jobs))
        return st["copy"].done()

    def finish(self, h):
        jobs, ev, tensors, (pin, host), site_off, _, st = h
        ev[3].synchronize()
        h2d, kern, d2h = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
        for j in jobs:
            j.t_h2d_ms, j.t_kernel_ms, j.t_d2h_ms = h2d, kern, d2h
        if st["copy"] is None:
            st["copy"] = self._copiers.submit(self._copy_out, host, site_off, len(jobs))
        out = st["copy"].result()
        tensors = None  # allocated on the launch's stream and used only there
        self._pinned[pin[0]].append(pin[1])  # the copy back and out have completed
        return out


def latency_summary(jobs, t_start: float, t_end: float) -> dict:
    done = [j for j in jobs if j.status == "done"]
    lat = np.array([j.latency for j in done]) * 1e3
    sites = sum(j.n_sites for j in done)
    span = max(t_end - t_start, 1e-9)
    pct = lambda a, q: round(float(np.percentile(a, q)), 4) if len(a) else None
    out = {
        "requests": len(jobs), "completed": len(done),
        "rejected": sum(j.status == "rejected" for j in jobs),
        "throughput_req_s": round(len(done) / span, 2),
        "throughput_Gsites_s": round(sites / span / 1e9, 4),
        "p50_ms": pct(lat, 50),
        "p99_ms": pct(lat, 99),
        "mean_ms": round(float(lat.mean()), 4) if len(lat) else None,
    }
    if done and not np.isnan(done[0].t_h2d_ms):
        # where the latency goes: admission wait, the launch's device phases,
        # and the rest (earlier work on the same stream, host polling)
        queue = np.array([(j.t_admit - j.arrival) * 1e3 for j in done])
        h2d = np.array([j.t_h2d_ms for j in done])
        kern = np.array([j.t_kernel_ms for j in done])
        d2h = np.array([j.t_d2h_ms for j in done])
        rest = lat - queue - h2d - kern - d2h
        out["split_ms"] = {name: {"p50": pct(a, 50), "p99": pct(a, 99), "mean": round(float(a.mean()), 4)}
                           for name, a in (("admission_wait", queue), ("h2d", h2d), ("kernels", kern),
                                           ("d2h", d2h), ("stream_wait_and_host", rest))}
        out["jobs_in_ticks"] = int(sum(j.batched > 1 for j in done))
    return out
