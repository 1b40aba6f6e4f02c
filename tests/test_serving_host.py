"""Host logic of the serving loop, with a fake clock and a fake executor."""
import numpy as np
import pytest

from paper_1603_08357_amd.serving import Job, Scheduler, check_request, job_device_bytes


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """A job takes `cost * n_sites` seconds of fake time; records overlap."""

    def __init__(self, clock, cost=1e-6):
        self.clock, self.cost = clock, cost
        self.inflight = set()
        self.max_inflight = 0
        self.launched = []

    def launch(self, job):
        h = (job.rid, self.clock() + self.cost * max(job.n_sites, 1))
        self.inflight.add(job.rid)
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        self.launched.append(job.rid)
        return h

    def done(self, h):
        return self.clock() >= h[1]

    def finish(self, h):
        self.inflight.discard(h[0])
        return np.array([h[0]], np.int32)


def make_job(rid, n, m=None, arrival=0.0, bad=False):
    m = n if m is None else m
    rng = np.random.default_rng(rid)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if bad:
        dst[0] = n  # out of range
    return Job(rid, arrival, n, src, dst, np.ones(m, np.uint8))


def test_job_bytes():
    assert job_device_bytes(1000, 1500) == 2 * 6144 + 1536 + 4096
    assert job_device_bytes(0, 0) == 0


def test_check_request():
    assert check_request(make_job(0, 10)) == ""
    assert "outside" in check_request(make_job(1, 10, bad=True))
    j = make_job(2, 10)
    j.dst = j.dst[:-1]
    assert "lengths" in check_request(j)
    j = make_job(3, 10)
    j.src = j.src.astype(np.int64)
    assert "int32" in check_request(j)


def test_budget_never_exceeded_and_all_complete():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sizes = [1000, 50_000, 200, 80_000, 3_000, 120_000, 7, 60_000] * 5
    jobs = [make_job(i, n, arrival=i * 1e-3) for i, n in enumerate(sizes)]
    budget = job_device_bytes(120_000, 120_000) + job_device_bytes(60_000, 60_000)
    s = Scheduler(ex, budget, max_slots=4, clock=clock)
    i = 0
    while i < len(jobs) or not s.idle:
        while i < len(jobs) and jobs[i].arrival <= clock.t:
            s.submit(jobs[i])
            i += 1
        s.poll()
        assert s.used <= budget
        assert len(s.running) <= 4
        clock.t += 1e-4
    assert all(j.status == "done" for j in jobs)
    assert s.peak_used <= budget
    assert ex.max_inflight > 1  # work overlapped
    # each result is the job's own
    assert all(int(j.labels[0]) == j.rid for j in jobs)


def test_fifo_admission_and_continuous_refill():
    clock = FakeClock()
    ex = FakeExecutor(clock, cost=1e-3)
    s = Scheduler(ex, budget_bytes=10**9, max_slots=2, clock=clock)
    for i, n in enumerate([100, 10, 10, 10]):
        s.submit(make_job(i, n))
    s.poll()
    assert ex.launched == [0, 1]  # two slots
    clock.t = 0.011  # job 1 (10 sites) done, job 0 (100 sites) still running
    s.poll()
    assert ex.launched == [0, 1, 2]  # a slot freed -> next admitted without waiting for job 0
    assert 0 in s.running
    clock.t = 1.0
    for _ in range(1000):
        if s.idle:
            break
        s.poll()
        clock.t += 1e-3
    assert s.idle and ex.launched == [0, 1, 2, 3]


def test_malformed_and_oversized_requests_fail_alone():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    budget = job_device_bytes(1000, 1000)
    s = Scheduler(ex, budget, max_slots=2, clock=clock)
    good = [make_job(0, 500), make_job(2, 800)]
    bad = make_job(1, 500, bad=True)
    huge = make_job(3, 5000)
    for j in (good[0], bad, good[1], huge):
        s.submit(j)
    while not s.idle:
        s.poll()
        clock.t += 1e-3
    assert bad.status == "rejected" and "outside" in bad.reason
    assert huge.status == "rejected" and "budget" in huge.reason
    assert all(j.status == "done" for j in good)
    assert 1 not in ex.launched and 3 not in ex.launched


def test_serve_replays_arrivals_with_fake_clock():
    clock = FakeClock()

    class TickingExecutor(FakeExecutor):
        def done(self, h):
            clock.t += 1e-5  # time passes while polling
            return super().done(h)

    ex = TickingExecutor(clock)
    jobs = [make_job(i, 100 + i, arrival=i * 1e-4) for i in range(50)]

    def tick():
        clock.t += 1e-5
        return clock.t

    s = Scheduler(ex, 10**9, max_slots=3, clock=tick)
    done = s.serve(jobs, t0=0.0)
    assert len(done) == 50 and all(j.status == "done" for j in done)
    assert all(j.t_done >= j.arrival for j in done)
    assert all(j.t_admit >= j.arrival for j in done)


def test_autotune_candidates_and_layout_key():
    from paper_1603_08357_amd import autotune
    c = autotune.candidates()
    assert len(c) > 20
    assert all((max(t["small_sites"], 0) + 1) // 2 * 4 * t["blocks_per_cu"] <= 160 * 1024 for t in c)
    assert {t["schedule"] for t in c} == {1, 2, 3}
    # the tiled schedule has no merge items: one bonds_per_chunk only
    assert len({t["bonds_per_chunk"] for t in c if t["schedule"] == 3}) == 1
    assert autotune.space_key() != autotune.space_key({"schedule": (2,)})
    assert autotune.space_key({"schedule": (3, 2, 1)}) == autotune.space_key()
    k1 = autotune.layout_key([0, 100, 300, 1300])
    k2 = autotune.layout_key([0, 110, 320, 1270])  # sizes 110, 210, 950
    assert k1 == k2 and k1.startswith("K3-")
    assert autotune.layout_key([0]) == "empty"


class FakeBatchExecutor(FakeExecutor):
    """FakeExecutor that also takes ticks of small jobs."""

    tick_limits = {"sites": 1000, "jobs": 4, "total_sites": 2500, "total_bonds": 10**9}

    def __init__(self, clock, cost=1e-6):
        super().__init__(clock, cost)
        self.batches = []

    def launch_batch(self, jobs):
        assert 1 < len(jobs) <= self.tick_limits["jobs"]
        assert all(j.n_sites <= self.tick_limits["sites"] for j in jobs)
        assert sum(j.n_sites for j in jobs) <= self.tick_limits["total_sites"]
        self.batches.append([j.rid for j in jobs])
        end = self.clock() + self.cost * max(sum(j.n_sites for j in jobs), 1)
        for j in jobs:
            self.inflight.add(j.rid)
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return ("batch", tuple(j.rid for j in jobs), end)

    def done(self, h):
        return self.clock() >= h[-1]

    def finish(self, h):
        if h[0] == "batch":
            for r in h[1]:
                self.inflight.discard(r)
            return [np.array([r], np.int32) for r in h[1]]
        return super().finish(h)


def test_ticks_group_small_jobs_in_order_within_budget():
    clock = FakeClock()
    ex = FakeBatchExecutor(clock)
    sizes = [300, 200, 900, 5000, 100, 100, 100, 100, 100, 700, 20_000, 50, 60] * 3
    jobs = [make_job(i, n, arrival=0.0) for i, n in enumerate(sizes)]
    budget = sum(j.bytes for j in jobs) // 2
    s = Scheduler(ex, budget, max_slots=3, clock=clock)
    for j in jobs:
        s.submit(j)
    order = []
    while not s.idle:
        before = set(s.running)
        s.poll()
        for key in set(s.running) - before:
            order.extend(j.rid for j in s.running[key][0])
        assert s.used <= budget and len(s.running) <= 3
        clock.t += 1e-4
    # only small jobs riding in a tick may pass earlier jobs, and only larger
    # ones that were not at the head of the queue
    pos = {r: i for i, r in enumerate(order)}
    for a in range(len(sizes)):
        for b in range(a + 1, len(sizes)):
            if pos[b] < pos[a]:
                assert sizes[a] > ex.tick_limits["sites"] and sizes[b] <= ex.tick_limits["sites"], (a, b)
    assert s.ticks == len(ex.batches) > 0
    assert all(len(b) > 1 for b in ex.batches)
    for j in jobs:
        assert j.status == "done" and list(j.labels) == [j.rid]
        assert (j.batched > 1) == any(j.rid in b for b in ex.batches)
    # a job too large for a tick never rides in one
    assert not any(r in b for b in ex.batches for r, n in enumerate(sizes) if n > 1000)
