"""Admission logic of the serving loop on the CPU, with a mock executor that
only models durations and bytes (no device code)."""
import numpy as np

from paper_2507_07031_amd.serve import Admission, Busy, Job, serve, summarize
from workloads import generators as gen


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self):
        self.t += 1e-4


class MockExecutor:
    """Job of N points takes N * 1e-8 s; checks budget and slots as it runs."""

    def __init__(self, clock, budget, slots, per_point=1e-8):
        self.clock = clock
        self.budget = budget
        self.slots = slots
        self.per_point = per_point
        self.live = {}
        self.max_bytes = 0
        self.max_live = 0
        self.starts = []

    def footprint(self, job):
        return job.N * 200

    def start(self, job):
        self.live[job.jid] = job
        self.starts.append(job.jid)
        b = sum(self.footprint(j) for j in self.live.values())
        self.max_bytes = max(self.max_bytes, b)
        self.max_live = max(self.max_live, len(self.live))
        assert b <= self.budget and len(self.live) <= self.slots
        job.handle = self.clock() + job.N * self.per_point

    def poll(self, job):
        if self.clock() >= job.handle:
            del self.live[job.jid]
            return True
        return False


def _jobs(count, seed=5, lo=10, hi=22, rate=200.0):
    sizes = gen.log_uniform_sizes(seed, count, lo, hi)
    arr = gen.poisson_arrivals(seed, count, rate)
    return [Job(i, n, a) for i, (n, a) in enumerate(zip(sizes, arr))]


def test_job_padding():
    assert [Job(0, n, 0).N for n in (1, 2, 3, 1024, 1025)] == [1, 2, 4, 1024, 2048]


def test_budget_and_slots_hold_and_all_finish():
    clock = FakeClock()
    budget = 1 << 30
    ex = MockExecutor(clock, budget, 4)
    jobs = _jobs(300)
    fin, rej, wall = serve(jobs, ex, budget, 4, clock=clock, sleep=clock.tick)
    assert len(fin) + len(rej) == 300
    assert all(j.footprint <= budget for j in fin)
    assert all(j.footprint > budget for j in rej)
    assert ex.max_bytes <= budget and ex.max_live <= 4
    assert ex.max_live > 1  # jobs do overlap
    # strict FIFO: starts follow arrival order
    assert ex.starts == sorted(ex.starts)
    s = summarize(fin, wall)
    assert s["jobs"] == len(fin) and s["p99_ms"] >= s["p50_ms"]


def test_tight_budget_serialises_large_jobs():
    clock = FakeClock()
    budget = (1 << 22) * 200  # exactly one 2^22 job
    ex = MockExecutor(clock, budget, 8)
    jobs = [Job(i, 1 << 22, 0.0) for i in range(3)] + [Job(3, 1 << 10, 0.0)]
    fin, rej, _ = serve(jobs, ex, budget, 8, clock=clock, sleep=clock.tick)
    assert not rej and len(fin) == 4
    big = sorted((j for j in fin if j.N == 1 << 22), key=lambda j: j.start)
    for a, b in zip(big, big[1:]):
        assert b.start >= a.finish  # never two at once
    small = [j for j in fin if j.N == 1 << 10][0]
    assert small.start >= big[-1].start  # FIFO: no overtaking


def test_oversize_rejected():
    clock = FakeClock()
    ex = MockExecutor(clock, 1000, 2)
    fin, rej, _ = serve([Job(0, 4, 0.0), Job(1, 1 << 20, 0.0)], ex, 1000, 2, clock=clock, sleep=clock.tick)
    assert [j.jid for j in rej] == [1] and [j.jid for j in fin] == [0]


def test_admission_queue_unit():
    adm = Admission(100, 2, lambda j: j.n)
    a, b, c = Job(0, 60, 0), Job(1, 50, 0), Job(2, 10, 0)
    for j in (a, b, c):
        assert adm.submit(j)
    assert adm.admissible() == [a]          # b does not fit beside a; c must wait behind b
    adm.release(a)
    assert adm.admissible() == [b, c]
    assert adm.used == 60 and np.isclose(adm.used, 60)


def test_queue_full_back_pressure():
    clock = FakeClock()
    ex = MockExecutor(clock, 10 ** 12, 1, per_point=1e-6)
    jobs = [Job(i, 1 << 12, 0.0) for i in range(6)]
    fin, rej, _ = serve(jobs, ex, 10 ** 12, 1, clock=clock, sleep=clock.tick, max_queue=2)
    # all six arrive together: two wait, the rest are refused
    assert sorted(j.jid for j in fin) == [0, 1]
    assert sorted(j.jid for j in rej) == [2, 3, 4, 5]
    assert all(j.error == "rejected: queue full" for j in rej)
    fin2, rej2, _ = serve([Job(i, 1 << 12, i * 0.01) for i in range(6)], MockExecutor(clock, 10 ** 12, 1),
                          10 ** 12, 1, clock=clock, sleep=clock.tick, max_queue=2)
    assert len(fin2) == 6 and not rej2


class FailingExecutor(MockExecutor):
    """Raises for chosen jobs at start (before any work) or at completion."""

    def __init__(self, clock, budget, slots, fail_start=(), fail_poll=()):
        super().__init__(clock, budget, slots)
        self.fail_start, self.fail_poll = set(fail_start), set(fail_poll)

    def start(self, job):
        if job.jid in self.fail_start:
            raise RuntimeError("zk error -3: injected device failure")
        super().start(job)

    def poll(self, job):
        done = super().poll(job)
        if done and job.jid in self.fail_poll:
            raise RuntimeError("zk error -3: injected completion failure")
        return done


def test_failed_jobs_are_isolated():
    clock = FakeClock()
    jobs = _jobs(40, seed=9)
    ex = FailingExecutor(clock, 10 ** 9, 3, fail_start=(3, 17), fail_poll=(8,))
    fin, rej, wall = serve(jobs, ex, 10 ** 9, 3, clock=clock, sleep=clock.tick)
    assert not rej and len(fin) == 40
    failed = {j.jid for j in fin if j.error is not None}
    assert failed == {3, 8, 17}
    assert all(j.finish >= j.start >= j.arrival for j in fin)
    s = summarize(fin, wall)
    assert s["jobs"] == 37 and s["failed"] == 3
    assert not ex.live  # every slot and byte released


class BusyExecutor(MockExecutor):
    """Refuses (Busy) any start while `cap` jobs already run, as the library
    does when cached and in-use scratch reach its budget."""

    def __init__(self, clock, budget, slots, cap):
        super().__init__(clock, budget, slots)
        self.cap = cap
        self.refusals = 0

    def start(self, job):
        if len(self.live) >= self.cap:
            self.refusals += 1
            raise Busy("scratch at the budget")
        super().start(job)


def test_busy_is_back_pressure():
    clock = FakeClock()
    jobs = _jobs(60, seed=13)
    ex = BusyExecutor(clock, 10 ** 12, 4, cap=2)
    fin, rej, wall = serve(jobs, ex, 10 ** 12, 4, clock=clock, sleep=clock.tick)
    assert not rej and len(fin) == 60
    assert all(j.error is None for j in fin)
    assert ex.refusals > 0 and ex.max_live <= 2
    assert ex.starts == sorted(ex.starts)        # retried jobs keep their place
    assert summarize(fin, wall)["retried"] > 0


def test_busy_alone_fails_the_job():
    clock = FakeClock()
    ex = BusyExecutor(clock, 10 ** 12, 2, cap=0)
    fin, rej, _ = serve([Job(0, 8, 0.0), Job(1, 8, 0.0)], ex, 10 ** 12, 2, clock=clock, sleep=clock.tick)
    assert not rej and len(fin) == 2
    assert all(j.error is not None and j.error.startswith("failed") for j in fin)
