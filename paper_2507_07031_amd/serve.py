"""Serving loop for commit jobs: admission by HBM budget, overlap on the device.

A commit job is one basic-block witness of n field elements (its tensor's
evaluations on H, padded with zero evaluations to N = 2^ceil(log2 n)):
inverse NTT to coefficients, the KZG commitment (MSM against the resident
SRS) and the 4x coset evaluation that the quotient by X^N - 1 needs.

* `Admission` is the scheduling policy, free of any device code: jobs wait in
  arrival order; the head job starts as soon as a stream slot is free and its
  HBM footprint fits the budget next to the jobs already running (strict
  FIFO, so a large job is never starved by small ones behind it).  A job
  whose footprint exceeds the whole budget is rejected, and so is a job that
  arrives while `max_queue` jobs already wait (back-pressure).
* `GpuExecutor` runs each admitted job on its own HIP stream (all at the
  default priority), so jobs admitted while others are on the GPU overlap
  with them; completion is detected by polling an event per job.  A job is
  one `zk_commit_job` call (the library overlaps its coset transform with
  the MSM's reduction on a companion stream of the slot's stream).
* `serve` drives a timed arrival stream through both and records per-job
  arrival, start and finish times (host clock).  A job whose start or
  completion raises (a library error such as ZK_EDEVICE) is finished with
  `error` set and its slot and bytes released; the other jobs go on.

The executor is pluggable; the tests use a mock that only models durations
and bytes to check the admission logic on the CPU.
"""
import collections
import time

import numpy as np


class Job:
    __slots__ = ("jid", "n", "N", "arrival", "offset", "start", "finish", "footprint", "handle", "result", "error")

    def __init__(self, jid, n, arrival, offset=0):
        self.jid = int(jid)
        self.n = int(n)
        self.N = 1 << max(0, (int(n) - 1).bit_length())
        self.arrival = float(arrival)
        self.offset = int(offset)
        self.start = None
        self.finish = None
        self.footprint = 0
        self.handle = None
        self.result = None
        self.error = None


class Admission:
    """FIFO admission under a byte budget and a number of concurrent slots."""

    def __init__(self, budget_bytes, slots, footprint, max_queue=None):
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.footprint = footprint
        self.max_queue = max_queue
        self.queue = collections.deque()
        self.running = []
        self.used = 0
        self.rejected = []

    def submit(self, job):
        job.footprint = int(self.footprint(job))
        if job.footprint > self.budget:
            job.error = "rejected: footprint exceeds the budget"
            self.rejected.append(job)
            return False
        if self.max_queue is not None and len(self.queue) >= self.max_queue:
            job.error = "rejected: queue full"
            self.rejected.append(job)
            return False
        self.queue.append(job)
        return True

    def admissible(self):
        """Pop and return the jobs that may start now (in arrival order)."""
        out = []
        while self.queue and len(self.running) + len(out) < self.slots:
            head = self.queue[0]
            if self.used + head.footprint > self.budget:
                break
            self.queue.popleft()
            self.used += head.footprint
            out.append(head)
        self.running.extend(out)
        return out

    def release(self, job):
        self.running.remove(job)
        self.used -= job.footprint
        assert self.used >= 0


class GpuExecutor:
    """Runs commit jobs on HIP streams through the C-ABI (one stream per slot)."""

    def __init__(self, zk, srs, pool, slots, keep_results=False, timing=False):
        import torch
        self.timing = timing
        self.zk = zk
        self.torch = torch
        self.srs = srs
        self.pool = pool                 # (P, 8) device tensor of uniform Fr
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free = list(range(slots))
        self.keep = keep_results

    def footprint(self, job):
        N = job.N
        L = N.bit_length() - 1
        zk = self.zk
        return (N * 32 + 4 * N * 32 + zk.msm_srs_workspace_bytes(self.srs, N)
                + zk.ntt_workspace_bytes(L) + zk.ntt_workspace_bytes(L + 2))

    def start(self, job):
        torch, zk = self.torch, self.zk
        slot = self.free.pop()
        s = self.streams[slot]
        try:
            with torch.cuda.stream(s):
                N = job.N
                ev = self.pool[job.offset:job.offset + N]
                if job.n < N:
                    ev = torch.cat([self.pool[job.offset:job.offset + job.n],
                                    torch.zeros((N - job.n, 8), dtype=torch.int32, device=ev.device)])
                coeffs, com, coset = zk.commit_job(self.srs, ev, log_blowup=2)
                done = torch.cuda.Event(enable_timing=self.timing)
                done.record(s)
        except Exception:
            self.free.append(slot)
            raise
        job.handle = (slot, done, com, coset, coeffs, ev)

    def poll(self, job):
        slot, done, com, coset, coeffs, ev = job.handle
        if not done.query():
            return False
        if self.keep:
            job.result = (self.zk.to_host(com).copy(), self.zk.to_host(coset).copy())
        job.handle = None
        self.free.append(slot)
        return True


def serve(jobs, executor, budget_bytes, slots, clock=time.perf_counter, sleep=None, max_queue=None):
    """Feed `jobs` (sorted by arrival, seconds from start) through admission
    and the executor.  Returns (finished jobs, rejected jobs, wall seconds);
    finished jobs whose `error` is set failed on the device."""
    adm = Admission(budget_bytes, slots, executor.footprint, max_queue)
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    finished = []
    t0 = clock()
    while pending or adm.queue or adm.running:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            adm.submit(pending.popleft())
        for job in list(adm.running):
            if job.start is None:
                continue
            try:
                done = executor.poll(job)
            except Exception as e:  # completion reported a device error
                job.error, done = repr(e), True
            if done:
                job.finish = clock() - t0
                adm.release(job)
                finished.append(job)
        for job in adm.admissible():
            job.start = clock() - t0
            try:
                executor.start(job)
            except Exception as e:  # the call failed before running: no slot held
                job.error = repr(e)
                job.finish = clock() - t0
                adm.release(job)
                finished.append(job)
        if sleep is not None:
            sleep()
    return finished, adm.rejected, clock() - t0


def summarize(finished, wall):
    ok = [j for j in finished if j.error is None]
    lat = np.array([j.finish - j.arrival for j in ok]) * 1e3
    if lat.size == 0:
        return {"jobs": 0, "failed": len(finished)}
    return {"jobs": int(lat.size), "jobs_per_s": lat.size / wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "failed": len(finished) - len(ok)}
