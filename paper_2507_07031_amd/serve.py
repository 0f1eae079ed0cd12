"""Serving loop for commit-and-fold jobs: admission by HBM budget, overlap on the device.

A job is one basic-block witness of n field elements (its tensor's
evaluations on H, padded with zero evaluations to N = 2^ceil(log2 n)) and the
caller's running accumulator instance C_acc (one G1 commitment):

* commit: inverse NTT to coefficients, the KZG commitment com (MSM against
  the resident SRS) and the 4x coset evaluation that the quotient by
  X^N - 1 needs (one `zk_commit_job`);
* fold (Parallel Accumulation, prover step 5, on the job's commitments): the
  challenge gamma = rho(C_acc || com) from the device transcript, then
  C_acc'' = gamma * C_acc + com (`zk_transcript_challenge`, `zk_fold`).

Scheduling:

* `Admission` is the policy, free of any device code: jobs wait in arrival
  order; the head job starts as soon as a stream slot is free and its HBM
  footprint (caller buffers and library scratch) fits the budget next to the
  jobs already running (strict FIFO, so a large job is never starved by small
  ones behind it).  A job whose footprint exceeds the whole budget is
  rejected, and so is a job that arrives while `max_queue` jobs already wait.
* `GpuExecutor` runs each admitted job on its own HIP stream (all at the
  default priority), so jobs admitted while others are on the GPU overlap
  with them; completion is detected by polling an event per job.  Before
  each start it caps the library's scratch (cached blocks included) at the
  budget minus the caller buffers of the running jobs and this one, so the
  two together never exceed the budget; a start the library refuses with
  ZK_EBUDGET (cached and in-use scratch at the cap) raises `Busy`.
* `serve` drives a timed arrival stream through both and records per-job
  arrival, start and finish times (host clock).  `Busy` puts the job back at
  the head of the queue (back-pressure: it starts when running jobs release
  scratch).  A job whose start or completion raises anything else (a
  library error such as ZK_EDEVICE) is finished with `error` set and its
  slot and bytes released; the other jobs go on.

The executor is pluggable; the tests use a mock that only models durations
and bytes to check the admission logic on the CPU.
"""
import collections
import time

import numpy as np


class Busy(Exception):
    """The executor cannot start this job now; retry when running jobs finish."""


class Job:
    __slots__ = ("jid", "n", "N", "arrival", "offset", "acc_index", "start", "finish", "footprint", "handle",
                 "result", "error", "retries")

    def __init__(self, jid, n, arrival, offset=0, acc_index=0):
        self.jid = int(jid)
        self.n = int(n)
        self.N = 1 << max(0, (int(n) - 1).bit_length())
        self.arrival = float(arrival)
        self.offset = int(offset)
        self.acc_index = int(acc_index)
        self.start = None
        self.finish = None
        self.footprint = 0
        self.handle = None
        self.result = None
        self.error = None
        self.retries = 0


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

    def requeue(self, jobs):
        """Give admitted but unstarted jobs back, in order, to the queue head."""
        for job in reversed(jobs):
            self.release(job)
            self.queue.appendleft(job)


class GpuExecutor:
    """Runs commit-and-fold jobs on HIP streams through the C-ABI (one stream per slot).

    pool: (P, 8) device tensor of Fr values the jobs' witnesses are cut from;
    acc_pool: (A, 16) device tensor of G1 points, the jobs' input
    accumulators (None: commit only, no fold).  budget: the HBM budget the
    admission uses (None: the library's scratch is not capped)."""

    FOLD_SCRATCH = 1 << 16   # the two-instance fold's and transcript's scratch (bytes, a bound)

    def __init__(self, zk, srs, pool, slots, acc_pool=None, budget=None, keep_results=False, timing=False):
        import torch
        self.timing = timing
        self.zk = zk
        self.torch = torch
        self.srs = srs
        self.pool = pool
        self.acc_pool = acc_pool
        self.budget = budget
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free = list(range(slots))
        self.keep = keep_results
        self.live_caller = 0
        self.peak_scratch = 0
        self.peak_caller = 0
        self.busy_events = 0

    def caller_bytes(self, job):
        N = job.N
        pad = N * 32 if job.n < N else 0
        fold = 4 * 64 + 32 if self.acc_pool is not None else 0
        return N * 32 + 4 * N * 32 + pad + 64 + fold

    def footprint(self, job):
        N = job.N
        L = N.bit_length() - 1
        zk = self.zk
        scratch = (zk.msm_srs_workspace_bytes(self.srs, N) + zk.ntt_workspace_bytes(L)
                   + zk.ntt_workspace_bytes(L + 2))
        if self.acc_pool is not None:
            scratch += self.FOLD_SCRATCH
        return self.caller_bytes(job) + scratch

    def start(self, job):
        torch, zk = self.torch, self.zk
        mine = self.caller_bytes(job)
        if self.budget is not None:
            zk.set_scratch_budget(max(1, int(self.budget) - self.live_caller - mine))
        slot = self.free.pop()
        s = self.streams[slot]
        try:
            with torch.cuda.stream(s):
                N = job.N
                ev = self.pool[job.offset:job.offset + N]
                if job.n < N:
                    ev = torch.zeros((N, 8), dtype=torch.int32, device=ev.device)
                    ev[:job.n].copy_(self.pool[job.offset:job.offset + job.n])
                coeffs, com, coset = zk.commit_job(self.srs, ev, log_blowup=2)
                acc_out = None
                if self.acc_pool is not None:
                    inst = torch.empty((2, 1, 16), dtype=torch.int32, device=ev.device)
                    inst[0, 0].copy_(self.acc_pool[job.acc_index])
                    inst[1, 0].copy_(com[0])
                    gamma = zk.transcript_challenge(inst)
                    acc_out = zk.fold(inst, gamma)
                done = torch.cuda.Event(enable_timing=self.timing)
                done.record(s)
        except zk.ZkError as e:
            self.free.append(slot)
            if e.code == zk.ZK_EBUDGET:
                self.busy_events += 1
                raise Busy(str(e))
            raise
        except Exception:
            self.free.append(slot)
            raise
        self.live_caller += mine
        self.peak_caller = max(self.peak_caller, self.live_caller)
        self.peak_scratch = max(self.peak_scratch, zk.scratch_held())
        job.handle = (slot, done, com, coset, acc_out, coeffs, ev, mine)

    def poll(self, job):
        slot, done, com, coset, acc_out, coeffs, ev, mine = job.handle
        if not done.query():
            return False
        if self.keep:
            job.result = (self.zk.to_host(com).copy(), self.zk.to_host(coset).copy(),
                          None if acc_out is None else self.zk.to_host(acc_out).copy())
        job.handle = None
        self.live_caller -= mine
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
        batch = adm.admissible()
        for k, job in enumerate(batch):
            job.start = clock() - t0
            try:
                executor.start(job)
            except Busy as e:
                # back-pressure: this job and the rest of the batch go back to
                # the queue head; alone on the device, the refusal is final
                job.start = None
                others = [j for j in adm.running if j not in batch[k:]]
                if not others:
                    job.error = "failed: " + str(e)
                    job.start = job.finish = clock() - t0
                    adm.release(job)
                    finished.append(job)
                    adm.requeue(batch[k + 1:])
                else:
                    job.retries += 1
                    adm.requeue(batch[k:])
                break
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
            "max_ms": float(lat.max()), "failed": len(finished) - len(ok),
            "retried": int(sum(1 for j in finished if j.retries))}
