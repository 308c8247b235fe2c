"""Continuous-batching server for sort jobs on one GPU.

Requests (string arrays already in device memory) arrive over time.  A
request is admitted as soon as a worker slot is free and its device-memory
estimate fits in the remaining budget; admitted requests run concurrently,
each on its own HIP stream driven by its own host thread (the C-ABI releases
the GIL), so their kernels overlap on the device.  Requests that do not fit yet
wait; later, smaller ones may be admitted ahead of them (backfill) as long as
the head of the queue has waited less than ``max_bypass`` admissions.  Results
stay on the device.  Latency is arrival -> results ready.

The scheduling logic (``Scheduler``) is pure host code and is tested without a
GPU; ``serve_trace`` runs it with the real executor.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field


@dataclass
class Job:
    rid: int
    arrival_s: float
    mem_bytes: int
    payload: object = None
    admitted_s: float | None = None
    done_s: float | None = None
    result: object = None


@dataclass
class Scheduler:
    """Admission by free slots and a device-memory budget (host logic only)."""

    budget_bytes: int
    slots: int
    max_bypass: int = 8
    used_bytes: int = 0
    running: dict = field(default_factory=dict)
    queue: list = field(default_factory=list)
    _bypassed: int = 0

    def submit(self, job: Job):
        if job.mem_bytes > self.budget_bytes:
            raise ValueError(f"request {job.rid} needs {job.mem_bytes} bytes, budget is {self.budget_bytes}")
        self.queue.append(job)

    def admissible(self) -> list[Job]:
        """Jobs to start now (removed from the queue, accounted as running)."""
        out = []
        i = 0
        while i < len(self.queue) and len(self.running) < self.slots:
            job = self.queue[i]
            if i > 0 and self._bypassed >= self.max_bypass:
                break  # stop backfilling until the head of the queue fits
            if self.used_bytes + job.mem_bytes <= self.budget_bytes:
                self.queue.pop(i)
                self.running[job.rid] = job
                self.used_bytes += job.mem_bytes
                out.append(job)
                self._bypassed = 0 if i == 0 else self._bypassed + 1
                continue  # index i now holds the next queued job
            i += 1
        return out

    def finish(self, job: Job):
        del self.running[job.rid]
        self.used_bytes -= job.mem_bytes


def job_mem_bytes(n: int, N: int) -> int:
    """Device memory of one sort job: its strings, outputs and workspaces."""
    import paper_2404_16517_amd as ss
    L = ss.lib()
    outputs = n * (4 + 4 + 4 + 4)  # perm, lcp, dist, dist_approx
    ws = max(L.ss_sort_workspace(n), L.ss_dist_prefix_workspace(n))
    return N + 8 * (n + 1) + outputs + ws


def run_job(strings, stream, ws=None):
    """The served work: sort + LCP + exact and approximate distinguishing prefixes."""
    import torch
    import paper_2404_16517_amd as ss
    with torch.cuda.stream(stream):
        perm, lcp = ss.sort(strings.bytes, strings.offsets)
        dist = ss.dist_exact(strings.offsets, perm, lcp)
        dpx, _ = ss.dist_prefix(strings.bytes, strings.offsets, 8, 64)
        stream.synchronize()
    return perm, lcp, dist, dpx


def serve_trace(requests, inputs, budget_bytes: int, slots: int = 4, time_scale: float = 1.0):
    """Replay a request trace.  ``inputs[rid]`` is the request's device string set.
    Returns (jobs, makespan_s)."""
    import torch
    sched = Scheduler(budget_bytes, slots)
    streams = [torch.cuda.Stream() for _ in range(slots)]
    free_streams = list(range(slots))
    lock = threading.Condition()
    done_events = []
    jobs = {r.rid: Job(r.rid, r.arrival_s * time_scale,
                       job_mem_bytes(inputs[r.rid].n, inputs[r.rid].N), inputs[r.rid]) for r in requests}
    pending = sorted(jobs.values(), key=lambda j: j.arrival_s)
    t0 = time.perf_counter()
    threads = []

    def worker(job, sidx):
        job.result = run_job(job.payload, streams[sidx])
        with lock:
            job.done_s = time.perf_counter() - t0
            sched.finish(job)
            free_streams.append(sidx)
            done_events.append(job.rid)
            lock.notify_all()

    nxt = 0
    finished = 0
    with lock:
        while finished < len(jobs):
            now = time.perf_counter() - t0
            while nxt < len(pending) and pending[nxt].arrival_s <= now:
                sched.submit(pending[nxt])
                nxt += 1
            for job in sched.admissible():
                job.admitted_s = now
                sidx = free_streams.pop()
                th = threading.Thread(target=worker, args=(job, sidx), daemon=True)
                threads.append(th)
                th.start()
            finished = len(done_events)
            if finished >= len(jobs):
                break
            wait = None
            if nxt < len(pending):
                wait = max(0.0, pending[nxt].arrival_s - (time.perf_counter() - t0))
            lock.wait(timeout=wait if wait is not None else 0.05)
            finished = len(done_events)
    for th in threads:
        th.join()
    makespan = max(j.done_s for j in jobs.values()) - min(j.arrival_s for j in jobs.values())
    return list(jobs.values()), makespan


def serve_sequential(requests, inputs):
    """Baseline: one job at a time on one stream, in arrival order."""
    import torch
    st = torch.cuda.Stream()
    t0 = time.perf_counter()
    out = {}
    for r in sorted(requests, key=lambda r: r.arrival_s):
        out[r.rid] = run_job(inputs[r.rid], st)
    return out, time.perf_counter() - t0


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)
