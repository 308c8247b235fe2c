"""Continuous-batching server for sort jobs on one GPU.

Requests (string arrays already in device memory) arrive over time.  A
request is admitted as soon as a worker slot is free and its device-memory
estimate fits in the remaining budget; admitted requests run concurrently,
each on its own HIP stream driven by its own host thread (the C-ABI releases
the GIL), so their kernels overlap on the device.  Requests that do not fit yet
wait; later, smaller ones may be admitted ahead of them (backfill) as long as
the head of the queue has waited less than ``max_bypass`` admissions.  Results
stay on the device and stay charged to the budget (with the request's input
strings) until they are released; a finished job gives back only its
workspace.  Latency is arrival -> results ready.

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
    mem_bytes: int          # everything the job holds while it runs
    payload: object = None
    result_bytes: int = 0   # the part still held after it finishes (input + outputs), until release
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
    held: dict = field(default_factory=dict)
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
        """The job's work is done: its workspace goes back to the budget; its
        input and results stay charged until ``release``."""
        del self.running[job.rid]
        self.used_bytes -= job.mem_bytes - job.result_bytes
        self.held[job.rid] = job

    def release(self, job: Job):
        """The caller is done with the job's results (and input)."""
        del self.held[job.rid]
        self.used_bytes -= job.result_bytes

    def stuck(self) -> bool:
        """Nothing runs, yet the head of the queue cannot start: only releases
        of held results can make room."""
        return bool(self.queue) and not self.running and \
            self.used_bytes + self.queue[0].mem_bytes > self.budget_bytes


def job_bytes(n: int, N: int) -> tuple[int, int]:
    """(device bytes while running, bytes still held after finishing) of one
    sort job: its input strings and outputs are held until release, its
    workspace only while it runs."""
    import paper_2404_16517_amd as ss
    L = ss.lib()
    held = N + 8 * (n + 1) + n * (4 + 4 + 4 + 4)  # input; perm, lcp, dist, dist_approx
    ws = max(L.ss_sort_workspace(n), L.ss_dist_prefix_workspace(n))
    return held + ws, held


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


def serve_trace(requests, inputs, budget_bytes: int, slots: int = 4, time_scale: float = 1.0,
                keep_results: bool = False, on_done=None):
    """Replay a request trace.  ``inputs[rid]`` is the request's device string set.

    ``on_done(job)`` (optional) is called by the job's worker thread once its
    results are ready, e.g. to consume them; the results are then released
    (the caller's hand-back), unless ``keep_results``: then they stay on the
    device and charged to the budget until the trace ends, and a head request
    that can never fit raises.  Returns (jobs, makespan_s)."""
    import torch
    sched = Scheduler(budget_bytes, slots)
    streams = [torch.cuda.Stream() for _ in range(slots)]
    free_streams = list(range(slots))
    lock = threading.Condition()
    done_events = []
    jobs = {}
    for r in requests:
        mem, held = job_bytes(inputs[r.rid].n, inputs[r.rid].N)
        jobs[r.rid] = Job(r.rid, r.arrival_s * time_scale, mem, inputs[r.rid], held)
    pending = sorted(jobs.values(), key=lambda j: j.arrival_s)
    t0 = time.perf_counter()
    threads = []
    errors = []

    def worker(job, sidx):
        try:
            job.result = run_job(job.payload, streams[sidx])
            if on_done is not None:
                on_done(job)
        except BaseException as exc:  # reported after the trace
            errors.append(exc)
        with lock:
            job.done_s = time.perf_counter() - t0
            sched.finish(job)
            if not keep_results:
                sched.release(job)
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
            if sched.stuck():
                raise RuntimeError("budget held by kept results: the next request can never be admitted")
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
    if errors:
        raise errors[0]
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
