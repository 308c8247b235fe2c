"""Served mode on the GPU: every request's outputs in the continuous-batching
mix equal its outputs when run alone, bit for bit.

The budget admits only a few of the larger requests at once, so requests
queue, smaller ones are backfilled past a waiting head, and up to four run
concurrently on their own streams."""
import pytest
import torch

import synth
from paper_2404_16517_amd import serve

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _trace(count, seed, size_hi):
    reqs = synth.poisson_requests(count, qps=5000.0, size_lo=1e3, size_hi=size_hi, seed=seed)
    inputs = {r.rid: synth.request_strings(r, device=DEV) for r in reqs}
    torch.cuda.synchronize()
    return reqs, inputs


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_results_in_the_mix_equal_results_alone_under_a_tight_budget():
    """Poisson arrivals of mixed requests; the budget admits at most two of
    the largest at once."""
    reqs, inputs = _trace(40, 7, 3e5)
    alone, _ = serve.serve_sequential(reqs, inputs)
    sizes = {r.rid: serve.job_bytes(inputs[r.rid].n, inputs[r.rid].N)[0] for r in reqs}
    budget = int(2.2 * max(sizes.values()))
    bad = []

    def check(job):
        if not _same(job.result, alone[job.rid]):
            bad.append(job.rid)

    jobs, _ = serve.serve_trace(reqs, inputs, budget, slots=4, time_scale=1.0, on_done=check)
    assert not bad, f"results differ from the job run alone: {bad}"
    assert len(jobs) == len(reqs) and all(j.done_s is not None for j in jobs)
    order = sorted(jobs, key=lambda j: j.admitted_s)
    assert any(a.done_s > b.admitted_s for a, b in zip(order, order[1:]))  # jobs overlapped


def test_backfill_past_a_blocked_head_keeps_every_result():
    """Three large requests queued first, then small ones, all at once: the
    budget holds two large jobs, so the third waits at the head while small
    requests are admitted past it; every result equals the job run alone."""
    big = [synth.Request(i, 0.0, 400_000, "dn" if i % 2 else "text", 0.5, 90 + i) for i in range(3)]
    small = [synth.Request(3 + i, 0.0, 2_000 + 500 * i, "text" if i % 2 else "dn", 0.1, 200 + i)
             for i in range(8)]
    reqs = big + small
    inputs = {r.rid: synth.request_strings(r, device=DEV) for r in reqs}
    torch.cuda.synchronize()
    alone, _ = serve.serve_sequential(reqs, inputs)
    mem = {r.rid: serve.job_bytes(inputs[r.rid].n, inputs[r.rid].N)[0] for r in reqs}
    large = max(mem[r.rid] for r in big)
    budget = int(2.2 * large)
    assert sum(mem[r.rid] for r in big) > budget  # the third large one must wait
    bad = []
    jobs, _ = serve.serve_trace(reqs, inputs, budget, slots=4, time_scale=0.0,
                                on_done=lambda j: bad.append(j.rid) if not _same(j.result, alone[j.rid]) else None)
    assert not bad, bad
    adm = {j.rid: j.admitted_s for j in jobs}
    blocked = max(range(3), key=lambda r: adm[r])          # the large request admitted last
    assert any(adm[r.rid] < adm[blocked] for r in small)   # a small one passed it


def test_kept_results_stay_on_the_device_and_equal_results_alone():
    reqs, inputs = _trace(16, 11, 1e5)
    alone, _ = serve.serve_sequential(reqs, inputs)
    total = sum(sum(serve.job_bytes(inputs[r.rid].n, inputs[r.rid].N)) for r in reqs)
    jobs, _ = serve.serve_trace(reqs, inputs, total, slots=4, time_scale=0.0, keep_results=True)
    for j in jobs:
        assert all(t.is_cuda for t in j.result)
        assert _same(j.result, alone[j.rid]), j.rid
