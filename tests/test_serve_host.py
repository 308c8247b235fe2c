"""Host-only tests of the serving scheduler (admission by slots and memory budget)."""
import pytest

from paper_2404_16517_amd.serve import Job, Scheduler, percentile


def test_admission_respects_slots_and_budget():
    s = Scheduler(budget_bytes=100, slots=2)
    for i, m in enumerate([60, 30, 30, 50]):
        s.submit(Job(i, 0.0, m))
    started = s.admissible()
    assert [j.rid for j in started] == [0, 1]          # slots full
    assert s.used_bytes == 90
    s.finish(started[0])
    started = s.admissible()
    assert [j.rid for j in started] == [2]             # 30 fits, 50 would not (30 + 30 + 50 > 100)
    s.finish(started[0])
    assert [j.rid for j in s.admissible()] == [3]
    assert s.used_bytes == 80


def test_backfill_is_bounded():
    s = Scheduler(budget_bytes=100, slots=8, max_bypass=2)
    s.submit(Job(0, 0.0, 90))
    first = s.admissible()
    assert [j.rid for j in first] == [0]
    s.submit(Job(1, 0.0, 50))    # head: does not fit while job 0 runs
    for i in range(2, 6):
        s.submit(Job(i, 0.0, 1))
    got = [j.rid for j in s.admissible()]
    assert got == [2, 3]         # only max_bypass jobs pass the head
    s.finish(first[0])
    got = [j.rid for j in s.admissible()]
    assert got[0] == 1           # the head goes first once memory is free


def test_oversized_request_refused():
    s = Scheduler(budget_bytes=10, slots=1)
    with pytest.raises(ValueError):
        s.submit(Job(0, 0.0, 11))


def test_deterministic_replay_of_a_poisson_trace():
    import synth
    reqs = synth.poisson_requests(50, qps=20.0, seed=3)
    again = synth.poisson_requests(50, qps=20.0, seed=3)
    assert [(r.arrival_s, r.n, r.kind, r.ratio) for r in reqs] == [(r.arrival_s, r.n, r.kind, r.ratio) for r in again]
    assert all(b.arrival_s > a.arrival_s for a, b in zip(reqs, reqs[1:]))
    s = Scheduler(budget_bytes=10**9, slots=3)
    for r in reqs:
        s.submit(Job(r.rid, r.arrival_s, r.n))
    order = []
    while s.queue or s.running:
        for j in s.admissible():
            order.append(j.rid)
        for rid in list(s.running)[:1]:
            s.finish(s.running[rid])
    assert sorted(order) == list(range(50))


def test_percentile():
    assert percentile([1, 2, 3, 4], 0.5) == 2.5
    assert percentile([5], 0.99) == 5


def test_results_stay_charged_until_released():
    s = Scheduler(budget_bytes=100, slots=4)
    a, b = Job(0, 0.0, 60, result_bytes=20), Job(1, 0.0, 50, result_bytes=10)
    s.submit(a)
    s.submit(b)
    assert [j.rid for j in s.admissible()] == [0]      # 60 + 50 > 100
    s.finish(a)
    assert s.used_bytes == 20                           # workspace back, results held
    assert [j.rid for j in s.admissible()] == [1]      # 20 + 50 <= 100
    s.finish(b)
    assert s.used_bytes == 30 and set(s.held) == {0, 1}
    s.release(a)
    s.release(b)
    assert s.used_bytes == 0 and not s.held


def test_stuck_when_held_results_block_the_head():
    s = Scheduler(budget_bytes=100, slots=2)
    a = Job(0, 0.0, 90, result_bytes=80)
    s.submit(a)
    s.admissible()
    s.finish(a)                                        # 80 still held
    s.submit(Job(1, 0.0, 30))
    assert s.admissible() == [] and s.stuck()
    s.release(a)
    assert not s.stuck() and [j.rid for j in s.admissible()] == [1]
