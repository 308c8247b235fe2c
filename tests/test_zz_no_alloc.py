"""The allocation-free front-coding decode against the workspace one.

ss_fc_decode_noalloc keeps its scratch in a static device array and reports
data-dependent errors in a device status word; on valid runs its output must
equal ss_fc_decode's byte for byte, also on a second call with a smaller
input (the array keeps the first call's contents).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2404_16517_amd as ss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _runs(n, runs, seed):
    """Valid front-coded runs: e = 0 at each run start, e_i <= d_i, e_i <= d_(i-1)."""
    rng = np.random.default_rng(seed)
    d = rng.integers(1, 70, size=n).astype(np.int64)
    e = rng.integers(0, 60, size=n).astype(np.int64)
    e[: n // 3] = 17  # a plateau: previous-smaller values far away
    prev = np.concatenate([[0], d[:-1]])
    e = np.minimum(np.minimum(e, d), prev)
    run_off = np.linspace(0, n, runs + 1).astype(np.uint64)
    e[run_off[:-1].astype(np.int64)[run_off[:-1] < n]] = 0
    suf_off = np.concatenate([[0], np.cumsum(d - e)]).astype(np.uint64)
    suf = rng.integers(0, 256, size=max(int(suf_off[-1]), 1)).astype(np.uint8)
    return run_off, e.astype(np.uint32), d.astype(np.uint32), suf_off, suf


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a).view(dt).copy()).to(DEV)


def _both(n, runs, seed, cap_slack=0):
    run_off, e, d, suf_off, suf = _runs(n, runs, seed)
    args = (_dev(run_off, np.int64), _dev(e, np.int32), _dev(d, np.int32), _dev(suf_off, np.int64),
            torch.from_numpy(suf).to(DEV))
    ref_bytes, ref_off = ss.fc_decode(*args)
    total = int(d.astype(np.int64).sum())
    out_off = torch.full((n + 1,), -7, dtype=torch.int64, device=DEV)
    out = torch.full((max(total + cap_slack, 1),), 0xAB, dtype=torch.uint8, device=DEV)
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ss.fc_decode_noalloc(*args, out_off, out, status)
    torch.cuda.synchronize()
    return (run_off, e, d, suf_off, suf), (ref_bytes, ref_off), (out, out_off, int(status.item())), total


@pytest.mark.parametrize("first,second", [((300_000, 5), (4_100, 2)), ((2_000_000, 64), (1, 1))])
def test_noalloc_decode_equals_workspace_decode_twice(first, second):
    for (n, runs), seed in ((first, 1), (second, 2)):
        print(f"[noalloc decode] n={n} runs={runs}", flush=True)
        host, (rb, ro), (out, oo, st), total = _both(n, runs, seed, cap_slack=64)
        assert st == 0
        assert torch.equal(oo, ro)
        assert torch.equal(out[:total], rb)
        assert (out[total:] == 0xAB).all()  # nothing past the decoded bytes
        ob, ooff = oracle.fc_decode(*host[:4], host[4])
        np.testing.assert_array_equal(oo.cpu().numpy().view(np.uint64), ooff)
        assert bytes(out[:total].cpu().numpy()) == bytes(ob)


def test_noalloc_decode_at_the_size_limit_then_small():
    n = ss.SS_FC_DECODE_NOALLOC_MAX
    for nn, seed in ((n, 3), (1000, 4)):
        print(f"[noalloc decode] n={nn}", flush=True)
        _, (rb, ro), (out, oo, st), total = _both(nn, 7, seed)
        assert st == 0 and torch.equal(oo, ro) and torch.equal(out[:total], rb)


def test_noalloc_decode_reports_capacity_and_malformed_runs_on_the_device():
    run_off, e, d, suf_off, suf = _runs(5000, 3, 5)
    total = int(d.astype(np.int64).sum())
    args = [_dev(run_off, np.int64), _dev(e, np.int32), _dev(d, np.int32), _dev(suf_off, np.int64),
            torch.from_numpy(suf).to(DEV)]
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    oo = torch.empty(5001, dtype=torch.int64, device=DEV)
    out = torch.full((total - 1,), 0xAB, dtype=torch.uint8, device=DEV)
    ss.fc_decode_noalloc(*args, oo, out, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 2
    assert int(oo[-1].item()) == total  # offsets complete
    assert (out == 0xAB).all()          # no byte written
    bad = e.copy()
    bad[0] = 1  # a run must start with e = 0
    args[1] = _dev(bad, np.int32)
    out2 = torch.full((total,), 0xAB, dtype=torch.uint8, device=DEV)
    ss.fc_decode_noalloc(*args, oo, out2, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 1
    assert (out2 == 0xAB).all()


def test_noalloc_decode_rejects_sizes_beyond_the_limit():
    n = ss.SS_FC_DECODE_NOALLOC_MAX + 1
    assert ss.lib().ss_fc_decode_noalloc(1, None, None, None, None, None, n, None, None, 0, None, None) == -3
    assert b"limit" in ss.lib().ss_last_error()
