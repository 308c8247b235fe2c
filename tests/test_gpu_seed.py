"""GPU parity of the shared first read: ss_dist_prefix_first_seed leaves, with
its first hash pass, each string's first mismatch with the first string of its
set; ss_sort_seeded / ss_sort_batch_seeded sort from it.  The seed's records
are checked against their definition (the LCP with that string, computed here
on the CPU), the sorts against the oracle and against the unseeded sorts, and
the rounds continuing from the same first pass against ss_dist_prefix.  All
comparisons exact.
"""
import os
import random
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2404_16517_amd as ss
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
WINDOW = 256  # bytes of every string the deep first pass reads
TILE = 32     # strings per wavefront tile of that pass; a tile across sets is left open from 0
MAX_SETS = 16  # sets the pass seeds (more: it writes no seed)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def _mixed(seed):
    """String 0 with a 300-byte run; strings agreeing with it past the window,
    prefixes of it, exact copies, empty strings and unrelated ones."""
    rng = random.Random(seed)
    s0 = b"P" * 300 + b"Q" * 40
    out = [s0]
    for i in range(3000):
        k = i % 6
        if k == 0:
            out.append(s0[: rng.randint(257, 340)] + bytes(rng.choice(b"AZ") for _ in range(rng.randint(0, 9))))
        elif k == 1:
            out.append(s0[: rng.randint(0, 340)])
        elif k == 2:
            out.append(s0)
        elif k == 3:
            out.append(b"")
        elif k == 4:
            out.append(b"P" * rng.randint(0, 300) + bytes([rng.choice(b"AOPZ")]) + b"x" * rng.randint(0, 20))
        else:
            out.append(bytes(rng.choice(b"PQ\x00") for _ in range(rng.randint(1, 30))))
    return synth.from_list(out)


def _zero_bytes(seed):
    """NUL bytes everywhere, string 0 short: differences past the shorter
    string's end must not count."""
    rng = random.Random(seed)
    out = [b"\x00" * 10]
    for _ in range(2000):
        out.append(bytes(rng.choice(b"\x00\x01") if rng.random() < 0.1 else 0 for _ in range(rng.randint(0, 300))))
    return synth.from_list(out)


CASES = {
    "dn": lambda: synth.dn_strings(20_000, 500, 0.5, seed=1),
    "dn_past_window": lambda: synth.dn_strings(5_000, 800, 0.6, seed=2),
    "mixed": lambda: _mixed(3),
    "short0": lambda: synth.from_list([b"PQ"] + [b"PQ" * random.Random(i).randint(0, 200) for i in range(1500)]),
    "empty0": lambda: synth.from_list([b""] + [bytes([65 + i % 3]) * (i % 290) for i in range(1500)]),
    "zero_bytes": lambda: _zero_bytes(4),
    "text": lambda: synth.text_strings(30_000, seed=3),
}


def _expected_records(b, o, bounds=None):
    """Per string: (resolved, r, tk, word) from the seed's definition."""
    n = len(o) - 1
    bounds = [0, n] if bounds is None else list(bounds)
    set_of = np.searchsorted(np.asarray(bounds[:-1]), np.arange(n), side="right") - 1
    recs = []
    for i in range(n):
        t0, t1 = TILE * (i // TILE), min(TILE * (i // TILE) + TILE - 1, n - 1)
        if set_of[t0] != set_of[t1]:
            recs.append((False, 0, None, None))
            continue
        f = bounds[set_of[i]]
        s0 = bytes(b[o[f]:o[f + 1]])
        si = bytes(b[o[i]:o[i + 1]])
        E = min(len(si), len(s0))
        lim = min(E, WINDOW)
        r = len(os.path.commonprefix([si[:lim], s0[:lim]]))
        if r < WINDOW or E <= WINDOW:
            tk = min(len(si) - r, 8)
            word = int.from_bytes(si[r:r + tk] + b"\x00" * (8 - tk), "big")
            recs.append((True, r, tk, word))
        else:
            recs.append((False, WINDOW, None, None))
    return recs


def _check_seed(seed, n, b, o, name, bounds=None):
    raw = seed.cpu().numpy()
    hdr = raw[:4].view(np.uint32)[0]
    assert hdr == 1, f"{name}: deep pass wrote no seed"
    words = raw[256:256 + 8 * n].view(np.uint64)
    pos = raw[256 + 8 * n:256 + 16 * n].view(np.uint32).reshape(n, 2)
    exp = _expected_records(b, o, bounds)
    for i, (res, r, tk, word) in enumerate(exp):
        if res:
            assert (pos[i, 0], pos[i, 1], int(words[i])) == (r, tk, word), f"{name}: string {i}"
        else:
            assert (pos[i, 0], pos[i, 1]) == (r, 0xFFFFFFFF), f"{name}: string {i} should stay open at {r}"


@pytest.mark.parametrize("mode", ["deep", "plain", "auto"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_seeded_sort_and_rounds(name, mode):
    s = CASES[name]()
    _log(f"[seed] {name} mode={mode} n={s.n} N={s.N}")
    g = s.to(DEV)
    b, o = oracle.strings_np(s)
    ws, seed = ss.dist_prefix_first_seed(g.bytes, g.offsets, 8, 64, first_pass=mode)
    torch.cuda.synchronize()
    if mode == "deep":
        _check_seed(seed, s.n, b, o, name)
    elif mode == "plain":
        assert seed.cpu().numpy()[:4].view(np.uint32)[0] == 0
    # the sort beside the remaining rounds, as a pipeline runs them
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        perm, lcp = ss.sort_seeded(g.bytes, g.offsets, seed)
    dpx, rounds = ss.dist_prefix_rounds(g.bytes, g.offsets, ws, 8, 64)
    torch.cuda.synchronize()
    p_ref = oracle.sort(b, o)
    np.testing.assert_array_equal(u32(perm), p_ref)
    np.testing.assert_array_equal(u32(lcp), oracle.lcp(b, o, p_ref))
    p2, l2 = ss.sort(g.bytes, g.offsets)
    d_ref, r_ref = ss.dist_prefix(g.bytes, g.offsets, 8, 64)
    torch.cuda.synchronize()
    assert torch.equal(perm, p2) and torch.equal(lcp, l2)
    assert rounds == r_ref and torch.equal(dpx, d_ref)


def test_seed_buffer_reused_for_a_smaller_set():
    """A seed buffer from a larger deep call, then a plain call on fewer
    strings: the header says no seed, and the sort ignores the stale records."""
    big = synth.dn_strings(8_000, 500, 0.5, seed=7).to(DEV)
    _, seed = ss.dist_prefix_first_seed(big.bytes, big.offsets, 8, 64, first_pass="deep")
    small = synth.text_strings(3_000, seed=8)
    g = small.to(DEV)
    _, seed2 = ss.dist_prefix_first_seed(g.bytes, g.offsets, 8, 64, first_pass="plain", seed=seed)
    assert seed2.data_ptr() == seed.data_ptr()
    perm, lcp = ss.sort_seeded(g.bytes, g.offsets, seed2)
    torch.cuda.synchronize()
    b, o = oracle.strings_np(small)
    p_ref = oracle.sort(b, o)
    np.testing.assert_array_equal(u32(perm), p_ref)
    np.testing.assert_array_equal(u32(lcp), oracle.lcp(b, o, p_ref))


def test_seeded_sort_few_strings_and_empty():
    """Up to 256 strings take the one-launch rank sort (the seed is unused);
    no strings: nothing to do."""
    s = synth.from_list([b"B" * 300, b"A" * 300, b"B" * 299, b""] * 40)
    g = s.to(DEV)
    _, seed = ss.dist_prefix_first_seed(g.bytes, g.offsets, 8, 64, first_pass="deep")
    perm, lcp = ss.sort_seeded(g.bytes, g.offsets, seed)
    torch.cuda.synchronize()
    b, o = oracle.strings_np(s)
    p_ref = oracle.sort(b, o)
    np.testing.assert_array_equal(u32(perm), p_ref)
    np.testing.assert_array_equal(u32(lcp), oracle.lcp(b, o, p_ref))
    e = synth.from_list([]).to(DEV)
    seed0 = torch.zeros(ss.lib().ss_sort_seed_bytes(0), dtype=torch.uint8, device=DEV)
    p0, _ = ss.sort_seeded(e.bytes, e.offsets, seed0)
    assert p0.numel() == 0


def _sets(name, n):
    rng = random.Random(len(name) + n)
    if name == "equal16":
        return [n * i // 16 for i in range(17)]
    if name == "ragged":  # empty sets, single strings, sizes that straddle tiles (16 sets)
        cuts = sorted(rng.sample(range(40, n), 9) + [5, 5, 6, 6, 7])
        return [0] + cuts + [n, n]
    if name == "tiny":  # many sets smaller than a tile: more than the pass seeds
        return list(range(0, n, 7)) + [n]
    raise KeyError(name)


@pytest.mark.parametrize("global_ids", [False, True])
@pytest.mark.parametrize("sets", ["equal16", "ragged", "tiny"])
@pytest.mark.parametrize("name", ["dn", "dn_past_window", "mixed", "zero_bytes"])
def test_seeded_batch_sort(name, sets, global_ids):
    s = CASES[name]()
    bounds = _sets(sets, s.n)
    _log(f"[seed batch] {name} sets={sets} ({len(bounds) - 1}) global_ids={global_ids} n={s.n}")
    g = s.to(DEV)
    so = torch.tensor(bounds, dtype=torch.int64, device=DEV)
    b, o = oracle.strings_np(s)
    ws, seed = ss.dist_prefix_first_seed(g.bytes, g.offsets, 8, 64, first_pass="deep", set_off=so)
    torch.cuda.synchronize()
    if len(bounds) - 1 <= MAX_SETS:
        _check_seed(seed, s.n, b, o, f"{name}/{sets}", bounds)
    else:
        assert seed.cpu().numpy()[:4].view(np.uint32)[0] == 0
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        perm, lcp = ss.sort_batch_seeded(g.bytes, g.offsets, so, seed, global_ids=global_ids)
    dpx, rounds = ss.dist_prefix_rounds(g.bytes, g.offsets, ws, 8, 64)
    torch.cuda.synchronize()
    p2, l2 = ss.sort_batch(g.bytes, g.offsets, so, global_ids=global_ids)
    d_ref, r_ref = ss.dist_prefix(g.bytes, g.offsets, 8, 64)
    torch.cuda.synchronize()
    assert torch.equal(perm, p2) and torch.equal(lcp, l2)
    assert rounds == r_ref and torch.equal(dpx, d_ref)
    if sets == "equal16" and global_ids:  # one set against the oracle directly
        lo, hi = bounds[3], bounds[4]
        sub = synth.from_list([bytes(b[o[i]:o[i + 1]]) for i in range(lo, hi)])
        bs, os_ = oracle.strings_np(sub)
        p_ref = oracle.sort(bs, os_)
        np.testing.assert_array_equal(u32(perm)[lo:hi] - lo, p_ref)
        np.testing.assert_array_equal(u32(lcp)[lo:hi], oracle.lcp(bs, os_, p_ref))
