"""GPU parity: every entry point of the C-ABI against the CPU oracle, bit-exact.

Inputs are seeded synthetic workloads (synth) and hand-picked edge sets.
All comparisons are integer and exact (tolerance 0).
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
from tests import closed_forms as cf

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


EDGE_SETS = {
    "n1": [b"HELLO"],
    "n2_equal": [b"AB", b"AB"],
    "n2": [b"B", b"A"],
    "empty_strings": [b"", b"", b"A", b""],
    "all_equal": [b"SAME" * 5] * 300,
    "prefix_chain": [b"A" * k for k in range(40, 0, -1)] + [b""],
    "word_boundaries": [bytes([65 + (i % 3)]) * L for i, L in enumerate([7, 8, 9, 15, 16, 17, 6, 14, 1, 0, 23, 24, 25])],
    "zero_ff": [b"\x00", b"\x00\x00", b"", b"\xff", b"\xff\x00", b"\x00\xff", b"A\x00", b"A", b"A\x00\x00"],
    "long_among_short": [b"Q" * 4096 + b"Z"] + [b"Q" * k for k in range(1, 60)] + [b"Q" * 4096 + b"A"],
    "deep_shared": [b"P" * 300 + bytes([65 + (i * 7) % 26]) + b"X" * (i % 5) for i in range(500)],
}


@pytest.mark.parametrize("name", ["n1", "n2_equal", "empty_strings", "prefix_chain", "zero_ff", "deep_shared"])
@pytest.mark.parametrize("by_input", [True, False])
def test_dist_exact_bounded_any_bound(name, by_input):
    """dist from any bound dist <= d <= len equals the oracle's exact dist,
    written by input index (perm given) or by sorted position (perm NULL)."""
    s = synth.from_list(EDGE_SETS[name])
    _log(f"[dist_bounded] {name} by_input={by_input}")
    b, o = oracle.strings_np(s)
    p_ref = oracle.sort(b, o)
    l_ref = oracle.lcp(b, o, p_ref)
    d_ref = oracle.dist_exact(o, p_ref, l_ref)
    lens = np.diff(o.astype(np.int64))
    rng = np.random.default_rng(3)
    # a bound per sorted position anywhere in [dist, len]
    lo = d_ref[p_ref].astype(np.int64)
    hi = lens[p_ref]
    bound = (lo + (rng.random(s.n) * (hi - lo + 1)).astype(np.int64)).astype(np.uint32)
    perm = torch.from_numpy(p_ref.view(np.int32)).to(DEV)
    lcp_ = torch.from_numpy(l_ref.view(np.int32)).to(DEV)
    d = torch.from_numpy(bound.view(np.int32)).to(DEV)
    out = ss.dist_exact_bounded(perm if by_input else None, lcp_, d)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(out), d_ref if by_input else d_ref[p_ref])


def _rand_strings(rng, n, alphabet, max_len):
    return [bytes(rng.choice(alphabet) for _ in range(rng.randint(0, max_len))) for _ in range(n)]


def _check_sort(s: synth.StringSet, name=""):
    _log(f"[sort] {name} n={s.n} N={s.N}")
    g = s.to(DEV)
    perm, lcp = ss.sort(g.bytes, g.offsets)
    torch.cuda.synchronize()
    b, o = oracle.strings_np(s)
    p_ref = oracle.sort(b, o)
    np.testing.assert_array_equal(u32(perm), p_ref)
    np.testing.assert_array_equal(u32(lcp), oracle.lcp(b, o, p_ref))
    return g, perm, lcp, b, o, p_ref


@pytest.mark.parametrize("name", sorted(EDGE_SETS))
def test_sort_lcp_dist_edge_sets(name):
    s = synth.from_list(EDGE_SETS[name])
    g, perm, lcp, b, o, p_ref = _check_sort(s, name)
    # the same set through the round-based path (a one-set batch)
    pb, lb = ss.sort_batch(g.bytes, g.offsets, torch.tensor([0, s.n], device=DEV))
    np.testing.assert_array_equal(u32(pb), p_ref)
    np.testing.assert_array_equal(u32(lb), u32(lcp))
    d = ss.dist_exact(g.offsets, perm, lcp)
    lcp_ref = oracle.lcp(b, o, p_ref)
    np.testing.assert_array_equal(u32(d), oracle.dist_exact(o, p_ref, lcp_ref))
    l2 = ss.lcp(g.bytes, g.offsets, perm)
    np.testing.assert_array_equal(u32(l2), lcp_ref)


@pytest.mark.parametrize("seed", range(6))
def test_sort_random_small_alphabets(seed):
    rng = random.Random(seed)
    alpha = [(0, 1, 255), (65, 66), tuple(range(256)), (0,)][seed % 4]
    strs = _rand_strings(rng, rng.choice([5, 100, 3000, 20000]), alpha, rng.choice([3, 12, 40]))
    _check_sort(synth.from_list(strs), f"random seed={seed}")


@pytest.mark.parametrize("seed", [0, 1])
def test_sort_segment_size_boundaries(seed):
    """Groups whose sizes straddle the per-wavefront (64, 128) and LDS cutovers,
    with duplicates and equal 8-byte windows inside groups (next-round runs)."""
    rng = random.Random(seed)
    strs = []
    for size in [2, 3, 17, 63, 64, 65, 127, 128, 129, 200, 1000, 1025]:
        for i in range(size):
            tail = bytes(rng.choice(b"AB") for _ in range(rng.randint(0, 12)))
            if i % 5 == 0:
                tail = b"SAMEWINDOW" + tail  # equal key windows, strings continue
            strs.append(b"G%04d:" % size + tail)
    strs += strs[: len(strs) // 7]  # exact duplicates
    rng.shuffle(strs)
    _check_sort(synth.from_list(strs), f"size-boundaries seed={seed}")


@pytest.mark.parametrize("n", [2, 3, 64, 200, 255, 256, 257])
def test_sort_few_strings(n):
    """Up to 256 strings take the one-launch rank sort: duplicates, empty
    strings, prefixes of each other and common prefixes longer than one
    512-byte comparison round."""
    rng = random.Random(n)
    strs = []
    for i in range(n):
        kind = i % 5
        if kind == 0:
            strs.append(b"")
        elif kind == 1:
            strs.append(b"L" * rng.choice([511, 512, 513, 700, 1030]) + bytes([rng.choice(b"AB")]))
        elif kind == 2:
            strs.append(b"L" * rng.randint(0, 40))
        else:
            strs.append(bytes(rng.choice(b"ABC") for _ in range(rng.randint(1, 10))))
    strs += strs[: n // 9]
    strs = strs[:n]
    rng.shuffle(strs)
    _check_sort(synth.from_list(strs), f"few n={n}")


def test_sort_empty_input():
    g = synth.from_list([]).to(DEV)
    perm, lcp = ss.sort(g.bytes, g.offsets)
    assert perm.numel() == 0


@pytest.mark.parametrize("tune", [(128, 1024, 8), (256, 2048, 8), (1024, 4096, 8), (512, 16384, 8),
                                  (1024, 4096, 11), (512, 8192, 11), (1024, 16384, 11), (256, 4096, 11)])
def test_sort_tuning_variants_same_result(tune):
    sm, tile, bits = tune
    old_sm = ss.set_tuning(ss.SS_TUNE_SMALL_MAX, sm)
    old_t = ss.set_tuning(ss.SS_TUNE_TILE, tile)
    old_b = ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, bits)
    try:
        s = synth.text_strings(60_000, seed=4, median=12)
        _check_sort(s, f"tuning {tune}")
    finally:
        ss.set_tuning(ss.SS_TUNE_SMALL_MAX, old_sm)
        ss.set_tuning(ss.SS_TUNE_TILE, old_t)
        ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, old_b)


@pytest.mark.parametrize("kind", ["dn_500", "text", "sets", "edge_deep", "zero_ff_runs"])
@pytest.mark.parametrize("device_driven", [False, True])
def test_sort_with_11_bit_digits(kind, device_driven):
    """Six levels of 11 bits per key (the last ending with the length byte):
    the same order and LCPs as the oracle, host- and device-driven."""
    if kind == "dn_500":
        s, bounds = synth.concat([synth.dn_strings(150_000, 500, 0.5, seed=s) for s in range(2)])
    elif kind == "text":
        s, bounds = synth.concat([synth.text_strings(120_000, seed=9, median=12), synth.text_strings(5_000, seed=8)])
    elif kind == "sets":
        s, bounds = synth.random_sets(40, 2_000, 60_000, 8, 64, seed=2)
    elif kind == "edge_deep":
        s, bounds = synth.concat([synth.from_list(EDGE_SETS["deep_shared"] * 4),
                                  synth.from_list(EDGE_SETS["all_equal"] * 3)])
    else:
        rng = random.Random(5)
        strs = [bytes(rng.choice(b"\x00\xff") for _ in range(rng.randint(0, 20))) for _ in range(30_000)]
        s, bounds = synth.concat([synth.from_list(strs)])
    old = [ss.set_tuning(ss.SS_TUNE_SMALL_MAX, 512), ss.set_tuning(ss.SS_TUNE_TILE, 4096),
           ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, 11)]
    try:
        g = s.to(DEV)
        so = bounds.to(DEV)
        if device_driven:
            n = s.n
            perm = torch.empty(n, dtype=torch.int32, device=DEV)
            lcp = torch.empty(n, dtype=torch.int32, device=DEV)
            status = torch.full((2,), -1, dtype=torch.int32, device=DEV)
            ws = torch.empty(ss.lib().ss_sort_workspace(n), dtype=torch.uint8, device=DEV)
            max_len = int((s.offsets[1:] - s.offsets[:-1]).max())
            ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, ss.sort_batch_device_rounds(max_len))
            torch.cuda.synchronize()
            assert status.tolist() == [0, 0]
        else:
            perm, lcp = ss.sort_batch(g.bytes, g.offsets, so)
            torch.cuda.synchronize()
    finally:
        ss.set_tuning(ss.SS_TUNE_SMALL_MAX, old[0])
        ss.set_tuning(ss.SS_TUNE_TILE, old[1])
        ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, old[2])
    b, o = oracle.strings_np(s)
    bl = bounds.tolist()
    for j in range(len(bl) - 1):
        a, c = bl[j], bl[j + 1]
        sb, sob = b[o[a]:o[c]], o[a:c + 1] - o[a]
        p_ref = oracle.sort(sb, sob)
        np.testing.assert_array_equal(u32(perm[a:c]), p_ref, err_msg=f"set {j}")
        np.testing.assert_array_equal(u32(lcp[a:c]), oracle.lcp(sb, sob, p_ref), err_msg=f"set {j}")


def test_sort_c0_closed_form_and_oracle():
    """C0: 100,000 x 100 B, D/N 0.5."""
    s = synth.dn_strings(100_000, 100, 0.5, seed=0)
    g, perm, lcp, b, o, p_ref = _check_sort(s, "C0")
    pi = s.meta["pi"].numpy()
    np.testing.assert_array_equal(u32(perm), cf.dn_perm(pi))
    np.testing.assert_array_equal(u32(lcp), cf.dn_lcp(s.n, s.meta["k"], s.meta["filler"]))
    d = ss.dist_exact(g.offsets, perm, lcp)
    np.testing.assert_array_equal(u32(d)[u32(perm)], cf.dn_dist_sorted(s.n, s.meta["k"], s.meta["filler"], 100))


def test_sort_text_with_duplicates():
    s = synth.text_strings(200_000, seed=1)
    _check_sort(s, "text 200k")


@pytest.mark.parametrize("seed", [0, 1])
def test_sort_long_ties_in_small_segments(seed):
    """Groups of 2..90 strings that share 10..300 bytes (past several 7-byte
    keys and past the wavefront sort's own further keys), exact duplicates
    of every length among them, strings that are prefixes of others: the
    small-segment sorts resolve some ties themselves and hand the rest on."""
    rng = random.Random(seed)
    out = []
    for _ in range(1500):
        pre = bytes(rng.choice(b"ab") for _ in range(rng.randint(10, 300)))
        for _ in range(rng.randint(2, 90)):
            k = rng.random()
            if k < 0.3:
                out.append(pre)  # duplicates of the prefix itself
            elif k < 0.5:
                out.append(pre[: rng.randint(0, len(pre))])  # a prefix
            else:
                out.append(pre + bytes(rng.choice(b"xy") for _ in range(rng.randint(0, 12))))
    rng.shuffle(out)
    _check_sort(synth.from_list(out), f"long ties {seed}")


def test_sort_batch_equals_single_sorts():
    sets, bounds = synth.random_sets(64, 10, 3000, seed=3)
    _log(f"[batch] n={sets.n}")
    g = sets.to(DEV)
    perm, lcp = ss.sort_batch(g.bytes, g.offsets, bounds.to(DEV))
    torch.cuda.synchronize()
    P, Lc = u32(perm), u32(lcp)
    b, o = oracle.strings_np(sets)
    for j in range(64):
        a, e = int(bounds[j]), int(bounds[j + 1])
        sub_o = (o[a:e + 1] - o[a]).astype(np.uint64)
        sub_b = b[int(o[a]):int(o[e])]
        pr = oracle.sort(sub_b, sub_o)
        np.testing.assert_array_equal(P[a:e], pr)
        np.testing.assert_array_equal(Lc[a:e], oracle.lcp(sub_b, sub_o, pr))


def test_sort_batch_global_ids():
    sets, bounds = synth.random_sets(9, 1, 5000, seed=4)
    g = sets.to(DEV)
    pl, ll = ss.sort_batch(g.bytes, g.offsets, bounds.to(DEV))
    pg, lg = ss.sort_batch(g.bytes, g.offsets, bounds.to(DEV), global_ids=True)
    base = np.repeat(bounds[:-1].numpy(), (bounds[1:] - bounds[:-1]).numpy()).astype(np.uint32)
    np.testing.assert_array_equal(u32(pg), u32(pl) + base)
    np.testing.assert_array_equal(u32(lg), u32(ll))


def test_sort_batch_rejects_malformed_sets():
    s = synth.from_list([b"A", b"B", b"C"])
    g = s.to(DEV)
    for bad in ([0, 2, 1, 3], [0, 1, 2], [1, 2, 3]):
        with pytest.raises(ss.StrsortError):
            ss.sort_batch(g.bytes, g.offsets, torch.tensor(bad, device=DEV))


def test_sort_batch_with_empty_and_single_sets():
    strs = [b"C", b"A", b"B", b"Z", b"Y", b"Y"]
    s = synth.from_list(strs)
    bounds = torch.tensor([0, 0, 3, 3, 4, 6, 6], dtype=torch.int64)
    g = s.to(DEV)
    perm, lcp = ss.sort_batch(g.bytes, g.offsets, bounds.to(DEV))
    assert list(u32(perm)) == [1, 2, 0, 0, 0, 1]
    assert list(u32(lcp)) == [0, 0, 0, 0, 0, 1]


# ------------------------------------------------------------- prefix doubling

def test_doubling_keys_match_golden_vectors():
    """Every round's key of the frozen vectors, through the matrix-core passes
    (plain and deep first pass, then round passes up to 4096 bytes)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "kr_vectors.txt")
    data, keys = [], []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        h, k = line.split()
        data.append(bytes.fromhex(h) if h != "-" else b"")
        keys.append(int(k, 16))
    assert max(len(x) for x in data) <= 4096
    g = synth.from_list(data).to(DEV)
    for mode in ("plain", "deep"):
        got = ss.doubling_keys(g.bytes, g.offsets, 4, 11, 64, first_pass=mode)  # l = 4 .. 4096
        last = u64(got[-1])
        assert [int(x) for x in last] == keys, mode
        for t in range(11):
            l = 4 << t
            assert [int(x) for x in u64(got[t])] == [oracle.kr_key(x[:l]) for x in data], (mode, t)


def _key_strings(seed):
    """Text strings of mixed lengths (up to 2100 bytes) plus strings sharing
    long prefixes, at every alignment of the byte buffer."""
    rng = random.Random(seed)
    strs = synth.text_strings(1500, seed=seed, median=30).as_list()
    strs += [b"Q" * rng.randint(0, 300) + bytes(rng.randrange(256) for _ in range(rng.randint(0, 40)))
             for _ in range(400)]
    strs += [bytes(rng.randrange(256) for _ in range(rng.randint(1000, 2100))) for _ in range(60)]
    strs += [b"", b"\x00", b"\xff" * 64, b"\x00" * 129]
    rng.shuffle(strs)
    return strs


@pytest.mark.parametrize("mode", ["plain", "deep", "auto"])
@pytest.mark.parametrize("init_len,bits", [(8, 64), (4, 64), (16, 20), (12, 64), (64, 8)])
def test_doubling_keys_key_for_key(mode, init_len, bits):
    """Keys of the first pass (plain or deep), the single-round and the
    two-round passes equal the oracle's Karp-Rabin keys of each prefix, masked
    to the low ``bits`` bits, for every string and round."""
    strs = _key_strings(init_len + bits)
    for lead in (0, 3):  # shift every string's alignment
        g = synth.from_list([b"#" * lead] + strs).to(DEV)
        rounds = 0
        while (init_len << rounds) < 2400:
            rounds += 1
        got = ss.doubling_keys(g.bytes, g.offsets, init_len, rounds, bits, first_pass=mode)
        mask = (1 << bits) - 1 if bits < 64 else (1 << 64) - 1
        allstr = [b"#" * lead] + strs
        for t in range(rounds):
            l = init_len << t
            exp = [oracle.kr_key(x[:l]) & mask for x in allstr]
            assert [int(x) for x in u64(got[t])] == exp, (lead, t, l)


def _deep_mixed(seed):
    """Strings sharing 100+ bytes: some distinguished by 128 bytes, some by 256,
    duplicated ones that end at 300 bytes, and a group sharing 1500 bytes, so
    that rounds are skipped, hashed two at a time, and shrink in between."""
    rng = random.Random(seed)
    rnd = lambda k: bytes(rng.choice(b"ACGT") for _ in range(k))
    strs = [b"P" * 100 + rnd(20) for _ in range(1000)]
    strs += [b"P" * 200 + rnd(20) for _ in range(1000)]
    dups = [b"P" * 280 + rnd(20) for _ in range(30)]
    strs += [d for d in dups for _ in range(10)]
    strs += [b"P" * 1500 + rnd(10) for _ in range(500)]
    rng.shuffle(strs)
    return synth.from_list(strs)


@pytest.mark.parametrize("case", ["c0", "text", "text_bits12", "text_bits8", "edge", "dn_long", "deep_mixed"])
def test_dist_prefix_matches_oracle(case):
    if case == "c0":
        s, bits = synth.dn_strings(100_000, 100, 0.5, seed=0), 64
    elif case == "dn_long":
        s, bits = synth.dn_strings(50_000, 500, 0.5, seed=3), 64
    elif case == "deep_mixed":
        s, bits = _deep_mixed(4), 64
    elif case == "edge":
        s, bits = synth.from_list(EDGE_SETS["prefix_chain"] + EDGE_SETS["zero_ff"] + EDGE_SETS["all_equal"]), 64
    else:
        s = synth.text_strings(100_000, seed=2)
        bits = {"text": 64, "text_bits12": 12, "text_bits8": 8}[case]
    _log(f"[dist_prefix] {case} n={s.n}")
    g = s.to(DEV)
    d, rounds = ss.dist_prefix(g.bytes, g.offsets, 8, bits)
    b, o = oracle.strings_np(s)
    ref, r_ref, coll = oracle.dist_prefix(b, o, 8, bits)
    np.testing.assert_array_equal(u32(d), ref)
    assert rounds == r_ref


def _very_deep(seed):
    """Groups sharing 700, 2100 and 4500 bytes (several 1024-byte chunks of
    the later doubling rounds), with duplicates among the deepest."""
    rng = random.Random(seed)
    rnd = lambda k: bytes(rng.choice(b"ACGT") for _ in range(k))
    strs = [b"Q" * 700 + rnd(12) for _ in range(300)]
    strs += [b"Q" * 2100 + rnd(12) for _ in range(300)]
    deep = [b"Q" * 4500 + rnd(6) for _ in range(40)]
    strs += [x for x in deep for _ in range(3)]
    strs += [b"Q" * k for k in range(0, 5000, 97)]
    rng.shuffle(strs)
    return synth.from_list(strs)


@pytest.mark.parametrize("init_len", [4, 12, 64, 100, 128])
@pytest.mark.parametrize("bits", [64, 16])
def test_dist_prefix_init_lengths(init_len, bits):
    """First-pass and later rounds at every alignment of the round lengths
    (rounds that start inside a 64-byte step, no first pass at all)."""
    s = _very_deep(init_len + bits)
    _log(f"[dist_prefix] very_deep init={init_len} bits={bits} n={s.n}")
    g = s.to(DEV)
    d, rounds = ss.dist_prefix(g.bytes, g.offsets, init_len, bits)
    b, o = oracle.strings_np(s)
    ref, r_ref, coll = oracle.dist_prefix(b, o, init_len, bits)
    np.testing.assert_array_equal(u32(d), ref)
    assert rounds == r_ref


@pytest.mark.parametrize("case", ["text300k_bits64", "text300k_bits20", "dn200k", "dups200k"])
def test_dist_prefix_two_level_detection(case):
    """Lists long enough for the bitmap pre-filter of duplicate detection:
    unique keys, keys colliding by the hash width, and many repeated strings."""
    if case.startswith("text"):
        s, bits = synth.text_strings(300_000, seed=21), int(case.split("bits")[1])
    elif case == "dn200k":
        s, bits = synth.dn_strings(200_000, 120, 0.5, seed=22), 64
    else:
        base = synth.text_strings(70_000, seed=23, median=16).as_list()
        rng = random.Random(23)
        s, bits = synth.from_list([rng.choice(base) for _ in range(200_000)]), 64
    _log(f"[dist_prefix] {case} n={s.n}")
    g = s.to(DEV)
    d, rounds = ss.dist_prefix(g.bytes, g.offsets, 8, bits)
    b, o = oracle.strings_np(s)
    ref, r_ref, coll = oracle.dist_prefix(b, o, 8, bits)
    np.testing.assert_array_equal(u32(d), ref)
    assert rounds == r_ref


def _deep_mix(n, shared, frac_odd, seed):
    """Most strings share a `shared`-byte prefix (so the first pass also reads
    to 256 bytes); a fraction differs early, some are short or end inside the
    deep rounds, and repeats make duplicates at every depth."""
    rng = random.Random(seed)
    pre = bytes(rng.choice(b"ACGT") for _ in range(shared))
    out = []
    for k in range(n):
        u = rng.random()
        if u < frac_odd:  # differs early, random length
            out.append(bytes(rng.choice(b"ACGT") for _ in range(rng.randint(0, 90))))
        elif u < frac_odd + 0.02 and out:  # a repeat of an earlier string
            out.append(out[rng.randrange(len(out))])
        else:  # shared prefix, then a tail that ends anywhere up to 400 bytes
            tail = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(0, 400 - shared)))
            out.append(pre + tail)
    return synth.from_list(out)


def _equal_but_last(n, length, at, seed):
    """n copies of one string; the last (in input order, so in the last
    workgroup of the pass) differs at byte `at` (none when at is None)."""
    rng = random.Random(seed)
    base = bytes(rng.choice(b"ACGT") for _ in range(length))
    strs = [base] * n
    if at is not None:
        strs[-1] = base[:at] + bytes([base[at] ^ 1]) + base[at + 1:]
    return synth.from_list(strs)


@pytest.mark.parametrize("case", ["deep5", "deep5_bits12", "deep8_init4", "shallow30", "deep_shared100",
                                  "deep_all_equal", "deep_odd_last20", "deep_odd_last200"])
def test_dist_prefix_deep_first_pass(case):
    """The first pass's deep form (rounds 128 and 256 read with rounds <= 64)
    against the oracle: lists where the sample decides for it (and, shallow30,
    against it), with early finishers, short strings, strings ending inside
    the deep rounds, repeats, and narrow keys whose collisions decide; and
    rounds whose keys are all equal, or all equal but one in the last
    workgroup (the per-workgroup flags must combine across the grid)."""
    bits, init = 64, 8
    if case == "deep_all_equal":
        s = _equal_but_last(40_000, 300, None, seed=36)
    elif case == "deep_odd_last20":
        s = _equal_but_last(40_000, 300, 20, seed=37)
    elif case == "deep_odd_last200":
        s = _equal_but_last(40_000, 300, 200, seed=38)
    elif case == "deep5":
        s = _deep_mix(40_000, 150, 0.05, seed=31)
    elif case == "deep5_bits12":
        s, bits = _deep_mix(40_000, 150, 0.05, seed=32), 12
    elif case == "deep8_init4":
        s, init = _deep_mix(40_000, 140, 0.06, seed=33), 4
    elif case == "shallow30":
        s = _deep_mix(40_000, 150, 0.30, seed=34)
    else:
        s = _deep_mix(20_000, 300, 0.0, seed=35)
    _log(f"[dist_prefix deep] {case} n={s.n}")
    g = s.to(DEV)
    ss.profile_enable(True)  # (the records name the first-pass kernel that worked)
    try:
        d, rounds = ss.dist_prefix(g.bytes, g.offsets, init, bits)
        torch.cuda.synchronize()
        ran = ss.profile_report()
    finally:
        ss.profile_enable(False)
    deep = "k_hash_first_deep" in ran or "k_hash_first_lazy" in ran
    assert deep == (case != "shallow30"), sorted(ran)
    b, o = oracle.strings_np(s)
    ref, r_ref, coll = oracle.dist_prefix(b, o, init, bits)
    np.testing.assert_array_equal(u32(d), ref)
    assert rounds == r_ref


# ---------------------------------------------------------- partition / coding

def _partition(s, r, pdms):
    g = s.to(DEV)
    perm, lcp = ss.sort(g.bytes, g.offsets)
    dist = ss.dist_prefix(g.bytes, g.offsets, 8, 64)[0] if pdms else None
    ids = ss.select_splitters(perm, r)
    sb, so = ss.gather_strings(g.bytes, g.offsets, ids)
    fc = ss.partition_encode(g.bytes, g.offsets, perm, lcp, dist, sb, so)
    torch.cuda.synchronize()
    return g, perm, lcp, dist, ids, sb, so, fc


@pytest.mark.parametrize("pdms", [False, True])
@pytest.mark.parametrize("r", [1, 2, 16, 300])
def test_partition_encode_matches_oracle(pdms, r):
    _check_partition(synth.text_strings(30_000, seed=5, median=20), r, pdms)


@pytest.mark.parametrize("pdms", [False, True])
def test_partition_encode_long_literals(pdms):
    """300-byte strings: whole-string literals overflow the staging buffer of
    the literal copy (direct writes); PDMS literals stay short (staged)."""
    _check_partition(synth.dn_strings(20_000, 300, 0.3, seed=8), 5, pdms)


@pytest.mark.parametrize("median", [30, 90])
def test_partition_encode_medium_literals(median):
    """Whole text strings of median 30 and 90 bytes as literals: workgroups
    past the staging buffer copy them 4 or 8 lanes per string."""
    _check_partition(synth.text_strings(20_000, seed=11 + median, median=median), 4, False)


@pytest.mark.parametrize("long_literals", [False, True])
@pytest.mark.parametrize("base", [7, 4096 + 9])
def test_partition_encode_unaligned_suf_base(base, long_literals):
    """Literals written at an odd offset of a shared buffer: bytes outside
    [base, base + total) stay untouched and suf_off is absolute (short
    literals staged in LDS; whole 300-byte strings copied word by word)."""
    s = synth.dn_strings(8_000, 300, 0.3, seed=10) if long_literals else synth.text_strings(20_000, seed=9, median=24)
    _log(f"[partition] suf_base={base} long={long_literals}")
    g, perm, lcp, dist, ids, sb, so, fc = _partition(s, 4, not long_literals)
    t = fc["total"]
    cap = base + t + 64
    out = dict(run_off=torch.empty_like(fc["run_off"]), lcp=torch.empty_like(fc["lcp"]),
               len=torch.empty_like(fc["len"]), id=torch.empty_like(fc["id"]),
               suf_off=torch.empty_like(fc["suf_off"]),
               suf=torch.full((cap,), 0xEE, dtype=torch.uint8, device=DEV))
    fc2 = ss.partition_encode(g.bytes, g.offsets, perm, lcp, dist, sb, so, out=out, suf_base=base)
    torch.cuda.synchronize()
    buf = fc2["suf"].cpu().numpy()
    assert bytes(buf[base:base + t]) == bytes(fc["suf"].cpu().numpy())
    assert (buf[:base] == 0xEE).all() and (buf[base + t:] == 0xEE).all()
    np.testing.assert_array_equal(u64(fc2["suf_off"]).astype(np.int64) - base, u64(fc["suf_off"]).astype(np.int64))


@pytest.mark.parametrize("r", [1, 2, 3, 17, 300])
def test_select_splitters_batch_matches_per_set(r):
    """One launch samples every set: same ids as regular sampling of each set
    on its own (ragged set sizes, sets smaller than r included)."""
    rng = np.random.default_rng(r)
    sizes = np.concatenate([[1, 2, 5, 16, 17], rng.integers(1, 5000, 40), [70_001]])
    set_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(set_off[-1])
    perm = rng.integers(0, 2**32 - 1, n, dtype=np.uint32)
    _log(f"[select_batch] r={r} sets={len(sizes)} n={n}")
    ids = ss.select_splitters_batch(torch.from_numpy(perm.view(np.int32)).to(DEV),
                                    torch.from_numpy(set_off).to(DEV), r)
    ref = [oracle.select_splitters(int(b - a), perm[a:b], r) for a, b in zip(set_off[:-1], set_off[1:])]
    ref = np.concatenate(ref) if r > 1 else np.zeros(0, np.uint32)
    np.testing.assert_array_equal(u32(ids), ref)


def test_select_splitters_batch_rejects_empty_and_malformed_sets():
    perm = torch.arange(6, dtype=torch.int32, device=DEV)
    for bad in ([0, 0, 6], [0, 3, 3, 6], [0, 4, 2, 6], [0, 3, 5], [1, 3, 6], [0, 3, 7]):
        with pytest.raises(ss.StrsortError):
            ss.select_splitters_batch(perm, torch.tensor(bad, device=DEV), 4)
    ok = ss.select_splitters_batch(perm, torch.tensor([0, 2, 6], device=DEV), 2)
    assert list(u32(ok)) == [0, 3]


@pytest.mark.parametrize("hint", [None, 0, 1, 37])
def test_gather_strings_capacity_hint(hint):
    """The byte buffer is regrown once when the hint is too small."""
    s = synth.text_strings(5000, seed=14, median=30)
    g = s.to(DEV)
    ids = torch.tensor([4999, 0, 17, 17, 2500, 3], dtype=torch.int32, device=DEV)
    gb, go = ss.gather_strings(g.bytes, g.offsets, ids, cap_hint=hint)
    strs = s.as_list()
    want = [strs[i] for i in ids.tolist()]
    assert bytes(gb.cpu().numpy()) == b"".join(want)
    np.testing.assert_array_equal(go.cpu().numpy(), np.cumsum([0] + [len(x) for x in want]))


@pytest.mark.parametrize("r", [2, 17])
def test_select_splitters_batch_unchecked(r):
    """Without the check nothing is read back and well-formed sets give the
    checked call's samples; a bad set's samples are 0xFFFFFFFF."""
    rng = np.random.default_rng(40 + r)
    sizes = rng.integers(1, 3000, 25)
    set_off = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)).to(DEV)
    perm = torch.from_numpy(rng.integers(0, 2**31 - 1, int(sizes.sum()), dtype=np.int64).astype(np.int32)).to(DEV)
    a = ss.select_splitters_batch(perm, set_off, r)
    b = ss.select_splitters_batch(perm, set_off, r, check=False)
    assert torch.equal(a, b)
    p6 = torch.arange(6, dtype=torch.int32, device=DEV)
    bad = ss.select_splitters_batch(p6, torch.tensor([0, 3, 3, 6], device=DEV), 2, check=False)
    assert list(u32(bad)) == [1, 0xFFFFFFFF, 4]


@pytest.mark.parametrize("cap", [10**6, 120, 0])
def test_gather_strings_without_read_back(cap):
    """sync=False: offsets are complete on the device; strings that would end
    past the capacity are not copied, the others are; an id past the last
    string is an empty string."""
    s = synth.text_strings(5000, seed=15, median=30)
    g = s.to(DEV)
    ids = torch.tensor([4999, 0, 17, 17, -1, 2500, 3], dtype=torch.int32, device=DEV)  # -1 = 0xFFFFFFFF
    gb, go = ss.gather_strings(g.bytes, g.offsets, ids, cap_hint=cap, sync=False)
    torch.cuda.synchronize()
    strs = s.as_list()
    want = [strs[i] if i >= 0 else b"" for i in ids.tolist()]
    offs = np.cumsum([0] + [len(x) for x in want])
    np.testing.assert_array_equal(go.cpu().numpy(), offs)
    buf = bytes(gb.cpu().numpy())
    for k, w in enumerate(want):
        if offs[k + 1] <= cap:
            assert buf[offs[k]:offs[k + 1]] == w


@pytest.mark.parametrize("short_by", [1, 5000])
def test_partition_encode_capacity(short_by):
    """A literal buffer shorter than the literals: CAPACITY, no literal byte
    written, and the metadata and offsets complete."""
    s = synth.text_strings(20_000, seed=10, median=24)
    _log(f"[partition] capacity short by {short_by}")
    g, perm, lcp, dist, ids, sb, so, fc = _partition(s, 4, True)
    t = fc["total"]
    cap = t - short_by
    n = s.n
    out = dict(run_off=torch.empty_like(fc["run_off"]), lcp=torch.empty_like(fc["lcp"]),
               len=torch.empty_like(fc["len"]), id=torch.empty_like(fc["id"]),
               suf_off=torch.empty_like(fc["suf_off"]),
               suf=torch.full((t + 256,), 0xEE, dtype=torch.uint8, device=DEV))
    ws = torch.empty(ss.lib().ss_partition_encode_workspace(n), dtype=torch.uint8, device=DEV)
    rc = ss.lib().ss_partition_encode(ss._p(g.bytes), g.bytes.numel(), ss._p(g.offsets), n, ss._p(perm),
                                      ss._p(lcp), ss._p(dist), ss._p(sb), sb.numel(), ss._p(so), so.numel(),
                                      ss._p(out["run_off"]), ss._p(out["lcp"]), ss._p(out["len"]), ss._p(out["id"]),
                                      ss._p(out["suf_off"]), ss._p(out["suf"]), 0, cap, None, ss._p(ws), ws.numel(),
                                      ss._stream(g.bytes.device))
    torch.cuda.synchronize()
    assert rc == ss.SS_ERR_CAPACITY
    for k in ("run_off", "lcp", "len", "id", "suf_off"):
        np.testing.assert_array_equal(out[k].cpu().numpy(), fc[k].cpu().numpy())
    assert (out["suf"].cpu().numpy() == 0xEE).all()


def _check_partition(s, r, pdms):
    _log(f"[partition] n={s.n} r={r} pdms={pdms}")
    g, perm, lcp, dist, ids, sb, so, fc = _partition(s, r, pdms)
    b, o = oracle.strings_np(s)
    p_ref = oracle.sort(b, o)
    l_ref = oracle.lcp(b, o, p_ref)
    d_ref = oracle.dist_prefix(b, o, 8, 64)[0] if pdms else None
    np.testing.assert_array_equal(u32(ids), oracle.select_splitters(s.n, p_ref, r))
    strs = s.as_list()
    spl = synth.from_list([strs[i] for i in oracle.select_splitters(s.n, p_ref, r)])
    assert bytes(sb.cpu().numpy()) == bytes(spl.bytes.numpy())
    sbn, son = oracle.strings_np(spl)
    bounds = oracle.bucket_bounds(b, o, p_ref, sbn, son)
    np.testing.assert_array_equal(u64(fc["run_off"]), bounds)
    ref = oracle.fc_encode(b, o, p_ref, l_ref, d_ref, bounds)
    np.testing.assert_array_equal(u32(fc["lcp"]), ref["lcp"])
    np.testing.assert_array_equal(u32(fc["len"]), ref["len"])
    np.testing.assert_array_equal(u32(fc["id"]), ref["id"])
    np.testing.assert_array_equal(u64(fc["suf_off"]), ref["suf_off"])
    assert bytes(fc["suf"].cpu().numpy()) == bytes(ref["suf"])
    # decode on the GPU == oracle decode
    db, doff = ss.fc_decode(fc["run_off"], fc["lcp"], fc["len"], fc["suf_off"], fc["suf"])
    rb, roff = oracle.fc_decode(bounds, ref["lcp"], ref["len"], ref["suf_off"], ref["suf"])
    np.testing.assert_array_equal(u64(doff), roff)
    assert bytes(db.cpu().numpy()) == bytes(rb)


def _fc_patterns(n, runs, seed):
    """Valid front-coded arrays (e_0 = 0 per run, e_i <= d_i, e_i <= d_(i-1)) whose
    LCP sequence has far previous-smaller values: long plateaus broken by rare
    dips, staircases, sawtooths and random stretches."""
    rng = np.random.default_rng(seed)
    d = rng.integers(20, 90, size=n).astype(np.int64)
    e = np.empty(n, np.int64)
    q = n // 4
    e[:q] = 18
    if q:
        e[:q][rng.integers(0, q, size=3)] = 1                 # plateau, dips ~100k apart
    e[q:2 * q] = np.arange(q) % 85                             # staircase
    e[2 * q:3 * q] = 80 - (np.arange(q) % 79)                  # sawtooth down
    e[3 * q:] = rng.integers(0, 60, size=n - 3 * q)            # random
    prev = np.concatenate([[0], d[:-1]])
    e = np.minimum(np.minimum(e, d), prev)
    run_off = np.linspace(0, n, runs + 1).astype(np.uint64)
    e[run_off[:-1].astype(np.int64)] = 0
    lit = d - e
    suf_off = np.concatenate([[0], np.cumsum(lit)]).astype(np.uint64)
    suf = rng.integers(65, 91, size=int(suf_off[-1])).astype(np.uint8)
    return run_off, e.astype(np.uint32), d.astype(np.uint32), suf_off, suf


@pytest.mark.parametrize("n,runs", [(1, 1), (255, 1), (257, 2), (400_000, 3)])
def test_fc_decode_far_previous_smaller(n, runs):
    run_off, e, d, suf_off, suf = _fc_patterns(n, runs, seed=n)
    _log(f"[decode] n={n} runs={runs}")
    T = lambda a, dt: torch.from_numpy(a.view(dt).copy()).to(DEV)
    db, doff = ss.fc_decode(T(run_off, np.int64), T(e, np.int32), T(d, np.int32), T(suf_off, np.int64),
                            torch.from_numpy(suf.copy()).to(DEV))
    torch.cuda.synchronize()
    rb, roff = oracle.fc_decode(run_off, e, d, suf_off, suf)
    np.testing.assert_array_equal(u64(doff), roff)
    assert bytes(db.cpu().numpy()) == bytes(rb)


def test_bucket_bounds_with_external_splitters():
    s = synth.text_strings(20_000, seed=6, median=8)
    strs = s.as_list()
    rng = random.Random(6)
    spl = sorted(rng.sample(strs, 40) + [b"", b"\xff\xff", strs[0], strs[0]])
    g = s.to(DEV)
    perm, _ = ss.sort(g.bytes, g.offsets)
    sp = synth.from_list(spl).to(DEV)
    got = ss.bucket_bounds(g.bytes, g.offsets, perm, sp.bytes, sp.offsets)
    b, o = oracle.strings_np(s)
    sbn, son = oracle.strings_np(synth.from_list(spl))
    np.testing.assert_array_equal(u64(got), oracle.bucket_bounds(b, o, oracle.sort(b, o), sbn, son))


# ----------------------------------------------------------------------- merge

def _runs_from_oracle(s, k, seed, pdms=False, assign=None):
    """k sorted front-coded runs built by the oracle from a random split
    (or the given run of every string)."""
    rng = np.random.default_rng(seed)
    b, o = oracle.strings_np(s)
    strs = s.as_list()
    if assign is None:
        assign = rng.integers(0, k, size=s.n)
    parts = []
    for j in range(k):
        idx = np.nonzero(assign == j)[0]
        sub = synth.from_list([strs[i] for i in idx])
        sb, so = oracle.strings_np(sub)
        p = oracle.sort(sb, so)
        lc = oracle.lcp(sb, so, p)
        d = oracle.dist_prefix(sb, so, 8, 64)[0] if pdms else None
        enc = oracle.fc_encode(sb, so, p, lc, d, np.array([0, sub.n], np.uint64))
        enc["id"] = idx[enc["id"]].astype(np.uint32)
        parts.append(enc)
    run_off = np.zeros(k + 1, np.uint64)
    for j, e in enumerate(parts):
        run_off[j + 1] = run_off[j] + len(e["lcp"])
    lcp_ = np.concatenate([e["lcp"] for e in parts])
    len_ = np.concatenate([e["len"] for e in parts])
    id_ = np.concatenate([e["id"] for e in parts])
    suf = np.concatenate([e["suf"] for e in parts]) if parts else np.zeros(0, np.uint8)
    suf_off = np.zeros(s.n + 1, np.uint64)
    base, pos = 0, 0
    for e in parts:
        m = len(e["lcp"])
        suf_off[pos:pos + m] = e["suf_off"][:m] + base
        base += int(e["suf_off"][m])
        pos += m
    suf_off[s.n] = base
    return run_off, lcp_, len_, id_, suf_off, suf


@pytest.mark.parametrize("k,seed,pdms", [(1, 0, False), (2, 1, False), (7, 2, False), (64, 3, False),
                                         (16, 4, True)])
def test_lcp_merge_matches_oracle(k, seed, pdms):
    s = synth.text_strings(12_000, seed=20 + seed, median=10)
    _log(f"[merge] k={k}")
    ro, lc, ln, idv, so, suf = _runs_from_oracle(s, k, seed, pdms)
    T = lambda a, dt: torch.from_numpy(a.view(dt).copy()).to(DEV)
    src, gid, glcp = ss.lcp_merge_runs(T(ro, np.int64), T(lc, np.int32), T(ln, np.int32), T(idv, np.int32),
                                  T(so, np.int64), torch.from_numpy(suf.copy()).to(DEV))
    torch.cuda.synchronize()
    rsrc, rid, rlcp = oracle.merge(ro, lc, ln, idv, so, suf)
    np.testing.assert_array_equal(u64(src), rsrc)
    np.testing.assert_array_equal(u32(gid), rid)
    np.testing.assert_array_equal(u32(glcp), rlcp)


def test_lcp_merge_ties_across_runs_only():
    """Inside each run no two neighbours share 7 bytes, but strings of
    different runs share 20 or more (and some are equal): every such pair is
    compared past the cached keys, from the strings' own literals."""
    rng = np.random.default_rng(12)
    k = 6
    strs, assign = [], []
    for j in range(k):
        for i in range(200):
            head = bytes([33 + i % 90, 33 + i // 90])
            tail = b"" if i % 7 == 0 else bytes(rng.integers(65, 70, size=int(rng.integers(0, 6))).tolist())
            strs.append(head + b"Z" * 20 + (b"%d" % (j % 3)) + tail)
            assign.append(j)
    s = synth.from_list(strs)
    ro, lc, ln, idv, so, suf = _runs_from_oracle(s, k, 0, assign=np.array(assign))
    assert all(int(x) < 7 for x in lc)  # no neighbours in a run share 7 bytes
    T = lambda a, dt: torch.from_numpy(a.view(dt).copy()).to(DEV)
    src, gid, glcp = ss.lcp_merge_runs(T(ro, np.int64), T(lc, np.int32), T(ln, np.int32), T(idv, np.int32),
                                       T(so, np.int64), torch.from_numpy(suf.copy()).to(DEV))
    torch.cuda.synchronize()
    rsrc, rid, rlcp = oracle.merge(ro, lc, ln, idv, so, suf)
    np.testing.assert_array_equal(u64(src), rsrc)
    np.testing.assert_array_equal(u32(gid), rid)
    np.testing.assert_array_equal(u32(glcp), rlcp)
    assert int(rlcp.max()) >= 22


def test_lcp_merge_dn_closed_form():
    """C3b shape scaled down: DN strings of 64 B with D/N 0.3 in 32 runs."""
    n = 40_000
    s = synth.dn_strings(n, 64, 0.3, seed=7)
    ro, lc, ln, idv, so, suf = _runs_from_oracle(s, 32, 7)
    T = lambda a, dt: torch.from_numpy(a.view(dt).copy()).to(DEV)
    _, gid, glcp = ss.lcp_merge_runs(T(ro, np.int64), T(lc, np.int32), T(ln, np.int32), T(idv, np.int32),
                                T(so, np.int64), torch.from_numpy(suf.copy()).to(DEV))
    pi = s.meta["pi"].numpy()
    np.testing.assert_array_equal(u32(gid), cf.dn_perm(pi))
    np.testing.assert_array_equal(u32(glcp), cf.dn_lcp(n, s.meta["k"], s.meta["filler"]))


def test_lcp_merge_groups_runs_in_place():
    """Several groups merged in one call; runs scattered in shuffled order inside
    shared front-coded arrays (as the buckets each processing element receives)."""
    rng = np.random.default_rng(11)
    groups = []
    for gi, (n, k) in enumerate([(3000, 4), (1, 1), (5000, 9), (0, 2), (2000, 3)]):
        s = synth.text_strings(max(n, 1), seed=40 + gi, median=9) if n else synth.from_list([])
        if n == 1:
            s = synth.from_list([b"only"])
        groups.append((s, k) if n else (synth.from_list([]), k))
    # encode every group's runs with the oracle
    blocks = []   # (group, run-in-group, dict)
    for gi, (s, k) in enumerate(groups):
        ro, lc, ln, idv, so, suf = _runs_from_oracle(s, k, 100 + gi) if s.n else (
            np.zeros(k + 1, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint32),
            np.zeros(1, np.uint64), np.zeros(0, np.uint8))
        for j in range(k):
            a, b = int(ro[j]), int(ro[j + 1])
            blocks.append((gi, j, dict(lcp=lc[a:b], len=ln[a:b], id=idv[a:b],
                                       suf=suf[int(so[a]):int(so[b])] if b > a else np.zeros(0, np.uint8),
                                       so=(so[a:b] - so[a]) if b > a else np.zeros(0, np.uint64))))
    order = rng.permutation(len(blocks))
    FL, FD, FI, FS, SUF = [], [], [], [], []
    pos, sbase, where = 0, 0, {}
    for bi in order:
        gi, j, d = blocks[bi]
        m = len(d["lcp"])
        where[(gi, j)] = (pos, pos + m)
        FL.append(d["lcp"]); FD.append(d["len"]); FI.append(d["id"]); FS.append(d["so"] + sbase)
        SUF.append(d["suf"]); sbase += len(d["suf"]); pos += m
    fl = np.concatenate(FL); fd = np.concatenate(FD); fi = np.concatenate(FI)
    so_all = np.concatenate(FS + [np.array([sbase], np.uint64)]); suf_all = np.concatenate(SUF)
    rb, re_, gofs = [], [], [0]
    for gi, (s, k) in enumerate(groups):
        for j in range(k):
            a, b = where[(gi, j)]
            rb.append(a); re_.append(b)
        gofs.append(len(rb))
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt).copy()).to(DEV)
    src, gid, glcp = ss.lcp_merge(torch.tensor(rb, dtype=torch.int64), torch.tensor(re_, dtype=torch.int64),
                                  torch.tensor(gofs, dtype=torch.int32), T(fl, np.int32), T(fd, np.int32),
                                  T(fi, np.int32), T(so_all, np.int64), torch.from_numpy(suf_all.copy()).to(DEV))
    torch.cuda.synchronize()
    S, I, L = u64(src), u32(gid), u32(glcp)
    out = 0
    for gi, (s, k) in enumerate(groups):
        # oracle: merge this group's runs laid out contiguously
        ro = [0]; lcs, lns, ids, sos, sufs = [], [], [], [], []
        base = 0
        for j in range(k):
            a, b = where[(gi, j)]
            lcs.append(fl[a:b]); lns.append(fd[a:b]); ids.append(fi[a:b])
            if b > a:
                seg = suf_all[int(so_all[a]):int(so_all[b])]
                sos.append(so_all[a:b] - so_all[a] + base); sufs.append(seg); base += len(seg)
            ro.append(ro[-1] + (b - a))
        m = ro[-1]
        if m == 0:
            continue
        rsrc, rid, rlcp = oracle.merge(np.array(ro, np.uint64), np.concatenate(lcs), np.concatenate(lns),
                                       np.concatenate(ids), np.concatenate(sos + [np.array([base], np.uint64)]),
                                       np.concatenate(sufs) if sufs else np.zeros(0, np.uint8))
        run_base = gofs[gi]
        exp_src = ((rsrc >> np.uint64(32)) + np.uint64(run_base)) << np.uint64(32) | (rsrc & np.uint64(0xFFFFFFFF))
        np.testing.assert_array_equal(S[out:out + m], exp_src)
        np.testing.assert_array_equal(I[out:out + m], rid)
        np.testing.assert_array_equal(L[out:out + m], rlcp)
        out += m
    assert out == len(S)


@pytest.mark.parametrize("pdms", [False, True])
def test_partition_encode_batch_matches_oracle_per_set(pdms):
    """Each processing element's sorted array split with common splitters, all in one call."""
    sets, bounds = synth.random_sets(7, 50, 4000, len_lo=1, len_hi=30, seed=8)
    g = sets.to(DEV)
    perm_l, lcp = ss.sort_batch(g.bytes, g.offsets, bounds.to(DEV))
    base = torch.repeat_interleave(bounds[:-1], bounds[1:] - bounds[:-1]).to(DEV).to(torch.int32)
    perm = perm_l + base
    dist = ss.dist_prefix(g.bytes, g.offsets, 8, 64)[0] if pdms else None
    strs = sets.as_list()
    spl = sorted(random.Random(3).sample(strs, 11))
    sp = synth.from_list(spl).to(DEV)
    fc = ss.partition_encode_batch(g.bytes, g.offsets, bounds.to(DEV), perm, lcp, dist, sp.bytes, sp.offsets)
    torch.cuda.synchronize()
    b, o = oracle.strings_np(sets)
    sbn, son = oracle.strings_np(synth.from_list(spl))
    d_ref = oracle.dist_prefix(b, o, 8, 64)[0] if pdms else None
    r = len(spl) + 1
    RO = u64(fc["run_off"]).reshape(len(bounds) - 1, r + 1)
    FL, FD, FI, SO = u32(fc["lcp"]), u32(fc["len"]), u32(fc["id"]), u64(fc["suf_off"])
    SUF = fc["suf"][:fc["total"]].cpu().numpy()
    for j in range(len(bounds) - 1):
        a, e = int(bounds[j]), int(bounds[j + 1])
        sub_o = (o[a:e + 1] - o[a]).astype(np.uint64)
        sub_b = b[int(o[a]):int(o[e])]
        pr = oracle.sort(sub_b, sub_o)
        prg = (pr + a).astype(np.uint32)
        lr = oracle.lcp(sub_b, sub_o, pr)
        bb = oracle.bucket_bounds(b, o, prg, sbn, son)
        np.testing.assert_array_equal(RO[j], bb + np.uint64(a))
        ref = oracle.fc_encode(b, o, prg, lr, d_ref, bb)
        np.testing.assert_array_equal(FL[a:e], ref["lcp"])
        np.testing.assert_array_equal(FD[a:e], ref["len"])
        np.testing.assert_array_equal(FI[a:e], ref["id"])
        np.testing.assert_array_equal(SO[a:e] - SO[a], ref["suf_off"][:e - a])
        assert bytes(SUF[int(SO[a]):int(SO[e])]) == bytes(ref["suf"])


def _pipeline(sets, bounds, spl, pdms):
    """The one-device form of the distributed sort: per-set sorts, common
    splitters, bucket partition + front coding, one merge per bucket, LCPs
    joined across buckets, exact distinguishing prefixes."""
    g = sets.to(DEV)
    so = bounds.to(DEV)
    p = len(bounds) - 1
    perm, lcp = ss.sort_batch(g.bytes, g.offsets, so, global_ids=True)
    dist = ss.dist_prefix(g.bytes, g.offsets, 8, 64)[0] if pdms else None
    sp = synth.from_list(spl).to(DEV)
    fc = ss.partition_encode_batch(g.bytes, g.offsets, so, perm, lcp, dist, sp.bytes, sp.offsets)
    r = len(spl) + 1
    ro = fc["run_off"].view(p, r + 1)
    run_begin = ro[:, :-1].t().reshape(-1)      # group j = bucket j, run i = set i
    run_end = ro[:, 1:].t().reshape(-1)
    group_off = torch.arange(0, p * r + 1, p, dtype=torch.int32, device=DEV)
    src, order, mlcp, mlen = ss.lcp_merge(run_begin, run_end, group_off, fc["lcp"], fc["len"], fc["id"],
                                          fc["suf_off"], fc["suf"], n_out=sets.n, with_len=True)
    # out_len is the fc_len entry of each merged element
    rb = run_begin.cpu().numpy()
    S = u64(src)
    pos = rb[(S >> np.uint64(32)).astype(np.int64)] + (S & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.testing.assert_array_equal(u32(mlen), u32(fc["len"])[pos])
    ss.join_group_lcps(g.bytes, g.offsets, order, mlcp, run_begin, run_end, group_off)
    dist_x = ss.dist_exact(g.offsets, order, mlcp)
    dist_b = ss.dist_exact_bounded(order, mlcp, mlen)
    dist_s = ss.dist_exact_bounded(None, mlcp, mlen)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(dist_b), u32(dist_x))
    np.testing.assert_array_equal(u32(dist_s), u32(dist_x)[u32(order)])
    return order, mlcp, dist_x


@pytest.mark.parametrize("pdms", [False, True])
@pytest.mark.parametrize("spl_kind", ["sampled", "empty_buckets"])
def test_pipeline_join_group_lcps(pdms, spl_kind):
    """Whole order, its LCP array (joined at every bucket boundary) and the
    exact distinguishing prefixes against the oracle on all strings."""
    sets, bounds = synth.random_sets(6, 20, 3000, len_lo=0, len_hi=40, seed=12)
    strs = sets.as_list()
    if spl_kind == "sampled":
        spl = sorted(random.Random(5).sample(strs, 9))
    else:  # repeated and extreme splitters leave buckets empty
        mid = sorted(strs)[len(strs) // 2]
        spl = sorted([b"", b"", mid, mid, mid, b"\xff" * 3, b"\xff" * 3])
    _log(f"[pipeline] n={sets.n} pdms={pdms} splitters={spl_kind}")
    order, mlcp, dist_x = _pipeline(sets, bounds, spl, pdms)
    b, o = oracle.strings_np(sets)
    p_ref = oracle.sort(b, o)
    l_ref = oracle.lcp(b, o, p_ref)
    np.testing.assert_array_equal(u32(order), p_ref)
    np.testing.assert_array_equal(u32(mlcp), l_ref)
    np.testing.assert_array_equal(u32(dist_x), oracle.dist_exact(o, p_ref, l_ref))


def test_join_group_lcps_leaves_other_positions():
    """Only the first position of each non-empty group after the first changes."""
    s = synth.from_list([b"AAA", b"AAB", b"AB", b"B", b"BA", b"BAA"])
    g = s.to(DEV)
    order = torch.arange(6, dtype=torch.int32, device=DEV)
    lcp = torch.full((6,), 77, dtype=torch.int32, device=DEV)
    rb = torch.tensor([0, 2, 2, 3], dtype=torch.int64, device=DEV)   # runs: [0,2) [2,2) [2,3) [3,6)
    re_ = torch.tensor([2, 2, 3, 6], dtype=torch.int64, device=DEV)
    go = torch.tensor([0, 1, 2, 3, 4], dtype=torch.int32, device=DEV)  # group 1 is empty
    ss.join_group_lcps(g.bytes, g.offsets, order, lcp, rb, re_, go)
    assert list(u32(lcp)) == [77, 77, 1, 0, 77, 77]


@pytest.mark.parametrize("case", ["c0", "text", "deep_mixed", "init64"])
def test_dist_prefix_in_two_calls_equals_one(case):
    """ss_dist_prefix_first then ss_dist_prefix_rounds (same workspace, the
    rounds on another stream ordered after the first) = ss_dist_prefix."""
    if case == "c0":
        s, l0 = synth.dn_strings(100_000, 100, 0.5, seed=0), 8
    elif case == "text":
        s, l0 = synth.text_strings(200_000, seed=5), 8
    elif case == "deep_mixed":
        s, l0 = _deep_mixed(3), 8
    else:
        s, l0 = synth.text_strings(50_000, seed=6, median=90), 128
    g = s.to(DEV)
    ref, r_ref = ss.dist_prefix(g.bytes, g.offsets, l0, 64)
    ws = ss.dist_prefix_first(g.bytes, g.offsets, l0, 64)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got, rounds = ss.dist_prefix_rounds(g.bytes, g.offsets, ws, l0, 64)
    torch.cuda.synchronize()
    assert rounds == r_ref and torch.equal(got, ref)


def test_dist_prefix_rounds_without_a_first_pass_is_refused():
    s = synth.text_strings(1000, seed=1).to(DEV)
    ws = torch.zeros(ss.lib().ss_dist_prefix_workspace(s.n), dtype=torch.uint8, device=DEV)
    with pytest.raises(ss.StrsortError):
        ss.dist_prefix_rounds(s.bytes, s.offsets, ws, 8, 64)
