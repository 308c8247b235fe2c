"""Pins of the CPU oracle against facts that do not come from the oracle.

Sources of truth used here: Python's own bytes ordering (an independent
implementation of the lexicographic order with the shorter-prefix-first rule),
exhaustive enumeration of permutations, brute force over all pairs, closed
forms of the D/N workload (integer arithmetic on the generator's permutation),
and algebraic identities of the polynomial hash.
"""
import itertools
import os
import random

import numpy as np
import pytest

import oracle
import synth
from tests import closed_forms as cf


def _arrays(strings):
    s = synth.from_list(strings)
    return oracle.strings_np(s)


def _rand_strings(rng, n, alphabet=(0, 65, 66, 255), max_len=5):
    return [bytes(rng.choice(alphabet) for _ in range(rng.randint(0, max_len))) for _ in range(n)]


def _py_lcp(a: bytes, b: bytes) -> int:
    return len(os.path.commonprefix([a, b]))


# ------------------------------------------------------------------ sorting

@pytest.mark.parametrize("seed", range(12))
def test_sort_unique_sorted_permutation_by_enumeration(seed):
    """Among all n! orders exactly one is sorted with index ties; the oracle returns it."""
    rng = random.Random(seed)
    n = rng.randint(1, 6)
    strs = _rand_strings(rng, n)
    if seed % 3 == 0 and n > 1:
        strs[1] = strs[0]  # force an exact duplicate
    b, o = _arrays(strs)
    sorted_ones = []
    for p in itertools.permutations(range(n)):
        if all((strs[p[i - 1]], p[i - 1]) < (strs[p[i]], p[i]) for i in range(1, n)):
            sorted_ones.append(p)
    assert len(sorted_ones) == 1
    assert list(oracle.sort(b, o)) == list(sorted_ones[0])


@pytest.mark.parametrize("seed", range(5))
def test_sort_matches_python_sorted(seed):
    rng = random.Random(100 + seed)
    strs = _rand_strings(rng, 300, alphabet=(0, 1, 65, 66, 67, 254, 255), max_len=12)
    strs += [b"", b"", b"\x00", b"\x00\x00", b"A", b"AA", b"AAA"]
    rng.shuffle(strs)
    b, o = _arrays(strs)
    expect = sorted(range(len(strs)), key=lambda i: (strs[i], i))
    perm = oracle.sort(b, o)
    assert list(perm) == expect
    lcp = oracle.lcp(b, o, perm)
    assert lcp[0] == 0
    assert all(lcp[i] == _py_lcp(strs[perm[i - 1]], strs[perm[i]]) for i in range(1, len(strs)))
    assert oracle.check_sorted(b, o, perm, lcp) == -1


def test_prefix_and_zero_byte_order():
    strs = [b"AB\x00", b"AB", b"A", b"", b"AB\x00\x00", b"\x00", b"AB\x01"]
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    assert [strs[i] for i in perm] == [b"", b"\x00", b"A", b"AB", b"AB\x00", b"AB\x00\x00", b"AB\x01"]


def test_check_sorted_rejects_wrong_answers():
    strs = [b"B", b"A", b"A", b"C"]
    b, o = _arrays(strs)
    good = oracle.sort(b, o)
    assert list(good) == [1, 2, 0, 3]
    assert oracle.check_sorted(b, o, good) == -1
    assert oracle.check_sorted(b, o, np.array([2, 1, 0, 3], np.uint32)) == 1  # unstable tie
    assert oracle.check_sorted(b, o, np.array([1, 1, 0, 3], np.uint32)) == -2  # not a permutation
    lcp = oracle.lcp(b, o, good)
    bad = lcp.copy(); bad[2] += 1
    assert oracle.check_sorted(b, o, good, bad) == 2


# ------------------------------------------------------ D/N closed forms

@pytest.mark.parametrize("n,length,ratio", [(1, 10, 0.5), (2, 10, 0.5), (27, 12, 0.5), (700, 40, 0.3),
                                            (100_000, 100, 0.5)])
def test_dn_closed_form_sort_lcp_dist(n, length, ratio):
    s = synth.dn_strings(n, length, ratio, seed=0)
    b, o = oracle.strings_np(s)
    k, F = s.meta["k"], s.meta["filler"]
    pi = s.meta["pi"].numpy()
    perm = oracle.sort(b, o)
    np.testing.assert_array_equal(perm, cf.dn_perm(pi))
    lcp = oracle.lcp(b, o, perm)
    np.testing.assert_array_equal(lcp, cf.dn_lcp(n, k, F))
    dist = oracle.dist_exact(o, perm, lcp)
    np.testing.assert_array_equal(dist[perm], cf.dn_dist_sorted(n, k, F, length))


def test_dn_c0_dist_prefix_closed_form():
    """C0 shape: 100k x 100 B, D/N 0.5 -> filler 46, k 4; prefix doubling from 8 bytes."""
    n, length = 100_000, 100
    s = synth.dn_strings(n, length, 0.5, seed=0)
    b, o = oracle.strings_np(s)
    k, F = s.meta["k"], s.meta["filler"]
    assert (k, F) == (4, 46)
    pi = s.meta["pi"].numpy()
    dist_sorted = cf.dn_dist_sorted(n, k, F, length)
    dist = np.empty(n, np.uint32)
    dist[cf.dn_perm(pi)] = dist_sorted
    approx, rounds, coll = oracle.dist_prefix(b, o, 8, 64)
    assert coll == 0
    np.testing.assert_array_equal(approx, cf.doubling_closed_form(dist, np.full(n, length), 8))
    assert set(np.unique(approx)) == {64}
    assert rounds == 4  # l = 8, 16, 32, 64


# ------------------------------------------------------- distinguishing prefix

@pytest.mark.parametrize("seed", range(8))
def test_dist_exact_equals_bruteforce(seed):
    rng = random.Random(200 + seed)
    strs = _rand_strings(rng, rng.randint(1, 40), alphabet=(0, 65, 66), max_len=6)
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    lcp = oracle.lcp(b, o, perm)
    d = oracle.dist_exact(o, perm, lcp)
    # brute force in Python over all pairs (independent of the oracle's C)
    n = len(strs)
    for i in range(n):
        best = max((_py_lcp(strs[i], strs[j]) for j in range(n) if j != i), default=0)
        assert d[i] == min(len(strs[i]), best + 1)
    np.testing.assert_array_equal(d, oracle.dist_bruteforce(b, o))


def test_dist_special_cases():
    strs = [b"", b"ABC", b"ABC", b"AB", b"ABD", b"Z"]
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    d = oracle.dist_exact(o, perm, oracle.lcp(b, o, perm))
    # empty -> 0; duplicates saturate at len; a prefix of another saturates; Z needs 1
    assert list(d) == [0, 3, 3, 2, 3, 1]
    one = _arrays([b"HELLO"])
    assert list(oracle.dist_exact(one[1], np.zeros(1, np.uint32), np.zeros(1, np.uint32))) == [1]


# ------------------------------------------------------------ the frozen hash

P = (1 << 61) - 1
B = 0x0B3C4D5E6F708192


def test_kr_zero_prefix_closed_form():
    # all limbs zero -> C = 0 -> key = m
    for m in (0, 1, 3, 4, 5, 8, 64, 1000):
        assert oracle.kr_key(bytes(m)) == m


def test_kr_single_difference_is_one_power_of_B():
    """Changing byte t of limb j by delta changes the key by delta*256^t*B^(q-j) mod p
    (q = number of limbs): pins the base, limb order, in-limb byte order and the
    trailing length digit."""
    rng = random.Random(7)
    for _ in range(200):
        m = rng.randint(1, 70)
        x = bytearray(rng.randrange(256) for _ in range(m))
        pos = rng.randrange(m)
        y = bytearray(x)
        y[pos] = rng.randrange(256)
        q = (m + 3) // 4
        j, t = divmod(pos, 4)
        delta = (y[pos] - x[pos]) * (256 ** t)
        expect = (delta * pow(B, q - j, P)) % P
        assert (oracle.kr_key(bytes(y)) - oracle.kr_key(bytes(x))) % P == expect


def test_kr_length_digit_separates_zero_padding():
    assert oracle.kr_key(b"A") != oracle.kr_key(b"A\x00")
    assert (oracle.kr_key(b"A\x00") - oracle.kr_key(b"A")) % P == 1
    assert oracle.kr_key(b"ABCD", 3) == oracle.kr_key(b"ABC")


def test_kr_golden_vectors():
    """Frozen test vectors (written by tests/golden/make_kr_vectors.py from the oracle)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "kr_vectors.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        hexdata, key = line.split()
        data = bytes.fromhex(hexdata) if hexdata != "-" else b""
        assert oracle.kr_key(data) == int(key, 16)
        n += 1
    assert n >= 20


# ------------------------------------------------------------- prefix doubling

@pytest.mark.parametrize("seed", range(6))
def test_dist_prefix_invariants_text(seed):
    s = synth.text_strings(3000, seed=seed, median=12)
    b, o = oracle.strings_np(s)
    perm = oracle.sort(b, o)
    d = oracle.dist_exact(o, perm, oracle.lcp(b, o, perm))
    lens = (o[1:] - o[:-1]).astype(np.int64)
    approx, rounds, coll = oracle.dist_prefix(b, o, 8, 64)
    assert (approx >= d).all()
    assert (approx <= lens).all()
    if coll == 0:
        np.testing.assert_array_equal(approx, cf.doubling_closed_form(d, lens, 8))
        assert rounds == cf.doubling_rounds_closed_form(d, lens, 8)
        # no collisions: dist_approx <= max(l0, 2 dist - 2) when below len (E[dist_approx] = O(dist))
        bound = np.maximum(8, 2 * d.astype(np.int64) - 2)
        assert (approx.astype(np.int64) <= np.maximum(bound, 0) + (approx == lens) * 10**9).all()
    lmax = int(lens.max())
    import math
    assert rounds <= max(1, math.ceil(math.log2(max(lmax, 8) / 8))) + 1


@pytest.mark.parametrize("bits", [8, 12, 16])
def test_dist_prefix_forced_collisions_only_delay(bits):
    s = synth.text_strings(4000, seed=3, median=10)
    b, o = oracle.strings_np(s)
    perm = oracle.sort(b, o)
    d = oracle.dist_exact(o, perm, oracle.lcp(b, o, perm))
    lens = (o[1:] - o[:-1]).astype(np.int64)
    approx, rounds, coll = oracle.dist_prefix(b, o, 8, bits)
    assert coll > 0
    assert (approx >= d).all()
    assert (approx >= cf.doubling_closed_form(d, lens, 8)).all()
    assert (approx <= lens).all()


def test_dist_prefix_edge_cases():
    strs = [b"", b"A", b"A", b"ABCDEFGH", b"ABCDEFGHI", b"ABCDEFGHI", b"XYZ" * 10]
    b, o = _arrays(strs)
    approx, rounds, coll = oracle.dist_prefix(b, o, 8, 64)
    # empty and short strings end in round 1 at their length; duplicates saturate at len
    assert list(approx) == [0, 1, 1, 8, 9, 9, 8]
    with pytest.raises(ValueError):
        oracle.dist_prefix(b, o, 6, 64)


# --------------------------------------------------------- splitters / buckets

@pytest.mark.parametrize("seed,r", [(0, 2), (1, 7), (2, 64), (3, 300)])
def test_buckets_bruteforce(seed, r):
    rng = random.Random(300 + seed)
    strs = _rand_strings(rng, 250, alphabet=(65, 66, 67), max_len=6)
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    n = len(strs)
    ids = oracle.select_splitters(n, perm, r)
    spl = [strs[i] for i in ids]
    sb, so = _arrays(spl)
    bounds = oracle.bucket_bounds(b, o, perm, sb, so)
    assert bounds[0] == 0 and bounds[-1] == n and len(bounds) == r + 1
    srt = [strs[i] for i in perm]
    for j in range(1, r):
        assert bounds[j] == sum(1 for x in srt if x <= spl[j - 1])
    for j in range(r):
        lo = spl[j - 1] if j > 0 else None
        hi = spl[j] if j < r - 1 else None
        for x in srt[bounds[j]:bounds[j + 1]]:
            assert (lo is None or lo < x) and (hi is None or x <= hi)


# ----------------------------------------------------------------- front coding

@pytest.mark.parametrize("pdms", [False, True])
@pytest.mark.parametrize("seed", range(4))
def test_front_coding_round_trip(seed, pdms):
    s = synth.text_strings(2000, seed=10 + seed, median=14)
    b, o = oracle.strings_np(s)
    strs = s.as_list()
    perm = oracle.sort(b, o)
    lcp = oracle.lcp(b, o, perm)
    dist = oracle.dist_prefix(b, o, 8, 64)[0] if pdms else None
    ids = oracle.select_splitters(len(strs), perm, 16)
    sb, so = _arrays([strs[i] for i in ids])
    bounds = oracle.bucket_bounds(b, o, perm, sb, so)
    fc = oracle.fc_encode(b, o, perm, lcp, dist, bounds)
    dec, doff = oracle.fc_decode(bounds, fc["lcp"], fc["len"], fc["suf_off"], fc["suf"])
    total = 0
    for j in range(16):
        for i in range(int(bounds[j]), int(bounds[j + 1])):
            src = strs[perm[i]]
            d = int(dist[perm[i]]) if pdms else len(src)
            e = 0 if i == bounds[j] else _py_lcp(strs[perm[i - 1]], src)
            assert fc["lcp"][i] == e and fc["len"][i] == d and fc["id"][i] == perm[i]
            assert bytes(dec[doff[i]:doff[i + 1]]) == src[:d]
            total += d - e
    assert total == len(fc["suf"]) == int(fc["suf_off"][-1])


def test_front_coding_truncation_keeps_lcp():
    s = synth.text_strings(3000, seed=21, median=10)
    b, o = oracle.strings_np(s)
    strs = s.as_list()
    perm = oracle.sort(b, o)
    lcp = oracle.lcp(b, o, perm)
    dist = oracle.dist_prefix(b, o, 8, 64)[0]
    tr = [strs[i][:dist[i]] for i in range(len(strs))]
    for i in range(1, len(strs)):
        a, c = tr[perm[i - 1]], tr[perm[i]]
        assert _py_lcp(a, c) == lcp[i]
        assert a <= c


# ----------------------------------------------------------------------- merge

def _encode_runs_py(runs):
    """Front-code runs given as lists of bytes (sorted within each run), in Python."""
    run_off, lc, ln, ids, suf_off, suf = [0], [], [], [], [0], bytearray()
    for r in runs:
        for p, (sid, x) in enumerate(r):
            e = 0 if p == 0 else _py_lcp(r[p - 1][1], x)
            lc.append(e); ln.append(len(x)); ids.append(sid)
            suf += x[e:]
            suf_off.append(len(suf))
        run_off.append(len(lc))
    return (np.array(run_off, np.uint64), np.array(lc, np.uint32), np.array(ln, np.uint32),
            np.array(ids, np.uint32), np.array(suf_off, np.uint64), np.frombuffer(bytes(suf) or b"\0", np.uint8))


@pytest.mark.parametrize("seed,k", [(0, 1), (1, 2), (2, 5), (3, 16)])
def test_merge_of_random_split_returns_sorted_union(seed, k):
    rng = random.Random(400 + seed)
    strs = _rand_strings(rng, 400, alphabet=(0, 65, 66, 67), max_len=7)
    runs = [[] for _ in range(k)]
    for sid, x in enumerate(strs):
        runs[rng.randrange(k)].append((sid, x))
    runs = [sorted(r, key=lambda t: (t[1], t[0])) for r in runs]
    ro, lc, ln, ids, so, suf = _encode_runs_py(runs)
    src, idv, olcp = oracle.merge(ro, lc, ln, ids, so, suf)
    flat = [(x, ri, p, sid) for ri, r in enumerate(runs) for p, (sid, x) in enumerate(r)]
    expect = sorted(flat, key=lambda t: (t[0], t[1], t[2]))
    assert [((t[1] << 32) | t[2]) for t in expect] == [int(v) for v in src]
    assert [t[3] for t in expect] == list(idv)
    assert olcp[0] == 0
    assert all(olcp[i] == _py_lcp(expect[i - 1][0], expect[i][0]) for i in range(1, len(expect)))


def test_merge_dn_closed_form():
    n, length = 5000, 32
    s = synth.dn_strings(n, length, 0.3, seed=5)
    strs = s.as_list()
    pi = s.meta["pi"].numpy()
    rng = random.Random(5)
    k = 8
    runs = [[] for _ in range(k)]
    for i in range(n):
        runs[rng.randrange(k)].append((i, strs[i]))
    runs = [sorted(r, key=lambda t: pi[t[0]]) for r in runs]   # sorted by construction
    ro, lc, ln, ids, so, suf = _encode_runs_py(runs)
    _, idv, olcp = oracle.merge(ro, lc, ln, ids, so, suf)
    np.testing.assert_array_equal(idv, cf.dn_perm(pi))
    np.testing.assert_array_equal(olcp, cf.dn_lcp(n, s.meta["k"], s.meta["filler"]))


# ------------------------------------------- finish rule, masking, splitter index

@pytest.mark.parametrize("length,l0,expect_rounds", [(8, 8, 1), (16, 8, 2), (32, 8, 3), (4, 4, 1), (12, 4, 3)])
def test_dist_prefix_exhausted_duplicates_leave_when_len_reaches_l(length, l0, expect_rounds):
    """Section 4: a string stops taking part once its tested prefix is unique
    or covers the whole string.  Copies of one string never become unique, so
    they leave in the first round whose tested length l0 * 2^(t-1) reaches
    their length, with dist_approx = len."""
    s = bytes((65 + (7 * i) % 26) for i in range(length))
    b, o = _arrays([s, s, s])
    approx, rounds, coll = oracle.dist_prefix(b, o, l0, 64)
    assert list(approx) == [length] * 3
    assert rounds == expect_rounds
    assert coll == 0


def test_dist_prefix_round_count_closed_form_duplicates_of_many_lengths():
    """Every length from 0 to 70, each string present twice: the round count
    and dist_approx follow the collision-free closed forms exactly."""
    rng = random.Random(11)
    strs = []
    for L in range(71):
        x = bytes(rng.randrange(65, 91) for _ in range(L))
        strs += [x, x]
    rng.shuffle(strs)
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    d = oracle.dist_exact(o, perm, oracle.lcp(b, o, perm))
    lens = (o[1:] - o[:-1]).astype(np.int64)
    approx, rounds, coll = oracle.dist_prefix(b, o, 8, 64)
    assert coll == 0
    assert (approx == lens).all()  # every string has a copy: dist = len
    np.testing.assert_array_equal(approx, cf.doubling_closed_form(d, lens, 8))
    assert rounds == cf.doubling_rounds_closed_form(d, lens, 8) == 5  # 8, 16, 32, 64, 128 >= 70


def _find_key_pair(rng, m, same, differ, tries=200_000):
    """Two random m-byte strings over 'A'..'Z' whose prefix keys agree on the
    bit mask `same` and differ somewhere on the bit mask `differ`."""
    seen = {}
    for _ in range(tries):
        x = bytes(rng.randrange(65, 91) for _ in range(m))
        k = oracle.kr_key(x)
        y = seen.get(k & same)
        if y is not None and y != x and (oracle.kr_key(y) ^ k) & differ:
            return y, x
        seen[k & same] = x
    raise AssertionError("no pair found")


def test_dist_prefix_hash_bits_keeps_the_low_bits():
    """hash_bits = b compares the low b bits of each key.  Pair A: 8-byte
    prefixes whose keys share their low 8 bits (and differ in the high bits)
    collide at b = 8, so both strings stay one more round (a collision only
    delays, Section 4).  Pair B: keys sharing bits 53..63 but not the low 8
    bits do not collide at b = 8.  Keeping any other 8 bits swaps the two
    outcomes."""
    rng = random.Random(5)
    low = (1 << 8) - 1
    high = ~((1 << 53) - 1) & ((1 << 64) - 1)
    a8, a8b = _find_key_pair(rng, 8, same=low, differ=high)
    b8, b8b = _find_key_pair(rng, 8, same=high, differ=low)
    # extend to 16 bytes so that the full keys differ in the low bits
    for _ in range(1000):
        ta = bytes(rng.randrange(65, 91) for _ in range(8))
        tb = bytes(rng.randrange(65, 91) for _ in range(8))
        if (oracle.kr_key(a8 + ta) ^ oracle.kr_key(a8b + tb)) & low:
            break
    pair_a = [a8 + ta, a8b + tb]
    pair_b = [b8 + ta, b8b + tb]
    for strs, want8, want_rounds in ((pair_a, [16, 16], 2), (pair_b, [8, 8], 1)):
        b, o = _arrays(strs)
        approx, rounds, coll = oracle.dist_prefix(b, o, 8, 8)
        assert list(approx) == want8 and rounds == want_rounds
        full, rounds64, _ = oracle.dist_prefix(b, o, 8, 64)
        assert list(full) == [8, 8] and rounds64 == 1  # distinct 8-byte prefixes


def _lower_quantile_positions(n, r):
    """Sorted position of the lower j/r-quantile for j = 1..r-1: the smallest
    position c with (c+1)/n >= j/r (numpy's 'inverted_cdf' quantile of 0..n-1)."""
    pos = np.arange(n)
    out = []
    for j in range(1, r):
        q = float(np.quantile(pos, j / r, method="inverted_cdf"))
        out.append(int(q))
    return out


@pytest.mark.parametrize("n,r", [(10, 4), (250, 7), (250, 64), (1000, 3), (97, 96), (5, 9), (1, 2), (64, 64),
                                 (100_003, 256)])
def test_select_splitters_are_lower_quantiles_with_balanced_buckets(n, r):
    """Regular sampling (Section 3.1) with every string a sample: splitter j is
    the j/r-quantile of the sorted array (the smallest string with at least
    j*n/r strings <= it).  On distinct strings every bucket then holds
    floor(n/r) or ceil(n/r) strings, within the string-based sampling bound
    (1 + r/v) n/r for any sampling factor v."""
    perm = np.arange(n, dtype=np.uint32)[::-1].copy()  # any permutation: ids are perm entries
    ids = oracle.select_splitters(n, perm, r)
    pos = _lower_quantile_positions(n, r)
    assert [int(x) for x in ids] == [int(perm[c]) for c in pos]
    # distinct strings: bucket j = sorted positions (c_{j-1}, c_j]
    bounds = [0] + [c + 1 for c in pos] + [n]
    sizes = np.diff(bounds)
    assert sizes.sum() == n
    assert set(sizes.tolist()) <= {n // r, -(-n // r)}
    for v in (1, 2, 16):
        if v <= n:  # ceil(n/r) <= n/r + 1 <= n/r + n/v
            assert sizes.max() <= (1 + r / v) * n / r


# ------------------------------------------------ character-based sampling

def _sorted_by_len_strings(n, seed, max_len=300):
    """Strings whose sorted order is also increasing length ('A' * k + tail):
    the worst case for string-based splitters, whose last buckets take all
    the long strings."""
    rng = random.Random(seed)
    strs = []
    for i in range(n):
        k = min(max_len - 2, int(rng.paretovariate(1.2))) if rng.random() < 0.9 else rng.randint(100, max_len - 2)
        strs.append(b"A" * k + bytes([66 + rng.randrange(20), 65 + rng.randrange(26)]))
    return strs


@pytest.mark.parametrize("n,r,L", [(10, 4, 3), (250, 7, 1), (250, 64, 5), (1000, 3, 17), (97, 96, 2), (5, 9, 4),
                                   (64, 64, 8), (3000, 128, 9)])
def test_char_splitters_on_equal_lengths_are_the_string_splitters(n, r, L):
    """With every string L characters long, the j-th character quantile lies
    in the j-th string quantile (Section 3.1: character-based sampling
    generalises string-based sampling), so both pick the same strings."""
    rng = random.Random(n + r)
    strs = [bytes(rng.randrange(65, 91) for _ in range(L)) for _ in range(n)]
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    np.testing.assert_array_equal(oracle.select_splitters_chars(perm, o, r), oracle.select_splitters(n, perm, r))
    # equal per-string character counts (e.g. equal distinguishing prefixes) likewise
    w = np.full(n, 3, np.uint32)
    np.testing.assert_array_equal(oracle.select_splitters_chars(perm, o, r, w), oracle.select_splitters(n, perm, r))


def test_char_splitters_count_the_given_characters():
    """Counting given characters (e.g. approximate distinguishing prefixes)
    samples exactly as counting the lengths of strings that long."""
    rng = random.Random(8)
    n = 2000
    strs = [bytes(rng.randrange(65, 70) for _ in range(rng.randint(0, 40))) for _ in range(n)]
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    w = np.array([rng.randint(0, 90) for _ in range(n)], np.uint32)
    o2 = np.concatenate([[0], np.cumsum(w.astype(np.uint64))]).astype(np.uint64)  # strings of length w_i
    for r in (2, 5, 33, 256):
        np.testing.assert_array_equal(oracle.select_splitters_chars(perm, o, r, w),
                                      oracle.select_splitters_chars(perm, o2, r))


@pytest.mark.parametrize("seed,r", [(0, 4), (1, 16), (2, 97), (3, 300)])
def test_char_sample_density(seed, r):
    """Appendix A, character sample density: a contiguous run of the sorted
    array holding k sampled strings has at most (k + 1)(w + l_max)
    characters, w the sampling distance (here ceil(N / r))."""
    strs = _sorted_by_len_strings(3000, seed)
    rng = random.Random(seed)
    rng.shuffle(strs)
    b, o = _arrays(strs)
    perm = oracle.sort(b, o)
    ids = oracle.select_splitters_chars(perm, o, r)
    lens = (o[1:] - o[:-1]).astype(np.int64)
    sl = lens[perm]
    C = np.concatenate([[0], np.cumsum(sl)])
    N, lmax = int(C[-1]), int(sl.max())
    w = -(-N // r)
    pos = {int(x): i for i, x in enumerate(perm)}
    sampled = np.zeros(len(strs), bool)
    for x in ids:
        sampled[pos[int(x)]] = True
    S = np.concatenate([[0], np.cumsum(sampled)])
    for _ in range(3000):
        a = rng.randrange(len(strs))
        e = rng.randrange(a, len(strs)) + 1
        k = int(S[e] - S[a])
        assert C[e] - C[a] <= (k + 1) * (w + lmax)


@pytest.mark.parametrize("seed", range(3))
def test_char_splitters_bound_bucket_characters(seed):
    """Appendix A's bucket bound for character-based regular sampling: with p
    arrays each sampled v + 1 times by characters, sorted samples V and
    f_j = V[j|V|/p - 1], every bucket holds at most
    (1 + p/v) N/p + (1 + (v+1)/p) p l_max characters.  On an input whose long
    strings sort last, string-based samples overload the last bucket."""
    p, v = 8, 4
    strs = _sorted_by_len_strings(4000, 10 + seed)
    random.Random(seed).shuffle(strs)
    b, o = _arrays(strs)
    n = len(strs)
    lens = (o[1:] - o[:-1]).astype(np.int64)
    bounds = [n * i // p for i in range(p + 1)]
    perms = []
    for a, e in zip(bounds[:-1], bounds[1:]):
        sb, so = b[o[a]:o[e]], o[a:e + 1] - o[a]
        perms.append(oracle.sort(sb, so).astype(np.int64) + a)

    def bucket_chars(per_pe_samples):
        V = sorted(set(int(x) for x in per_pe_samples), key=lambda i: (strs[i], i))
        spl = [V[len(V) * j // p - 1] for j in range(1, p)]
        spl_strs = [strs[i] for i in spl]
        sb, so = _arrays(spl_strs)
        tot = np.zeros(p, np.int64)
        for pm in perms:
            bb = oracle.bucket_bounds(b, o, pm.astype(np.uint32), sb, so)
            for j in range(p):
                tot[j] += lens[pm[int(bb[j]):int(bb[j + 1])]].sum()
        return tot

    chars = np.concatenate([oracle.select_splitters_chars(pm.astype(np.uint32), o, v + 2) for pm in perms])
    strings = np.concatenate([oracle.select_splitters(len(pm), pm.astype(np.uint32), v + 2) for pm in perms])
    N, lmax = int(lens.sum()), int(lens.max())
    bound = (1 + p / v) * N / p + (1 + (v + 1) / p) * p * lmax
    by_chars, by_strings = bucket_chars(chars), bucket_chars(strings)
    assert by_chars.sum() == by_strings.sum() == N
    assert by_chars.max() <= bound
    assert by_strings.max() > 2 * by_chars.max()


# ----------------------------------------------------------------- suffixes

def _py_suffix_array(t: bytes):
    sa = sorted(range(len(t)), key=lambda i: t[i:])
    lcp = ([0] if t else []) + [_py_lcp(t[sa[k - 1]:], t[sa[k]:]) for k in range(1, len(t))]
    return sa, lcp


def test_suffix_sort_every_binary_text_up_to_10():
    """All 2^N texts over {0x00, 0x01} (N <= 10) against Python's ordering of
    the suffixes as bytes."""
    for N in range(0, 11):
        for bits in range(1 << N):
            t = bytes((bits >> k) & 1 for k in range(N))
            sa, lcp = oracle.suffix_sort(np.frombuffer(t, np.uint8))
            esa, elcp = _py_suffix_array(t)
            assert list(sa) == esa and list(lcp) == elcp, t


@pytest.mark.parametrize("seed,N,alpha", [(0, 2000, b"AB"), (1, 3000, b"ACGT"), (2, 1500, bytes(range(256))),
                                          (3, 2500, b"A")])
def test_suffix_sort_random_texts(seed, N, alpha):
    rng = random.Random(seed)
    t = bytes(rng.choice(alpha) for _ in range(N))
    sa, lcp = oracle.suffix_sort(np.frombuffer(t, np.uint8))
    esa, elcp = _py_suffix_array(t)
    assert list(sa) == esa and list(lcp) == elcp


def test_suffix_sort_unary_text_closed_form():
    """a^N: shorter suffixes first, lcp of a^(k-1) and a^k is k - 1."""
    N = 5000
    sa, lcp = oracle.suffix_sort(np.full(N, 97, np.uint8))
    assert list(sa) == list(range(N - 1, -1, -1))
    assert list(lcp) == [0] + list(range(1, N))


def test_check_suffixes_accepts_exactly_the_suffix_array():
    t = np.frombuffer(b"mississippi", np.uint8)
    sa, lcp = oracle.suffix_sort(t)
    assert oracle.check_suffixes(t, sa, lcp) == -1
    bad = sa.copy(); bad[[3, 4]] = bad[[4, 3]]
    assert oracle.check_suffixes(t, bad) == 4
    assert oracle.check_suffixes(t, np.zeros(11, np.uint32)) == -2
    wrong = lcp.copy(); wrong[5] += 1
    assert oracle.check_suffixes(t, sa, wrong) == 5
