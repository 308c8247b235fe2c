"""Character-based splitters on the GPU against the oracle, set by set."""
import random

import numpy as np
import pytest
import torch

import oracle
import paper_2404_16517_amd as ss
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def _skewed(n, seed):
    rng = random.Random(seed)
    out = []
    for _ in range(n):
        k = min(400, int(rng.paretovariate(1.1)))
        out.append(b"A" * k + bytes(rng.randrange(65, 91) for _ in range(rng.randint(0, 3))))
    return out


def _cases():
    yield "text", synth.text_strings(60_000, seed=2, median=20), 8
    yield "skewed", synth.from_list(_skewed(30_000, 3) + [b""] * 500), 5
    yield "dn_equal", synth.dn_strings(40_000, 64, 0.5, seed=4), 16
    yield "tiny_sets", synth.from_list([b"", b"AB", b"", b"C" * 50, b"B"] * 7), 7


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("r", [2, 7, 300])
@pytest.mark.parametrize("name,case,p", list(_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_char_splitters_match_oracle_per_set(name, case, p, r, weighted):
    s = case
    g = s.to(DEV)
    n = s.n
    so = torch.tensor([n * i // p for i in range(p + 1)], dtype=torch.int64)
    perm, _ = ss.sort_batch(g.bytes, g.offsets, so.to(DEV), with_lcp=False, global_ids=True)
    w = None
    if weighted:
        w, _ = ss.dist_prefix(g.bytes, g.offsets, 8, 64)
    ids = ss.select_splitters_chars_batch(perm, g.offsets, so, r, weights=w)
    torch.cuda.synchronize()
    got = u32(ids).reshape(p, r - 1)
    pm = u32(perm)
    o = s.offsets.numpy().view(np.uint64)
    wh = u32(w) if weighted else None
    for b in range(p):
        a, e = int(so[b]), int(so[b + 1])
        exp = oracle.select_splitters_chars(pm[a:e], o, r, wh)
        np.testing.assert_array_equal(got[b], exp, err_msg=f"{name} set {b}")
    if name == "dn_equal" and not weighted:  # equal lengths: the string-based samples
        np.testing.assert_array_equal(u32(ids), u32(ss.select_splitters_batch(perm, so, r)))


def test_char_splitters_reject_empty_sets():
    s = synth.from_list([b"B", b"A", b"C"])
    g = s.to(DEV)
    perm = torch.tensor([1, 0, 2], dtype=torch.int32, device=DEV)
    with pytest.raises(ss.StrsortError):
        ss.select_splitters_chars_batch(perm, g.offsets, torch.tensor([0, 0, 3]), 3)


def test_bucket_bounds_of_each_pe_slice():
    """Bucket bounds of one PE's sorted run (a slice of the batch's order,
    whose values index the whole string array) equal the oracle's."""
    s = synth.text_strings(40_000, seed=6, median=12)
    g = s.to(DEV)
    p = 8
    so = torch.tensor([s.n * i // p for i in range(p + 1)], dtype=torch.int64)
    perm, _ = ss.sort_batch(g.bytes, g.offsets, so.to(DEV), with_lcp=False, global_ids=True)
    samp = ss.select_splitters_chars_batch(perm, g.offsets, so, 4)
    sb, sof = ss.gather_strings(g.bytes, g.offsets, samp)
    sperm, _ = ss.sort(sb, sof, with_lcp=False)
    fb, fo = ss.gather_strings(sb, sof, ss.select_splitters(sperm, p))
    b, o = oracle.strings_np(s)
    fbh, foh = fb.cpu().numpy(), fo.cpu().numpy().view(np.uint64)
    pm = u32(perm)
    for j in range(p):
        a, e = int(so[j]), int(so[j + 1])
        got = ss.bucket_bounds(g.bytes, g.offsets, perm[a:e], fb, fo)
        np.testing.assert_array_equal(got.cpu().numpy().view(np.uint64),
                                      oracle.bucket_bounds(b, o, pm[a:e], fbh, foh), err_msg=f"PE {j}")
