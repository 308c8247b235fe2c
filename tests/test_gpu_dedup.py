"""GPU parity of prefix doubling's duplicate detection in each of its forms:
the global hash table, and buckets of keys counted in LDS (with the number of
buckets forced low, so that buckets hold more distinct keys than one LDS pass
takes and are counted in several passes).  Every form must give the oracle's
dist_approx and round count exactly.
"""
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


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _heavy(seed):
    """One string repeated 30,000 times among 30,000 distinct ones, plus
    pairs: a bucket that holds many copies of one key."""
    rng = random.Random(seed)
    out = [b"HEAVY-HITTER-STRING-" * 3] * 30_000
    out += [b"u%09d" % rng.randrange(10**9) + bytes(rng.choice(b"xy") for _ in range(rng.randint(0, 30)))
            for _ in range(30_000)]
    out += [b"pair%06d" % k for k in range(5_000)] * 2
    rng.shuffle(out)
    return synth.from_list(out)


CASES = {
    "dn": (lambda: synth.dn_strings(80_000, 120, 0.5, seed=3), 64),
    "text": (lambda: synth.text_strings(120_000, seed=4), 64),
    "text_bits12": (lambda: synth.text_strings(70_000, seed=5), 12),
    "heavy": (lambda: _heavy(6), 64),
}

MODES = [
    ("table", 0, 0),
    ("buckets", 2, 0),
    ("two_buckets", 2, 1),   # ~35K+ distinct keys per bucket: several LDS passes
    ("eight_buckets", 2, 3),
    ("long_lists", 1, 0),
]


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
@pytest.mark.parametrize("case", sorted(CASES))
def test_duplicate_detection_forms(case, mode):
    make, bits = CASES[case]
    s = make()
    name, dm, logb = mode
    _log(f"[dedup] {case} form={name} n={s.n} bits={bits}")
    g = s.to(DEV)
    old = ss.set_tuning(ss.SS_TUNE_DEDUP, dm)
    oldb = ss.set_tuning(ss.SS_TUNE_DEDUP_LOG_BUCKETS, logb)
    try:
        got, rounds = ss.dist_prefix(g.bytes, g.offsets, 8, bits)
        torch.cuda.synchronize()
    finally:
        ss.set_tuning(ss.SS_TUNE_DEDUP, old)
        ss.set_tuning(ss.SS_TUNE_DEDUP_LOG_BUCKETS, oldb)
    b, o = oracle.strings_np(s)
    ref, r_ref, _ = oracle.dist_prefix(b, o, 8, bits)
    np.testing.assert_array_equal(got.cpu().numpy().view(np.uint32), ref)
    assert rounds == r_ref


def test_bucket_form_matches_table_at_full_size():
    """16M D/N strings (the benchmark's input): both forms, key for key the
    same dist_approx (and the D/N closed form's round count)."""
    s = synth.dn_strings(16_000_000, 500, 0.5, seed=0, device=DEV)
    out = {}
    for dm in (0, 1):
        old = ss.set_tuning(ss.SS_TUNE_DEDUP, dm)
        try:
            out[dm] = ss.dist_prefix(s.bytes, s.offsets, 8, 64)
            torch.cuda.synchronize()
        finally:
            ss.set_tuning(ss.SS_TUNE_DEDUP, old)
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
