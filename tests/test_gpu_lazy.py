"""GPU parity of the deep first pass that leaves its rounds of <= 64 bytes
unhashed.  It certifies how long a prefix every string shares with string 0
and the shortest length; the rounds call skips those rounds when the
certificate shows they finish nothing, and hashes them with the plain pass
otherwise.  Each case forces the deep pass on inputs that take one branch or
the other, and checks dist_approx and the round count against the oracle.
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


def _shared(n, prefix, seed, odd=()):
    """n strings = prefix + distinct tails; `odd` lists (index, string) overrides."""
    rng = random.Random(seed)
    out = [prefix + b"%07d" % rng.randrange(10**7) + bytes(rng.choice(b"xyz") for _ in range(rng.randint(0, 40)))
           for _ in range(n)]
    for i, s in odd:
        out[i] = s
    return synth.from_list(out)


P = b"Q" * 300
CASES = {
    # every string shares 300 bytes, none short: the small rounds are skipped
    "certified": lambda: _shared(20_000, P, 1),
    # a few strings differ from the rest at byte 10: the small rounds are hashed
    "differ_early": lambda: _shared(20_000, P, 2, [(17, b"Q" * 10 + b"R" * 300), (19_000, b"A" * 400)]),
    # short strings (prefixes of the others): hashed
    "short": lambda: _shared(20_000, P, 3, [(5, b"Q" * 30), (6, b"Q" * 30), (7_000, b"Q" * 64)]),
    # a string of exactly 64 bytes equal to the others' first 64: hashed
    "len64": lambda: _shared(20_000, P, 4, [(123, b"Q" * 64)]),
    # string 0 itself differs early
    "first_differs": lambda: _shared(20_000, P, 5, [(0, b"Z" * 350)]),
    # D/N strings (the benchmark's kind)
    "dn": lambda: synth.dn_strings(30_000, 500, 0.6, seed=6),
}


def _sets(n, k):
    return torch.tensor([n * i // k for i in range(k + 1)], dtype=torch.int64, device=DEV)


@pytest.mark.parametrize("sets", [0, 16, 40])
@pytest.mark.parametrize("case", sorted(CASES))
def test_lazy_small_rounds(case, sets):
    s = CASES[case]()
    _log(f"[lazy] {case} sets={sets} n={s.n}")
    g = s.to(DEV)
    so = _sets(s.n, sets) if sets else None
    ws, seed = ss.dist_prefix_first_seed(g.bytes, g.offsets, 8, 64, first_pass="deep", set_off=so)
    got, rounds = ss.dist_prefix_rounds(g.bytes, g.offsets, ws, 8, 64)
    torch.cuda.synchronize()
    b, o = oracle.strings_np(s)
    ref, r_ref, _ = oracle.dist_prefix(b, o, 8, 64)
    np.testing.assert_array_equal(got.cpu().numpy().view(np.uint32), ref)
    assert rounds == r_ref
    # the seed is still right: the seeded batch sort agrees with the unseeded one
    if sets and sets <= 16:
        p1, l1 = ss.sort_batch_seeded(g.bytes, g.offsets, so, seed, global_ids=True)
        p2, l2 = ss.sort_batch(g.bytes, g.offsets, so, global_ids=True)
        torch.cuda.synchronize()
        assert torch.equal(p1, p2) and torch.equal(l1, l2)


def test_doubling_keys_unaffected():
    """ss_doubling_keys (which exposes every round's keys) still hashes the
    small rounds in the deep pass: its keys equal the plain pass's."""
    s = CASES["certified"]().to(DEV)
    kd = ss.doubling_keys(s.bytes, s.offsets, 8, 6, 64, first_pass="deep")
    kp = ss.doubling_keys(s.bytes, s.offsets, 8, 6, 64, first_pass="plain")
    torch.cuda.synchronize()
    assert torch.equal(kd, kp)
