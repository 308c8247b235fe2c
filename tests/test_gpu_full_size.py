"""GPU parity at the workloads' full sizes.

At these sizes the oracle cannot redo the whole computation within a test, so
each case is checked by what the oracle can compute one by one or by
properties that hold at any size:

* text strings, 50M (log-normal lengths, Zipf bytes, 20% duplicates): the
  sorted order and LCP array by the oracle's linear-time check of every
  adjacent pair; exact dist from them; prefix doubling by its collision-free
  closed forms (dist_approx and the round count);
* the k-way merge, 256 front-coded runs of 64M D/N strings of 64 bytes
  (D/N 0.3), built from the D/N closed forms: the merged order and LCPs equal
  the closed forms, with full strings and with distinguishing prefixes only;
* 4096 independent sets of 1e3..1e6 strings (lengths 8..256): every set with
  index = 0 mod 64, the smallest and the largest against the oracle's sort;
* the whole PDMS step on 16M D/N strings of 500 bytes (D/N 0.5, 16 virtual
  PEs, sampling factor 2) in the benchmark's launch configuration (seeded
  first hash pass, later doubling rounds on a second stream beside the sort),
  twice on the same buffers: the merged order and LCPs by the oracle's check
  of every adjacent pair, dist by the oracle from them, and every output
  against the D/N closed forms.
"""
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


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_text_50M_sort_lcp_and_prefix_doubling():
    n = 50_000_000
    _log("[full] text 50M: generate")
    s = synth.text_strings(n, seed=0, device=DEV)
    perm, lcp = ss.sort(s.bytes, s.offsets)
    dpx, rounds = ss.dist_prefix(s.bytes, s.offsets, 8, 64)
    torch.cuda.synchronize()
    _log("[full] text 50M: check")
    b = s.bytes.cpu().numpy()
    o = s.offsets.cpu().numpy().view(np.uint64)
    del s
    p, l = u32(perm), u32(lcp)
    assert oracle.check_sorted(b, o, p, l) == -1
    dist = oracle.dist_exact(o, p, l)
    lens = (o[1:] - o[:-1]).astype(np.int64)
    d = u32(dpx)
    assert (d >= dist).all()
    np.testing.assert_array_equal(d, cf.doubling_closed_form(dist, lens, 8))
    assert rounds == cf.doubling_rounds_closed_form(dist, lens, 8)


@pytest.mark.parametrize("pdms", [False, True])
def test_merge_256_runs_of_64M_dn_strings(pdms):
    n, k = 64_000_000, 256
    _log(f"[full] merge 256 runs x 64M, pdms={pdms}: build runs")
    s = synth.dn_strings(n, 64, 0.3, seed=3, device=DEV)
    run = synth.random_runs(n, k, 3, device=DEV)
    run_off, e, d, ids, suf_off, suf = cf.dn_front_coded_runs(s, run, k, pdms)
    assert (s.meta["k"], s.meta["filler"]) == (6, 13)
    _log("[full] merge")
    _, gid, glcp = ss.lcp_merge_runs(run_off, e, d, ids, suf_off, suf)
    torch.cuda.synchronize()
    pi = s.meta["pi"].numpy()
    np.testing.assert_array_equal(u32(gid), cf.dn_perm(pi))
    np.testing.assert_array_equal(u32(glcp), cf.dn_lcp(n, 6, 13))


def test_4096_sets_of_1e3_to_1e6_strings_sampled_against_the_oracle():
    _log("[full] 4096 sets: generate")
    s, bounds = synth.random_sets(4096, 1e3, 1e6, 8, 256, seed=0, device=DEV)
    sizes = np.diff(bounds.numpy())
    n = int(bounds[-1])
    _log(f"[full] 4096 sets: n={n} N={s.N}: sort")
    perm, lcp = ss.sort_batch(s.bytes, s.offsets, bounds.to(DEV))
    torch.cuda.synchronize()
    pick = sorted(set(range(0, 4096, 64)) | {int(np.argmin(sizes)), int(np.argmax(sizes))})
    assert sizes.min() >= 1000 and sizes.max() <= 1_000_000
    offs = s.offsets
    for j in pick:
        a, c = int(bounds[j]), int(bounds[j + 1])
        b0, b1 = int(offs[a]), int(offs[c])
        b = s.bytes[b0:b1].cpu().numpy()
        o = (offs[a:c + 1] - b0).cpu().numpy().view(np.uint64)
        p_ref = oracle.sort(b, o)
        np.testing.assert_array_equal(u32(perm[a:c]), p_ref, err_msg=f"set {j}")
        np.testing.assert_array_equal(u32(lcp[a:c]), oracle.lcp(b, o, p_ref), err_msg=f"set {j}")
    _log(f"[full] 4096 sets: {len(pick)} sets checked")


def test_dn_16M_pdms_step_in_the_benchmark_configuration():
    import bench
    n, length, ratio, pes, v = 16_000_000, 500, 0.5, 16, 2
    _log("[full] D/N 16M step: generate")
    s = synth.dn_strings(n, length, ratio, seed=0, device=DEV)
    pipe = bench.Pipeline(s.bytes, s.offsets, pes, v, ss, torch, overlap=True)
    assert pipe.seeded and pipe.overlap
    marks = bench.Marks(torch, False)
    outs = []
    for rep in range(2):
        _log(f"[full] D/N 16M step: run {rep}")
        order, mlcp, dist, dpx, rounds = pipe.step(marks)
        torch.cuda.synchronize()
        outs.append([u32(t).copy() for t in (order, mlcp, dist, dpx)] + [rounds])
    _log("[full] D/N 16M step: check")
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    order, mlcp, dist, dpx, rounds = outs[0]
    k, F, pi = s.meta["k"], s.meta["filler"], s.meta["pi"].numpy()
    b = s.bytes.cpu().numpy()
    o = s.offsets.cpu().numpy().view(np.uint64)
    del pipe, s
    assert oracle.check_sorted(b, o, order, mlcp) == -1
    del b
    d_in = oracle.dist_exact(o, order, mlcp)  # by string, from the checked order and LCPs
    np.testing.assert_array_equal(dist, d_in[order])  # the step's dist is by merged position
    np.testing.assert_array_equal(dpx, cf.doubling_closed_form(d_in, np.full(n, length), 8))
    np.testing.assert_array_equal(order, cf.dn_perm(pi))
    np.testing.assert_array_equal(mlcp, cf.dn_lcp(n, k, F))
    np.testing.assert_array_equal(dist, cf.dn_dist_sorted(n, k, F, length))
