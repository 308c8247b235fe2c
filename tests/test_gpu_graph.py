"""The device-driven batch sort (nothing read back) and its capture in a graph.

The device-driven form must give exactly the host-driven result (and the
oracle's) when enough rounds are enqueued, report unresolved work when too
few are, and replay correctly from a graph: each replay, after the input
buffers have been rewritten by eager work, is checked against the eager
result and the oracle."""
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


def _buffers(n, dev=DEV):
    return (torch.empty(max(n, 1), dtype=torch.int32, device=dev), torch.empty(max(n, 1), dtype=torch.int32, device=dev),
            torch.full((2,), -1, dtype=torch.int32, device=dev),
            torch.empty(max(ss.lib().ss_sort_workspace(n), 1), dtype=torch.uint8, device=dev))


def _cases():
    edge = [[b"HELLO"], [b"AB", b"AB"], [b"", b"", b"A", b""], [b"SAME" * 5] * 300,
            [b"A" * k for k in range(40, 0, -1)] + [b""],
            [b"\x00", b"\x00\x00", b"", b"\xff", b"\xff\x00", b"\x00\xff", b"A\x00", b"A", b"A\x00\x00"],
            [b"P" * 300 + bytes([65 + (i * 7) % 26]) + b"X" * (i % 5) for i in range(500)],
            [b"Q" * 4096 + b"Z"] + [b"Q" * k for k in range(1, 60)] + [b"Q" * 4096 + b"A"]]
    yield "edge_sets", synth.concat([synth.from_list(e) for e in edge])
    yield "dn_500", synth.concat([synth.dn_strings(20_000, 500, 0.5, seed=s) for s in range(3)])
    yield "random_sets", synth.random_sets(200, 1e2, 3e4, 8, 256, seed=4)
    yield "text", synth.concat([synth.text_strings(5_000 * (s + 1), seed=s) for s in range(4)])


@pytest.mark.parametrize("name,case", list(_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_device_driven_equals_host_driven_and_oracle(name, case):
    s, bounds = case
    g = s.to(DEV)
    so = bounds.to(DEV)
    n = s.n
    max_len = int((s.offsets[1:] - s.offsets[:-1]).max())
    perm, lcp, status, ws = _buffers(n)
    ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, ss.sort_batch_device_rounds(max_len))
    ref_perm, ref_lcp = ss.sort_batch(g.bytes, g.offsets, so)
    torch.cuda.synchronize()
    assert status.tolist() == [0, 0]
    assert torch.equal(perm[:n], ref_perm) and torch.equal(lcp[:n], ref_lcp)
    b, o = oracle.strings_np(s)
    bnd = bounds.tolist()
    for j in range(0, len(bnd) - 1, max(1, (len(bnd) - 1) // 6)):
        a, c = bnd[j], bnd[j + 1]
        sb, sob = b[o[a]:o[c]], o[a:c + 1] - o[a]
        p_ref = oracle.sort(sb, sob)
        np.testing.assert_array_equal(u32(perm[a:c]), p_ref)
        np.testing.assert_array_equal(u32(lcp[a:c]), oracle.lcp(sb, sob, p_ref))


def test_too_few_rounds_report_unresolved_segments():
    s = synth.from_list([b"P" * 300 + bytes([65 + i % 26]) for i in range(400)])
    g = s.to(DEV)
    so = torch.tensor([0, s.n], dtype=torch.int64, device=DEV)
    perm, lcp, status, ws = _buffers(s.n)
    # the first round skips the 300 common bytes and resolves everything
    ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, 1)
    torch.cuda.synchronize()
    assert status.tolist() == [0, 0]
    # strings equal for 20 bytes after a skip point: two rounds of 7 are not enough
    strs = [bytes([65 + i % 3]) + b"Z" * 20 + bytes([65 + i % 26]) for i in range(400)]
    s = synth.from_list(strs)
    g = s.to(DEV)
    perm, lcp, status, ws = _buffers(s.n)
    ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, 1)
    torch.cuda.synchronize()
    assert status[0].item() > 0 and status[1].item() == 0
    ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, ss.sort_batch_device_rounds(22))
    torch.cuda.synchronize()
    assert status.tolist() == [0, 0]
    b, o = oracle.strings_np(s)
    p_ref = oracle.sort(b, o)
    np.testing.assert_array_equal(u32(perm), p_ref)
    np.testing.assert_array_equal(u32(lcp), oracle.lcp(b, o, p_ref))


@pytest.mark.parametrize("odd", [False, True])
@pytest.mark.parametrize("finish", ["host", "device"])
def test_incomplete_device_sort_continues_to_the_oracle_result(finish, odd):
    """A device-driven sort stopped after one or two rounds (leaving
    segments for later rounds, in either list) is finished by a continuation:
    host-driven, or device-driven with more rounds."""
    rng = np.random.default_rng(3)
    strs = [bytes([65 + i % 4]) + b"Z" * int(rng.integers(10, 30)) + bytes([65 + int(x) for x in rng.integers(0, 3, 3)])
            for i in range(3000)]
    s1 = synth.from_list(strs[:1700])
    s2 = synth.from_list(strs[1700:])
    s, bounds = synth.concat([s1, s2])
    g = s.to(DEV)
    so = bounds.to(DEV)
    perm, lcp, status, ws = _buffers(s.n)
    ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, 2 if odd else 1)
    torch.cuda.synchronize()
    assert status[0].item() > 0
    if finish == "host":
        ss.sort_batch(g.bytes, g.offsets, so, ws=ws, out=(perm, lcp))
    else:
        ss.sort_batch_device(g.bytes, g.offsets, so, perm, lcp, status, ws, ss.sort_batch_device_rounds(40),
                             cont=True)
    torch.cuda.synchronize()
    if finish == "device":
        assert status.tolist() == [0, 0]
    b, o = oracle.strings_np(s)
    for a, c in ((0, 1700), (1700, 3000)):
        sb, sob = b[o[a]:o[c]], o[a:c + 1] - o[a]
        p_ref = oracle.sort(sb, sob)
        np.testing.assert_array_equal(u32(perm[a:c]), p_ref)
        np.testing.assert_array_equal(u32(lcp[a:c]), oracle.lcp(sb, sob, p_ref))


def test_device_driven_flags_malformed_sets():
    s = synth.from_list([b"B", b"A", b"C", b"A"])
    g = s.to(DEV)
    bad = torch.tensor([0, 3, 2, 4], dtype=torch.int64, device=DEV)
    perm, lcp, status, ws = _buffers(4)
    ss.sort_batch_device(g.bytes, g.offsets, bad, perm, lcp, status, ws, 2)
    torch.cuda.synchronize()
    assert status[1].item() == 1


def test_graph_replays_match_eager_results_each_time():
    """Batch sort + exact dist captured once, replayed three times over new
    data written into the same buffers (a letter rotation, so every replay
    sorts a different order)."""
    s, bounds = synth.random_sets(96, 1e2, 2e4, 8, 64, seed=9, device=DEV)
    so = bounds.to(DEV)
    n = s.n
    base = s.bytes.clone()
    perm, lcp, status, ws = _buffers(n)
    dist = torch.zeros(n, dtype=torch.int32, device=DEV)
    rounds = ss.sort_batch_device_rounds(64)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()

    def body():
        ss.sort_batch_device(s.bytes, s.offsets, so, perm, lcp, status, ws, rounds, global_ids=True)
        ss.dist_exact(s.offsets, perm, lcp, out=dist)

    graph = ss.Graph.capture(body, st)
    assert graph.nodes() > 20
    b0, o0 = oracle.strings_np(s)
    for rep in range(3):
        s.bytes.copy_((base - 65 + 7 * rep) % 26 + 65)  # eager work between replays
        torch.cuda.synchronize()
        status.fill_(-1)
        torch.cuda.synchronize()
        graph.launch(st)
        st.synchronize()
        assert status.tolist() == [0, 0], rep
        ref_perm, ref_lcp = ss.sort_batch(s.bytes, s.offsets, so, global_ids=True)
        ref_dist = ss.dist_exact(s.offsets, ref_perm, ref_lcp)
        torch.cuda.synchronize()
        assert torch.equal(perm, ref_perm) and torch.equal(lcp, ref_lcp) and torch.equal(dist, ref_dist), rep
        b = ((b0.astype(np.int64) - 65 + 7 * rep) % 26 + 65).astype(np.uint8)
        for j in (0, 47, 95):
            a, c = int(bounds[j]), int(bounds[j + 1])
            sb, sob = b[o0[a]:o0[c]], o0[a:c + 1] - o0[a]
            p_ref = oracle.sort(sb, sob)
            np.testing.assert_array_equal(u32(perm[a:c]) - a, p_ref, err_msg=f"replay {rep} set {j}")
    graph.close()
