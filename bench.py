"""Benchmark of the one-GPU string-sorting hot path (prints ONE JSON line).

Workload (default): 16,000,000 strings x 500 bytes over 'A'..'Z' with D/N
ratio 0.5 (the paper's DNData shape; N = 8.0 GB), resident in HBM.

One step = the paper's single-level prefix-doubling merge sort (Section 3 with
k = 1, prefix doubling of Section 4) executed for p virtual processing elements
on one GPU; PE i holds the i-th 1/p of the input, and the exchange between
PEs is replaced by runs that already sit in HBM:
  1. approximate distinguishing prefixes by prefix doubling (hash rounds +
     duplicate detection over all strings),
  2. every PE sorts its array and builds its LCP array (one batched launch);
     steps 1 and 2 are independent: 1 runs on a second stream, driven by a
     worker thread, while 2 and 3 run (joined before 4; --serial runs them
     one after the other on one stream),
  3. regular sampling with sampling factor v = 2: v+1 samples per PE, sorted,
     splitters f_j = V[j|V|/p - 1],
  4. every PE splits its array into p buckets and front-codes the
     distinguishing prefixes of each bucket,
  5. bucket j merges the p runs it receives with the LCP-aware merge (all p
     merges in one call),
  6. exact distinguishing prefixes of the final order, by merged position as
     each PE holds its output (after joining the LCPs across bucket
     boundaries).
value = N / (seconds per step), in GB/s ("string bytes sorted per second").
"""
from __future__ import annotations

import argparse
import concurrent.futures
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


class Pipeline:
    def __init__(self, B, O, p, v, ss, torch, overlap=True, first_alone=False, seeded=True):
        self.B, self.O, self.p, self.v, self.ss, self.torch = B, O, p, v, ss, torch
        dev = B.device
        self.overlap = overlap
        # seeded: prefix doubling's first pass reads every string's first 256
        # bytes once for both passes (it leaves each PE's sort its first
        # round's comparisons); the sort then runs beside the later rounds
        self.seeded = seeded
        # first_alone: run prefix doubling's first pass (which reads the same
        # first bytes of every string as the sort's first round) alone, and
        # only its later rounds and duplicate detection beside the sort (on
        # the default workload the step is then ~0.55 ms slower than with all
        # of it beside the sort)
        self.first_alone = first_alone
        self.ms_mode = False  # True: the paper's MS (full strings, no prefix doubling) instead of PDMS
        self.literal_bytes = 0
        if overlap:
            self.side = torch.cuda.Stream(device=dev)
            self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        n = O.numel() - 1
        self.n = n
        self.bounds = [n * i // p for i in range(p + 1)]
        self.set_off = torch.tensor(self.bounds, dtype=torch.int64, device=dev)
        self.max_len = max(int((O[1:] - O[:-1]).max()), 1) if n else 1
        self.ws_sort = torch.empty(ss.lib().ss_sort_workspace(n), dtype=torch.uint8, device=dev)
        self.ws_pd = torch.empty(ss.lib().ss_dist_prefix_workspace(n), dtype=torch.uint8, device=dev)
        self.ws_merge = torch.empty(ss.lib().ss_lcp_merge_workspace(n, n, p * p), dtype=torch.uint8, device=dev)
        self.ws_pe = torch.empty(ss.lib().ss_partition_encode_workspace(n), dtype=torch.uint8, device=dev)
        self.seed = torch.empty(ss.lib().ss_sort_seed_bytes(n), dtype=torch.uint8, device=dev)
        self.group_off = torch.arange(0, p * p + 1, p, dtype=torch.int32, device=dev)

    def step(self, marks):
        ss, torch, B, O, p = self.ss, self.torch, self.B, self.O, self.p
        ev = marks.mark
        # 1. prefix doubling over all strings (on the side stream: it shares
        #    nothing with 2 and 3 but the input, and its host thread's waits
        #    for its own read-backs do not hold up the sort's launches)
        if self.ms_mode:
            dpx, rounds = None, 0
        elif self.seeded:
            main = torch.cuda.current_stream()
            ss.dist_prefix_first_seed(B, O, 8, 64, ws=self.ws_pd, seed=self.seed, set_off=self.set_off)
            ev("dist_prefix first pass")
            if self.overlap:
                self.side.wait_stream(main)
                fut = self.pool.submit(self._dist_prefix, marks)
        elif self.overlap:
            main = torch.cuda.current_stream()
            if self.first_alone:
                ss.dist_prefix_first(B, O, 8, 64, ws=self.ws_pd)
                ev("dist_prefix first pass")
            self.side.wait_stream(main)
            fut = self.pool.submit(self._dist_prefix, marks)
        else:
            dpx, rounds = ss.dist_prefix(B, O, 8, 64, ws=self.ws_pd)
            ev("dist_prefix")
        # 2. every PE sorts its array (+ LCP), one batched launch sequence
        if self.seeded and not self.ms_mode:
            perm, lcp = ss.sort_batch_seeded(B, O, self.set_off, self.seed, ws=self.ws_sort, global_ids=True)
        else:
            perm, lcp = ss.sort_batch(B, O, self.set_off, ws=self.ws_sort, global_ids=True)
        ev("sort_batch+lcp")
        if self.seeded and not self.ms_mode and not self.overlap:
            dpx, rounds = ss.dist_prefix_rounds(B, O, self.ws_pd, 8, 64)
            ev("dist_prefix rounds")
        # 3. regular sampling (v+1 samples per PE) and splitters (the sets are
        #    well formed by construction and the sample strings' longest
        #    length is known: nothing is read back)
        samp = ss.select_splitters_batch(perm, self.set_off, self.v + 2, check=False)
        sb, so = ss.gather_strings(B, O, samp, cap_hint=samp.numel() * self.max_len, sync=False)
        sperm, _ = ss.sort(sb, so, with_lcp=False)
        fid = ss.select_splitters(sperm, p)
        fb, fo = ss.gather_strings(sb, so, fid, cap_hint=fid.numel() * self.max_len, sync=False)
        ev("splitters")
        if self.overlap and not self.ms_mode:
            dpx, rounds = fut.result()
            main.wait_stream(self.side)
            dpx.record_stream(main)
            ev("join")
        # 4. every PE splits its array into p buckets and front-codes the
        #    distinguishing prefixes (all PEs in one batched call)
        fc = ss.partition_encode_batch(B, O, self.set_off, perm, lcp, dpx, fb, fo, ws=self.ws_pe)
        self.literal_bytes = fc["total"]
        ev("partition_encode")
        # 5. bucket j merges run (i, j) of every PE i: all p merges in one call
        ro = fc["run_off"].view(p, p + 1)                              # [PE, bucket bound], absolute
        run_begin = ro[:, :-1].t().reshape(-1)                          # group j = bucket j, run i = PE i
        run_end = ro[:, 1:].t().reshape(-1)
        _, order, mlcp, mlen = ss.lcp_merge(run_begin, run_end, self.group_off, fc["lcp"], fc["len"], fc["id"],
                                              fc["suf_off"], fc["suf"], ws=self.ws_merge, n_out=self.n,
                                              with_len=True, with_src=False)
        ev("lcp_merge")
        # 6. LCPs across bucket boundaries, exact distinguishing prefixes (the
        #    merged prefix lengths bound them: dist <= approximate dist <= len)
        ss.join_group_lcps(B, O, order, mlcp, run_begin, run_end, self.group_off)
        dist = ss.dist_exact_bounded(None, mlcp, mlen)  # by merged position
        ev("dist_exact")
        return order, mlcp, dist, dpx, rounds

    def _dist_prefix(self, marks):
        with self.torch.cuda.stream(self.side):
            marks.mark("side_start", side=True)
            if self.first_alone or self.seeded:
                r = self.ss.dist_prefix_rounds(self.B, self.O, self.ws_pd, 8, 64)
            else:
                r = self.ss.dist_prefix(self.B, self.O, 8, 64, ws=self.ws_pd)
            marks.mark("dist_prefix (side stream)", side=True)
            return r


class Marks:
    """Events between the stages; each stage's time runs from the previous
    event on its own stream (the main one, or the side one)."""

    def __init__(self, torch, record):
        self.torch, self.record, self.ev, self.side = torch, record, [], []
        if record:
            self.mark("start")

    def mark(self, name, side=False):
        if self.record:
            e = self.torch.cuda.Event(enable_timing=True)
            e.record()
            (self.side if side else self.ev).append((name, e))

    def times(self):
        t = {}
        for ev in (self.ev, self.side):
            t.update({b: ea.elapsed_time(eb) for (a, ea), (b, eb) in zip(ev[:-1], ev[1:])})
        return t


def verify_dn(s, order, mlcp, dist, dpx):
    """Closed forms of the D/N workload (sorted order, LCP, dist, prefix doubling)."""
    import numpy as np
    from tests import closed_forms as cf
    n, L = s.n, s.meta["length"]
    k, F = s.meta["k"], s.meta["filler"]
    pi = s.meta["pi"].numpy()
    perm_ref = cf.dn_perm(pi)
    ok = np.array_equal(order.cpu().numpy().view(np.uint32), perm_ref)
    ok &= np.array_equal(mlcp.cpu().numpy().view(np.uint32), cf.dn_lcp(n, k, F))
    d_sorted = cf.dn_dist_sorted(n, k, F, L)
    ok &= np.array_equal(dist.cpu().numpy().view(np.uint32), d_sorted)
    d_in = np.empty(n, np.uint32)
    d_in[perm_ref] = d_sorted
    ok &= np.array_equal(dpx.cpu().numpy().view(np.uint32), cf.doubling_closed_form(d_in, np.full(n, L), 8))
    return bool(ok)


def batch_leg(ss, torch, synth, num_sets=4096, lo=1e3, hi=1e6, len_lo=8, len_hi=256, reps=3, graph_rounds=3):
    """Many independent sorts (+ LCP): the device-driven batch sort captured in
    a graph and replayed, the host-driven batch sort, and one call per set, at
    equal output; a few sets are also checked against the oracle."""
    import numpy as np
    import oracle
    dev = torch.device("cuda:0")
    S, bounds = synth.random_sets(num_sets, lo, hi, len_lo, len_hi, seed=5, device=dev)
    bl = bounds.tolist()
    bd = bounds.to(dev)
    n = S.n
    ws = torch.empty(ss.lib().ss_sort_workspace(n), dtype=torch.uint8, device=dev)
    # host-driven batch (reads counts back between levels)
    pb, lb = ss.sort_batch(S.bytes, S.offsets, bd, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pb, lb = ss.sort_batch(S.bytes, S.offsets, bd, ws=ws)
    torch.cuda.synchronize()
    t_host = (time.perf_counter() - t0) / reps
    # device-driven batch captured once (a few rounds: enough for these
    # strings unless 7-byte runs repeat), replayed; the status word is read
    # after each replay and an incomplete sort would be finished host-driven
    pg = torch.empty(n, dtype=torch.int32, device=dev)
    lg = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.full((2,), -1, dtype=torch.int32, device=dev)
    st = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    graph = ss.Graph.capture(lambda: ss.sort_batch_device(S.bytes, S.offsets, bd, pg, lg, status, ws,
                                                           graph_rounds), st)
    continued = 0

    def replay():
        nonlocal continued
        graph.launch(st)
        st.synchronize()
        if status[0].item() != 0:
            continued += 1
            with torch.cuda.stream(st):
                ss.sort_batch(S.bytes, S.offsets, bd, ws=ws, out=(pg, lg))
            st.synchronize()
    replay()
    t0 = time.perf_counter()
    for _ in range(reps):
        replay()
    t_graph = (time.perf_counter() - t0) / reps
    nodes = graph.nodes()
    graph.close()
    complete = status[1].item() == 0
    same_graph = torch.equal(pg, pb) and torch.equal(lg, lb)

    def per_job():
        outs = []
        for a, b in zip(bl[:-1], bl[1:]):
            outs.append(ss.sort(S.bytes, S.offsets[a:b + 1], ws=ws))
        return outs
    per_job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = per_job()
    torch.cuda.synchronize()
    t_job = time.perf_counter() - t0
    same_job = torch.equal(torch.cat([o[0] for o in outs]), pb) and torch.equal(torch.cat([o[1] for o in outs]), lb)
    del outs
    sizes = np.diff(np.array(bl))
    checked = sorted({0, num_sets // 2, int(np.argmin(sizes)), int(np.argmax(sizes))})
    oracle_ok = True
    for j in checked:
        a, c = bl[j], bl[j + 1]
        b0, b1 = int(S.offsets[a]), int(S.offsets[c])
        hb = S.bytes[b0:b1].cpu().numpy()
        ho = (S.offsets[a:c + 1] - b0).cpu().numpy().view(np.uint64)
        p_ref = oracle.sort(hb, ho)
        oracle_ok &= bool(np.array_equal(pg[a:c].cpu().numpy().view(np.uint32), p_ref))
        oracle_ok &= bool(np.array_equal(lg[a:c].cpu().numpy().view(np.uint32), oracle.lcp(hb, ho, p_ref)))
    out = {"sets": num_sets, "set_sizes": f"log-uniform [{lo:.0f}, {hi:.0f}] strings",
           "lengths": f"uniform [{len_lo}, {len_hi}] bytes, 'A'..'Z'", "strings": n, "bytes": S.N,
           "graph_sets_per_s": num_sets / t_graph, "host_driven_sets_per_s": num_sets / t_host,
           "per_set_call_sets_per_s": num_sets / t_job,
           "graph_speedup_over_per_set_calls": t_job / t_graph, "graph_ms": t_graph * 1e3,
           "host_driven_ms": t_host * 1e3, "per_set_calls_ms": t_job * 1e3,
           "graph_GBps": S.N / t_graph / 1e9, "graph_strings_per_s": n / t_graph,
           "graph_rounds": graph_rounds, "graph_nodes": nodes, "graph_status_ok": complete,
           "graph_replays_continued_host_driven": continued,
           "results_identical": bool(same_graph and same_job),
           "oracle_checked_sets": checked, "oracle_agrees": oracle_ok}
    del S, ws, pb, lb, pg, lg
    torch.cuda.empty_cache()
    return out


def kway_leg(ss, torch, synth, n=64_000_000, k=256, length=64, ratio=0.3, reps=3):
    """The k-way variant of the batched workload: k pre-sorted LCP-annotated
    front-coded runs of D/N strings (dealt to the runs at random), merged
    into one sequence by the LCP-aware merge, with full strings (d = length)
    and with distinguishing prefixes only (the PDMS form).  Inputs are built
    on the device from the D/N closed forms and resident before timing; the
    merged order and LCPs are checked against the same closed forms."""
    import numpy as np
    from tests import closed_forms as cf
    dev = torch.device("cuda:0")
    s = synth.dn_strings(n, length, ratio, seed=3, device=dev)
    run = synth.random_runs(n, k, 3, device=dev)
    K, F = s.meta["k"], s.meta["filler"]
    perm_ref = lcp_ref = None
    out = {"workload": f"{k} sorted front-coded runs, {n} D/N strings of {length} B (ratio {ratio}) dealt at random",
           "n": n, "k": k, "string_bytes": n * length}
    for pdms in (False, True):
        run_off, e, d, ids, suf_off, suf = cf.dn_front_coded_runs(s, run, k, pdms)
        rb, re_ = run_off[:-1].contiguous(), run_off[1:].contiguous()
        go = torch.tensor([0, k], dtype=torch.int32, device=dev)
        ws = torch.empty(ss.lib().ss_lcp_merge_workspace(n, n, k), dtype=torch.uint8, device=dev)
        lit = int(suf_off[-1])

        def merge():
            return ss.lcp_merge(rb, re_, go, e, d, ids, suf_off, suf, ws=ws, n_out=n, with_src=False)
        _, gid, glcp = merge()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            _, gid2, glcp2 = merge()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) / 1e3)
        same = torch.equal(gid, gid2) and torch.equal(glcp, glcp2)
        if perm_ref is None:
            perm_ref = cf.dn_perm(s.meta["pi"].numpy())
            lcp_ref = cf.dn_lcp(n, K, F)
        ok = bool(np.array_equal(gid.cpu().numpy().view(np.uint32), perm_ref)
                  and np.array_equal(glcp.cpu().numpy().view(np.uint32), lcp_ref))
        t = sorted(ts)[len(ts) // 2]
        # algorithmic bytes: e, d, id and suf_off (4+4+4+8 B) and the literal
        # bytes read once, id and LCP (4+4 B) written once
        alg = 28 * n + lit
        out["pdms" if pdms else "full_strings"] = {
            "ms": t * 1e3, "strings_per_s": n / t, "string_GBps": n * length / t / 1e9,
            "literal_bytes": lit, "front_coded_bytes_per_string": lit / n + 12.0,
            "algorithmic_GBps": alg / t / 1e9, "hbm_frac_algorithmic": alg / t / 1e9 / HBM_PEAK_GBS,
            "results_identical": bool(same), "closed_forms_agree": ok}
        del run_off, e, d, ids, suf_off, suf, ws, gid, glcp, gid2, glcp2
        torch.cuda.empty_cache()
    del s, run
    torch.cuda.empty_cache()
    return out


def splitters_leg(ss, torch, synth, n=50_000_000, p=16, v=2):
    """Text strings (log-normal lengths, Zipf bytes, 20% duplicates), split
    over p virtual PEs, each sorted: characters per bucket with string-based
    and with character-based regular sampling (v + 1 samples per PE, sorted,
    f_j = V[j|V|/p - 1]; Section 3.1), and with samples weighted by the
    approximate distinguishing prefixes (the characters PDMS sends)."""
    dev = torch.device("cuda:0")
    s = synth.text_strings(n, seed=0, device=dev)
    so = torch.tensor([n * i // p for i in range(p + 1)], dtype=torch.int64)
    perm, _ = ss.sort_batch(s.bytes, s.offsets, so.to(dev), with_lcp=False, global_ids=True)
    dpx, _ = ss.dist_prefix(s.bytes, s.offsets, 8, 64)
    lens = (s.offsets[1:] - s.offsets[:-1])
    pl = perm.to(torch.int64)
    C = {"len": torch.zeros(n + 1, dtype=torch.int64, device=dev), "dist": torch.zeros(n + 1, dtype=torch.int64,
                                                                                        device=dev)}
    C["len"][1:] = torch.cumsum(lens[pl], 0)
    C["dist"][1:] = torch.cumsum(dpx.to(torch.int64)[pl], 0)
    bl = so.tolist()
    out = {"workload": f"text strings n={n} (log-normal lengths median 40, Zipf 1.1 bytes, 20% duplicates)",
           "virtual_pes": p, "N": int(C["len"][-1]), "D_approx": int(C["dist"][-1]),
           "note": "largest bucket over the mean, in characters, in distinguishing-prefix characters and in "
                   "strings, for v + 1 samples per PE"}
    lmax = int(lens.max())
    for vv in (v, 64):
        res = {}
        for kind in ("strings", "chars", "chars_by_dist"):
            if kind == "strings":
                samp = ss.select_splitters_batch(perm, so, vv + 2)
            else:
                samp = ss.select_splitters_chars_batch(perm, s.offsets, so, vv + 2,
                                                       weights=dpx if kind == "chars_by_dist" else None)
            sb, sof = ss.gather_strings(s.bytes, s.offsets, samp)
            sperm, _ = ss.sort(sb, sof, with_lcp=False)
            fid = ss.select_splitters(sperm, p)
            fb, fo = ss.gather_strings(sb, sof, fid)
            cnt = {"len": torch.zeros(p, dtype=torch.int64, device=dev),
                   "dist": torch.zeros(p, dtype=torch.int64, device=dev)}
            strs = torch.zeros(p, dtype=torch.int64, device=dev)
            for a, e in zip(bl[:-1], bl[1:]):
                bb = ss.bucket_bounds(s.bytes, s.offsets, perm[a:e], fb, fo) + a
                strs += bb[1:] - bb[:-1]
                for key in cnt:
                    cnt[key] += C[key][bb[1:]] - C[key][bb[:-1]]
            res[kind] = {"chars": float(cnt["len"].max()) / (out["N"] / p),
                         "dist_chars": float(cnt["dist"].max()) / (out["D_approx"] / p),
                         "strings": float(strs.max()) / (n / p)}
        res["appendix_A_char_bound"] = ((1 + p / vv) * out["N"] / p + (1 + (vv + 1) / p) * p * lmax) / (out["N"] / p)
        out[f"v={vv}"] = res
    del s, perm, dpx, C
    torch.cuda.empty_cache()
    return out


def text_step_leg(ss, torch, synth, n=50_000_000, p=16, v=2, steps=3, warmup=1):
    """The same PDMS step on variable-length text strings (log-normal lengths,
    median 40; Zipf 1.1 bytes over 96 printable codes; 20% exact duplicates),
    p virtual PEs, prefix doubling from 8 bytes with 64-bit keys: time per
    step (two streams, as the main step), string bytes and strings per
    second, the stages on one stream, and whether every timed step gave the
    same order, LCPs and distinguishing prefixes."""
    import time as _time
    dev = torch.device("cuda:0")
    s = synth.text_strings(n, seed=0, device=dev)
    N = int(s.offsets[-1])
    pipe = Pipeline(s.bytes, s.offsets, p, v, ss, torch, overlap=True)
    times, ref, same = [], None, True
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = _time.perf_counter()
        order, mlcp, dist, dpx, rounds = pipe.step(Marks(torch, False))
        torch.cuda.synchronize()
        dt = _time.perf_counter() - t0
        if it >= warmup:
            times.append(dt)
        if ref is None:
            ref = (order.clone(), mlcp.clone(), dist.clone())
        else:
            same = same and torch.equal(order, ref[0]) and torch.equal(mlcp, ref[1]) and torch.equal(dist, ref[2])
        del order, mlcp, dist, dpx
    pipe.overlap = False
    m = Marks(torch, True)
    pipe.step(m)
    torch.cuda.synchronize()
    stages = m.times()
    stages.pop("start", None)
    t = sorted(times)[len(times) // 2]
    out = {"workload": f"text strings n={n} (log-normal lengths median 40 in [1, 4096], Zipf 1.1 bytes over 96 "
                       f"codes, 20% duplicates), p={p}, v={v}, prefix doubling from 8 bytes, 64-bit keys",
           "n": n, "N": N, "steps": steps, "ms_per_step": t * 1e3, "GBps": N / t / 1e9, "strings_per_s": n / t,
           "hbm_frac_of_N_per_step": N / t / 1e9 / HBM_PEAK_GBS, "doubling_rounds": int(rounds),
           "stages_ms_one_stream": stages, "results_identical": bool(same)}
    del s, pipe, ref
    torch.cuda.empty_cache()
    return out


def suffix_leg(ss, torch, synth, N=100_000_000, reps=3):
    """Suffix array + LCP array of one text (the bytes of text-like strings:
    Zipf-distributed printable characters with repeats), by prefix doubling
    over equal-length rank-pair strings sorted with the library's sort."""
    import numpy as np
    import oracle
    dev = torch.device("cuda:0")
    s = synth.text_strings(N // 60, seed=3, device=dev)
    text = s.bytes[:N].contiguous()
    del s
    ws = torch.empty(ss.lib().ss_suffix_sort_workspace(text.numel()), dtype=torch.uint8, device=dev)
    sa, lcp, steps = ss.suffix_sort(text, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sa, lcp, steps = ss.suffix_sort(text, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # verified pair by pair by the oracle's linear-time check
    ok = oracle.check_suffixes(text.cpu().numpy(), sa.cpu().numpy().view(np.uint32),
                               lcp.cpu().numpy().view(np.uint32)) == -1
    n = text.numel()
    out = {"text": f"{n} bytes of text-like strings (Zipf 1.1 over 96 codes, 20% repeated strings)",
           "ms": dt * 1e3, "suffixes_per_s": n / dt, "text_GBps": n / dt / 1e9, "doubling_steps": steps,
           "verified": bool(ok)}
    del text, ws, sa, lcp
    torch.cuda.empty_cache()
    return out


def serve_leg(ss, torch, synth, count=200, lo=1e3, hi=1e7, budget_gb=200.0, tight_gb=4.0, slots=4, load=0.7):
    """Sort requests (sort + LCP + exact and approximate distinguishing
    prefixes) served with continuous batching (`slots` concurrent streams,
    HBM-budget admission, results held on the device until the client takes
    them) against one job at a time, at equal output: throughput with every
    request queued at once (with the stated budget, and with a tight one that
    makes admission wait), and latency of a Poisson trace offered at `load` x
    the one-at-a-time capacity (both servers replay the same trace).  Every
    served result must equal the job run alone."""
    from paper_2404_16517_amd import serve
    dev = torch.device("cuda:0")
    reqs = synth.poisson_requests(count, qps=1.0, size_lo=lo, size_hi=hi, seed=7)
    inputs = {r.rid: synth.request_strings(r, device=dev) for r in reqs}
    torch.cuda.synchronize()
    budget = int(budget_gb * 1e9)
    serve.serve_sequential(reqs[:4], inputs)  # warm-up
    alone, t_seq = serve.serve_sequential(reqs, inputs)
    capacity = count / t_seq
    mismatch = []

    def check(job):
        if not all(torch.equal(a, b) for a, b in zip(job.result, alone[job.rid])):
            mismatch.append(job.rid)
    # saturation: all requests waiting at t = 0
    jobs_sat, span_sat = serve.serve_trace(reqs, inputs, budget, slots=slots, time_scale=0.0, on_done=check)
    _, span_one = serve.serve_trace(reqs, inputs, budget, slots=1, time_scale=0.0)
    largest = max(serve.job_bytes(x.n, x.N)[0] for x in inputs.values())
    tight = max(int(tight_gb * 1e9), largest)
    jobs_tight, span_tight = serve.serve_trace(reqs, inputs, tight, slots=slots, time_scale=0.0, on_done=check)
    waited = sum(1 for j in jobs_tight if j.admitted_s > 1e-3)
    # latency at a fixed offered load
    scale = 1.0 / (capacity * load)
    jobs, makespan = serve.serve_trace(reqs, inputs, budget, slots=slots, time_scale=scale, on_done=check)
    jobs1, _ = serve.serve_trace(reqs, inputs, budget, slots=1, time_scale=scale)
    lat = [j.done_s - j.arrival_s for j in jobs]
    lat1 = [j.done_s - j.arrival_s for j in jobs1]
    total_bytes = sum(x.N for x in inputs.values())
    total_strings = sum(x.n for x in inputs.values())
    out = {"requests": count, "sizes": f"log-uniform [{lo:.0f}, {hi:.0f}] strings", "strings": total_strings,
           "bytes": total_bytes, "slots": slots, "budget_GB": budget_gb,
           "saturated_jobs_per_s": count / span_sat, "one_at_a_time_jobs_per_s": count / span_one,
           "saturated_speedup": span_one / span_sat, "saturated_GBps": total_bytes / span_sat / 1e9,
           "tight_budget_GB": tight / 1e9, "tight_jobs_per_s": count / span_tight,
           "tight_requests_that_waited": waited,
           "offered_qps": capacity * load,
           "p50_ms": serve.percentile(lat, 0.5) * 1e3, "p99_ms": serve.percentile(lat, 0.99) * 1e3,
           "one_at_a_time_p50_ms": serve.percentile(lat1, 0.5) * 1e3,
           "one_at_a_time_p99_ms": serve.percentile(lat1, 0.99) * 1e3,
           "results_identical": not mismatch}
    del inputs, alone, jobs_sat, jobs_tight, jobs, jobs1
    torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s_host, p, v, target_s=10.0, threads=1):
    """The CPU oracle running the same step on a bounded prefix of the input.
    With threads > 1 the independent parts run concurrently (the per-PE sorts,
    bucket encodings and per-bucket merges; the oracle's C calls release the
    GIL); prefix doubling and the final LCP pass stay single-threaded, as the
    oracle has them."""
    import numpy as np
    import oracle
    b_all, o_all = oracle.strings_np(s_host)
    pool = concurrent.futures.ThreadPoolExecutor(max_workers=threads) if threads > 1 else None
    pmap = (lambda f, xs: list(pool.map(f, xs))) if pool else (lambda f, xs: [f(x) for x in xs])

    def run(ns):
        o = o_all[:ns + 1].copy()
        b = b_all[:int(o[-1])]
        bounds = [ns * i // p for i in range(p + 1)]
        t0 = time.perf_counter()
        dpx, _, _ = oracle.dist_prefix(b, o, 8, 64)

        def sort_pe(ae):
            a, e = ae
            so = o[a:e + 1] - o[a]
            sb = b[int(o[a]):int(o[e])]
            pl = oracle.sort(sb, so)
            return pl.astype(np.uint32) + np.uint32(a), oracle.lcp(sb, so, pl)
        res = pmap(sort_pe, list(zip(bounds[:-1], bounds[1:])))
        perms = [r[0] for r in res]
        lcps = [r[1] for r in res]
        samp = np.concatenate([oracle.select_splitters(len(pm), pm, v + 2) for pm in perms])
        strs = [bytes(b[int(o[i]):int(o[i + 1])]) for i in samp]
        sl = np.cumsum([0] + [len(x) for x in strs]).astype(np.uint64)
        sbytes = np.frombuffer(b"".join(strs) or b"\0", np.uint8)
        sperm = oracle.sort(sbytes, sl)
        fid = oracle.select_splitters(len(samp), sperm, p)
        spl = [strs[i] for i in fid]
        fl = np.cumsum([0] + [len(x) for x in spl]).astype(np.uint64)
        fbytes = np.frombuffer(b"".join(spl) or b"\0", np.uint8)

        def encode_pe(pl):
            pm, lc = pl
            bb = oracle.bucket_bounds(b, o, pm, fbytes, fl)
            return bb, oracle.fc_encode(b, o, pm, lc, dpx, bb)
        encs = pmap(encode_pe, list(zip(perms, lcps)))

        def merge_bucket(j):
            ro, LC, LN, ID, SO, SUF, base = [0], [], [], [], [], [], 0
            for bb, enc in encs:
                x, y = int(bb[j]), int(bb[j + 1])
                LC.append(enc["lcp"][x:y]); LN.append(enc["len"][x:y]); ID.append(enc["id"][x:y])
                SO.append(enc["suf_off"][x:y] - enc["suf_off"][x] + base)
                SUF.append(enc["suf"][int(enc["suf_off"][x]):int(enc["suf_off"][y])])
                base += int(enc["suf_off"][y] - enc["suf_off"][x])
                ro.append(ro[-1] + y - x)
            if not ro[-1]:
                return np.zeros(0, np.uint32)
            _, ids, _ = oracle.merge(np.array(ro, np.uint64), np.concatenate(LC), np.concatenate(LN),
                                     np.concatenate(ID), np.concatenate(SO + [np.array([base], np.uint64)]),
                                     np.concatenate(SUF))
            return ids
        order = np.concatenate(pmap(merge_bucket, list(range(p))))
        full_lcp = oracle.lcp(b, o, order)
        oracle.dist_exact(o, order, full_lcp)
        return time.perf_counter() - t0, int(o[-1])

    ns = 20_000
    dt, nbytes = run(ns)
    while dt < target_s / 4 and ns < s_host.n:
        ns = min(s_host.n, int(ns * min(8.0, max(1.5, target_s / max(dt, 1e-3) * 0.8))))
        dt, nbytes = run(ns)
    if pool:
        pool.shutdown()
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"first {ns} strings ({nbytes} bytes) of the same workload, same step with p={p}, "
                      f"C oracle on {threads} thread(s), {dt:.1f} s; host: {ncpu} CPUs available, {_cpu_model()}"}


# Kernel -> the source files its code comes from (for the staleness check of
# committed counter summaries).
KERNEL_SOURCES = {
    "k_hash_round": ["paper_2404_16517_amd/csrc/hash.hip", "paper_2404_16517_amd/csrc/common.hpp"],
    "k_hash_first": ["paper_2404_16517_amd/csrc/hash.hip", "paper_2404_16517_amd/csrc/common.hpp"],
    "k_hash_first_deep": ["paper_2404_16517_amd/csrc/hash.hip", "paper_2404_16517_amd/csrc/common.hpp"],
    "k_hash_first_lazy": ["paper_2404_16517_amd/csrc/hash.hip", "paper_2404_16517_amd/csrc/common.hpp"],
    "k_skip": ["paper_2404_16517_amd/csrc/sort.hip", "paper_2404_16517_amd/csrc/common.hpp"],
}
DEFAULT_WORKLOAD = dict(n=16_000_000, length=500, ratio=0.5, pes=16, sampling=2)


def sources_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(kernel, args):
    """HBM bytes per launch of `kernel` from its committed counter summary
    (profiles/<kernel>_dn16M_traffic.txt), or None when there is none, the
    workload is not the default one, or the kernel's sources changed since."""
    if any(getattr(args, k) != v for k, v in DEFAULT_WORKLOAD.items()) or kernel not in KERNEL_SOURCES:
        return None
    path = os.path.join(ROOT, "profiles", f"{kernel}_dn16M_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = per = None
    with open(path) as f:
        for line in f:
            if line.startswith("# sources sha256 "):
                digest = line.split()[3]
            elif line.startswith("traffic_per_launch_bytes "):
                per = float(line.split()[1])
    if digest is None or per is None or digest != sources_digest(KERNEL_SOURCES[kernel]):
        return None
    return per


PASS_SOURCES = {"sort+lcp": ["paper_2404_16517_amd/csrc/sort.hip", "paper_2404_16517_amd/csrc/sort_core.hpp",
                             "paper_2404_16517_amd/csrc/util.hip", "paper_2404_16517_amd/csrc/common.hpp"]}


def committed_pass_traffic(name, args):
    """Counter-measured HBM bytes of a whole pass (every dispatch of it) and
    the pass's kernel-trace time, from its committed summary
    (profiles/pass_sort_lcp_dn16M_traffic.txt), while its sources match."""
    if any(getattr(args, k) != v for k, v in DEFAULT_WORKLOAD.items()) or name not in PASS_SOURCES:
        return None
    path = os.path.join(ROOT, "profiles", "pass_%s_dn16M_traffic.txt" % name.replace("+", "_"))
    if not os.path.exists(path):
        return None
    digest = per = span = None
    with open(path) as f:
        for line in f:
            if line.startswith("# sources sha256 "):
                digest = line.split()[3]
            elif line.startswith("pass_traffic_bytes "):
                per = float(line.split()[1])
            elif line.startswith("pass_span_ms "):
                span = float(line.split()[1])
    if digest is None or per is None or digest != sources_digest(PASS_SOURCES[name]):
        return None
    return {"bytes": per, "span_ms": span, "achieved_GBps": per / (span / 1e3) / 1e9 if span else None,
            "frac": per / (span / 1e3) / 1e9 / HBM_PEAK_GBS if span else None}


def pass_rooflines(stage_ms, n, D, D_approx, active_sum, literal, seeded=False, D_beyond=0):
    """Per-pass achieved bandwidth with each pass's algorithmic bytes: what the
    pass must move, independent of how the kernels do it --
      sort+LCP          D + 16n (each distinguishing prefix read once, offsets
                        8 B, perm and LCP written 4 + 4 B per string);
      dist_prefix       D_approx + 16 sum_t |A_t| (every round's key written
                        and read) + 12n (offsets, result);
      partition_encode  32n + 2 sum(d - e) (metadata in and out, every
                        literal byte read and written once);
      lcp_merge         28n + sum(d - e) (front-coded metadata and literals
                        in, order and LCP out).
    Seeded (the first hash pass reads every string's first 256 bytes for
    both passes and writes the sort's 16-byte seed record): dist_prefix adds
    16n and spans its first pass and its rounds; sort+LCP is D_beyond (the
    distinguishing-prefix bytes past the first 256 of each string) + 24n
    (seed records in, perm and LCP out)."""
    def entry(ms, by):
        gbs = by / (ms / 1e3) / 1e9 if ms and ms > 0 else None
        return {"ms": ms, "algorithmic_bytes": by, "achieved_GBps": gbs,
                "frac": gbs / HBM_PEAK_GBS if gbs else None}
    if seeded:
        dp = [stage_ms.get("dist_prefix first pass"), stage_ms.get("dist_prefix rounds")]
        dp_ms = sum(dp) if None not in dp else None
        return {"sort+lcp": entry(stage_ms.get("sort_batch+lcp"), D_beyond + 24 * n),
                "dist_prefix": entry(dp_ms, D_approx + 16 * active_sum + 28 * n),
                "partition_encode": entry(stage_ms.get("partition_encode"), 32 * n + 2 * literal),
                "lcp_merge": entry(stage_ms.get("lcp_merge"), 28 * n + literal)}
    return {"sort+lcp": entry(stage_ms.get("sort_batch+lcp"), D + 16 * n),
            "dist_prefix": entry(stage_ms.get("dist_prefix"), D_approx + 16 * active_sum + 12 * n),
            "partition_encode": entry(stage_ms.get("partition_encode"), 32 * n + 2 * literal),
            "lcp_merge": entry(stage_ms.get("lcp_merge"), 28 * n + literal)}


def doubling_active_sum(dpx, l0=8):
    """sum over rounds of the active strings: a string with approximate
    distinguishing prefix d took part in every round up to the first whose
    length l0 * 2^(t-1) reaches d (Section 4's finish rule)."""
    import numpy as np
    d = dpx.cpu().numpy().view(np.uint32).astype(np.int64)
    t = np.ones_like(d)
    L = np.full_like(d, l0)
    while True:
        m = d > L
        if not m.any():
            break
        t[m] += 1
        L[m] *= 2
    return int(t.sum())


def roofline(prof, steps, args):
    """Roofline object of the kernel with the largest event time."""
    name = max(prof, key=lambda k: prof[k][0])
    ms, by, cnt = prof[name]
    achieved = by / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": committed_traffic(name, args),
            "kernel": name, "launches_per_step": cnt / steps, "avg_launch_ms": ms / max(cnt, 1),
            "algorithmic_bytes_per_launch": by / max(cnt, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16_000_000)
    ap.add_argument("--length", type=int, default=500)
    ap.add_argument("--ratio", type=float, default=0.5)
    ap.add_argument("--pes", type=int, default=16, help="virtual processing elements")
    ap.add_argument("--sampling", type=int, default=2, help="sampling factor v")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--stages", action="store_true", help="per-stage times on stderr")
    ap.add_argument("--no-one-stream", action="store_true",
                    help="skip the one-stream steps after the timed ones (roofline_one_stream)")
    ap.add_argument("--serial", action="store_true",
                    help="run prefix doubling before the sort on one stream (by default it runs on a second "
                         "stream beside the sort, and per-kernel times include the other stream's kernels)")
    ap.add_argument("--dedup", choices=["table", "buckets"], default="table",
                    help="prefix doubling's duplicate detection (library tuning SS_TUNE_DEDUP)")
    ap.add_argument("--no-seed", action="store_true",
                    help="the sort reads every string's first bytes itself, beside all of prefix doubling "
                         "(by default prefix doubling's first pass reads them once for both and the sort "
                         "runs beside the later rounds)")
    ap.add_argument("--first-pass-alone", action="store_true",
                    help="run prefix doubling's first pass before the sort, only its later rounds beside it")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-per-job leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-kway", action="store_true", help="skip the k-way merge of 256 front-coded runs")
    ap.add_argument("--no-ms-mode", action="store_true", help="skip the full-string (MS) step")
    ap.add_argument("--no-suffix", action="store_true", help="skip the suffix-sorting leg")
    ap.add_argument("--no-text-step", action="store_true", help="skip the PDMS step on 50M text strings")
    ap.add_argument("--no-splitters", action="store_true",
                    help="skip the string- vs character-based splitter comparison on text strings")
    ap.add_argument("--no-profile", action="store_true",
                    help="time the steps without the per-launch events (no roofline)")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GB",
                    help="only run a plain device-to-device copy of this many GB (counter calibration)")
    ap.add_argument("--kway-only", action="store_true",
                    help="only run the k-way merge leg and print its results (for profiling it alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (use --gpus 1); the multi-GPU design is described, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2404_16517_amd as ss
    import synth

    from paper_2404_16517_amd import autotune
    tuned = autotune.apply("dn")
    ss.set_tuning(ss.SS_TUNE_DEDUP, {"table": 0, "buckets": 1}[args.dedup])
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        nbytes = int(args.calibrate_copy * 1e9) // 16 * 16
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}))
        return
    if args.kway_only:
        print(json.dumps({"kway_merge": kway_leg(ss, torch, synth)}))
        return
    t0 = time.time()
    s = synth.dn_strings(args.n, args.length, args.ratio, seed=0, device=dev)
    torch.cuda.synchronize()
    print(f"# generated n={s.n} N={s.N} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    pipe = Pipeline(s.bytes, s.offsets, args.pes, args.sampling, ss, torch, overlap=not args.serial,
                    first_alone=args.first_pass_alone, seeded=not args.no_seed)

    # (the warm-up steps also fill the library's pool of profiling events; the
    # last one, with every kernel timed, names the kernel with the largest
    # event time, and the timed steps record events around that kernel only,
    # so that the other kernels' events cost no host time in the timed region)
    wprof = {}
    for w in range(args.warmup):
        ss.profile_enable(not args.no_profile)
        pipe.step(Marks(torch, False))
        torch.cuda.synchronize()
    if args.warmup and not args.no_profile:
        wprof = ss.profile_report()
    dominant = max(wprof, key=lambda k: wprof[k][0]) if wprof else None  # (none: all kernels timed)
    ss.profile_only(dominant)
    stages = {}
    ss.profile_enable(not args.no_profile)  # HIP events around the dominant kernel in the timed steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mk = Marks(torch, args.stages)
        res = pipe.step(mk)
        if args.stages:
            torch.cuda.synchronize()
            for k, v in mk.times().items():
                stages.setdefault(k, []).append(v)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = ss.profile_report()
    ss.profile_enable(False)
    ss.profile_only(None)
    order, mlcp, dist, dpx, rounds = res
    print(f"# step {dt * 1e3:.3f} ms", file=sys.stderr, flush=True)
    verified = None
    if not args.no_verify:
        verified = verify_dn(s, order, mlcp, dist, dpx)
        print(f"# verified against the closed forms: {verified}", file=sys.stderr, flush=True)
    out = {
        "metric": "string bytes sorted/s",
        "value": s.N / dt / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"D/N-ratio strings n={s.n} len={args.length} D/N={args.ratio}",
                   "n": s.n, "N": s.N, "virtual_pes": args.pes, "sampling_factor": args.sampling,
                   "doubling_rounds": rounds, "streams": 1 if args.serial else 2,
                   "first_pass_alone": (not args.serial) and args.first_pass_alone,
                   "seeded": not args.no_seed,
                   "dedup": args.dedup,
                   "tuning": tuned or "library defaults"},
        "strings_per_s": s.n / dt,
        "hbm_frac_of_N_per_step": s.N / dt / 1e9 / HBM_PEAK_GBS,
        "verified": verified,
    }
    if prof:
        out["roofline"] = roofline(prof, args.steps, args)
        # every kernel's event time in the last warm-up step (two streams)
        kp, ks = (wprof, 1) if wprof else (prof, args.steps)
        out["kernels_ms_per_step"] = {k: v[0] / ks for k, v in sorted(kp.items(), key=lambda x: -x[1][0])}
        # each kernel's own bytes (its reads and writes as implemented, e.g.
        # 40 B per element per merge level), not the pass formulas
        out["kernels_impl_gbs"] = {k: (v[1] / (v[0] / 1e3) / 1e9 if v[0] > 0 else None) for k, v in kp.items()}
        if pipe.overlap and not args.no_one_stream:
            # The same kernels with the step on one stream (a few extra steps
            # after the timed ones): each kernel's time without the other
            # stream's kernels beside it.
            pipe.overlap = False
            pipe.step(Marks(torch, False))
            torch.cuda.synchronize()
            ss.profile_enable(True)
            serial_steps = 3
            sstages = {}
            for _ in range(serial_steps):
                mk = Marks(torch, True)
                res1 = pipe.step(mk)
                torch.cuda.synchronize()
                for k, v in mk.times().items():
                    sstages.setdefault(k, []).append(v)
            torch.cuda.synchronize()
            sprof = ss.profile_report()
            ss.profile_enable(False)
            pipe.overlap = True
            out["roofline_one_stream"] = roofline(sprof, serial_steps, args)
            out["kernels_ms_per_step_one_stream"] = {k: v[0] / serial_steps for k, v in
                                                     sorted(sprof.items(), key=lambda x: -x[1][0])}
            stage_ms = {k: sorted(v)[len(v) // 2] for k, v in sstages.items()}
            _, _, dist1, dpx1, _ = res1
            D = int(dist1.to(torch.int64).sum())
            Dx = int(dpx1.to(torch.int64).sum())
            Db = int((dist1.to(torch.int64) - 256).clamp_(min=0).sum())
            out["roofline"]["passes"] = pass_rooflines(stage_ms, s.n, D, Dx, doubling_active_sum(dpx1),
                                                       pipe.literal_bytes, seeded=pipe.seeded, D_beyond=Db)
            # what the counters saw the whole pass move (every dispatch), against its traced time
            out["roofline"]["passes"]["sort+lcp"]["counter_traffic"] = committed_pass_traffic("sort+lcp", args)
            out["roofline"]["passes_note"] = ("one-stream steps, median stage time (events on the stream), "
                                              "algorithmic bytes per pass; D = %d, D_approx = %d" % (D, Dx))
            out["stages_ms_one_stream"] = stage_ms
    if args.stages:
        out["stages_ms"] = {k: sum(v) / len(v) for k, v in stages.items()}
    if not args.no_ms_mode:
        # the paper's MS beside PDMS: the same step on full strings (no prefix
        # doubling), and the front-coded bytes each mode moves per string
        out["front_coded_bytes_per_string"] = {"pdms": pipe.literal_bytes / s.n + 12.0}
        pipe.overlap, was = False, pipe.overlap
        pipe.ms_mode = True
        pipe.step(Marks(torch, False))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            pipe.step(Marks(torch, False))
        torch.cuda.synchronize()
        ms_dt = (time.perf_counter() - t0) / 3
        out["front_coded_bytes_per_string"]["ms"] = pipe.literal_bytes / s.n + 12.0
        out["front_coded_bytes_per_string"]["note"] = "literal bytes / n + 12 B of metadata (e, d, id)"
        out["ms_mode"] = {"ms_per_step": ms_dt * 1e3, "GBps": s.N / ms_dt / 1e9,
                          "note": "one stream, full strings front-coded and merged (no prefix doubling)"}
        pipe.ms_mode = False
        pipe.overlap = was
    if not args.no_batch:
        used = autotune.apply("sets")
        out["batch"] = batch_leg(ss, torch, synth)
        out["batch"]["tuning"] = used or "library defaults"
        autotune.apply("dn")
        print(f"# batch leg: {out['batch']}", file=sys.stderr, flush=True)
    if not args.no_kway:
        out["kway_merge"] = kway_leg(ss, torch, synth)
        print(f"# k-way merge leg: {out['kway_merge']}", file=sys.stderr, flush=True)
    if not args.no_splitters:
        autotune.apply("text")
        out["splitters_text"] = splitters_leg(ss, torch, synth)
        autotune.apply("dn")
        print(f"# splitters leg: {out['splitters_text']}", file=sys.stderr, flush=True)
    if not args.no_text_step:
        autotune.apply("text")
        out["text_step"] = text_step_leg(ss, torch, synth)
        autotune.apply("dn")
        print(f"# text step leg: {out['text_step']}", file=sys.stderr, flush=True)
    if not args.no_suffix:
        out["suffix_sort"] = suffix_leg(ss, torch, synth)
        print(f"# suffix leg: {out['suffix_sort']}", file=sys.stderr, flush=True)
    if not args.no_serve:
        out["serve"] = serve_leg(ss, torch, synth)
        print(f"# serve leg: {out['serve']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        host = synth.StringSet(s.bytes[: int(s.offsets[min(s.n, 4_000_000)])].cpu(),
                               s.offsets[: min(s.n, 4_000_000) + 1].cpu(), dict(s.meta))
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = max(1, min(args.pes, 16, ncpu))
        out["cpu_baseline"] = cpu_baseline(host, args.pes, args.sampling, threads=threads)
        out["cpu_baseline_single_thread"] = cpu_baseline(host, args.pes, args.sampling, threads=1)
        print(f"# cpu baselines: {out['cpu_baseline']} / {out['cpu_baseline_single_thread']}", file=sys.stderr,
              flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
