"""Benchmark of the one-GPU string-sorting hot path (prints ONE JSON line).

Workload (default): 16,000,000 strings x 500 bytes over 'A'..'Z' with D/N ratio
0.5 (the paper's DNData shape; N = 8.0 GB), resident in HBM.

One step = the whole hot path over that input:
  sort + LCP array -> exact distinguishing prefixes -> prefix doubling
  (hash rounds + duplicate detection) -> r = 256 splitters, bucket bounds and
  front coding of the distinguishing prefixes -> LCP-aware merge of the r
  front-coded runs back into one sorted order.
value = N / (seconds per step) in GB/s ("string bytes sorted per second").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16_000_000)
    ap.add_argument("--length", type=int, default=500)
    ap.add_argument("--ratio", type=float, default=0.5)
    ap.add_argument("--buckets", type=int, default=256)
    ap.add_argument("--stages", action="store_true", help="print per-stage times to stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2404_16517_amd as ss
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    s = synth.dn_strings(args.n, args.length, args.ratio, seed=0, device=dev)
    torch.cuda.synchronize()
    print(f"# generated n={s.n} N={s.N} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    B, O = s.bytes, s.offsets
    n, N = s.n, s.N

    ws_sort = torch.empty(ss.lib().ss_sort_workspace(n), dtype=torch.uint8, device=dev)
    ws_pd = torch.empty(ss.lib().ss_dist_prefix_workspace(n), dtype=torch.uint8, device=dev)
    stages = {}

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def step(record):
        marks = [("start", ev())]
        perm, lcp = ss.sort(B, O, ws=ws_sort)
        marks.append(("sort+lcp", ev()))
        dist = ss.dist_exact(O, perm, lcp)
        marks.append(("dist_exact", ev()))
        dpx, rounds = ss.dist_prefix(B, O, 8, 64, ws=ws_pd)
        marks.append(("dist_prefix", ev()))
        ids = ss.select_splitters(perm, args.buckets)
        sb, so = ss.gather_strings(B, O, ids)
        fc = ss.partition_encode(B, O, perm, lcp, dpx, sb, so)
        marks.append(("partition_encode", ev()))
        src, mid, mlcp = ss.lcp_merge(fc["run_off"], fc["lcp"], fc["len"], fc["id"], fc["suf_off"], fc["suf"])
        marks.append(("lcp_merge", ev()))
        torch.cuda.synchronize()
        if record:
            for (a, ea), (b, eb) in zip(marks[:-1], marks[1:]):
                stages.setdefault(b, []).append(ea.elapsed_time(eb))
        return rounds, fc["total"]

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rounds, lit = step(True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    if args.stages:
        for k, v in stages.items():
            print(f"# stage {k:18s} {sum(v) / len(v):9.3f} ms", file=sys.stderr)
    out = {
        "metric": "string bytes sorted/s",
        "value": N / dt / 1e9,
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
        "config": {"workload": f"dn n={n} len={args.length} D/N={args.ratio}", "n": n, "N": N,
                   "buckets": args.buckets, "doubling_rounds": rounds, "literal_bytes": lit},
        "strings_per_s": n / dt,
        "stages_ms": {k: sum(v) / len(v) for k, v in stages.items()},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
