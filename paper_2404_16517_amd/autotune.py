"""Autotuner for the sort's launch parameters on the current GPU.

It times ``sort`` on sample workloads (D/N strings and text-like strings) for
every combination of the LDS cutover (segments up to this many strings are
sorted in LDS) and the radix tile (elements per workgroup in radix passes),
and writes the fastest combination to a JSON table.  ``apply()`` loads a table
and sets the library's tuning.  Results never depend on the tuning, only time.

    python -m paper_2404_16517_amd.autotune --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning.json")
SMALL_MAX = (256, 512, 1024)
TILES = (2048, 4096, 8192)


def apply(path: str | None = None) -> dict | None:
    """Set the tuning from a table written by ``autotune`` (if it exists)."""
    import paper_2404_16517_amd as ss
    path = path or DEFAULT_TABLE
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    ss.set_tuning(ss.SS_TUNE_SMALL_MAX, int(t["small_max"]))
    ss.set_tuning(ss.SS_TUNE_TILE, int(t["tile"]))
    return t


def autotune(n: int = 2_000_000, reps: int = 3, out: str | None = None) -> dict:
    import torch
    import paper_2404_16517_amd as ss
    import synth
    dev = torch.device("cuda:0")
    samples = {
        "dn": synth.dn_strings(n, 100, 0.5, seed=1, device=dev),
        "text": synth.text_strings(n, seed=1, device=dev),
    }
    ws = torch.empty(ss.lib().ss_sort_workspace(n), dtype=torch.uint8, device=dev)
    old_sm = ss.set_tuning(ss.SS_TUNE_SMALL_MAX, 1024)
    old_tile = ss.set_tuning(ss.SS_TUNE_TILE, 4096)
    timings = {}
    try:
        for sm in SMALL_MAX:
            for tile in TILES:
                ss.set_tuning(ss.SS_TUNE_SMALL_MAX, sm)
                ss.set_tuning(ss.SS_TUNE_TILE, tile)
                tot = 0.0
                for name, s in samples.items():
                    ss.sort(s.bytes, s.offsets, ws=ws)  # warm-up
                    torch.cuda.synchronize()
                    ts = []
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        ss.sort(s.bytes, s.offsets, ws=ws)
                        torch.cuda.synchronize()
                        ts.append(time.perf_counter() - t0)
                    tot += statistics.median(ts)
                timings[f"{sm},{tile}"] = tot * 1e3
    finally:
        ss.set_tuning(ss.SS_TUNE_SMALL_MAX, old_sm)
        ss.set_tuning(ss.SS_TUNE_TILE, old_tile)
    best = min(timings, key=timings.get)
    sm, tile = (int(x) for x in best.split(","))
    table = {"small_max": sm, "tile": tile, "sample_strings": n, "ms": timings,
             "device": torch.cuda.get_device_name(0)}
    if out:
        with open(out, "w") as f:
            json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    a = ap.parse_args()
    print(json.dumps(autotune(a.n, a.reps, a.out)))
