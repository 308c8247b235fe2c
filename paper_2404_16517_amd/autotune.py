"""Autotuner for the sort's launch parameters on the current GPU.

For each workload shape -- D/N strings (fixed length, long shared prefixes),
text-like strings (log-normal lengths, Zipf bytes, duplicates) and many
small independent sets -- it times the batched sort for every combination of
the radix digit width (8 or 11 bits), the radix tile (elements per workgroup
in a radix pass) and the LDS cutover (segments up to this many strings are
sorted in LDS or registers), and writes the fastest combination per workload
to a JSON table.  ``apply(workload)`` loads the table and sets that entry.
Results never depend on the tuning, only time.

    python -m paper_2404_16517_amd.autotune --out paper_2404_16517_amd/tuning.json
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
TILES = (2048, 4096, 8192, 16384)
DIGIT_BITS = (8, 11)
WORKLOADS = ("dn", "text", "sets")


def valid(sm: int, tile: int, bits: int) -> bool:
    """11-bit digits take effect only with tiles >= 4096 and a cutover >= 512."""
    return bits == 8 or (tile >= 4096 and sm >= 512)


def apply(workload: str = "dn", path: str | None = None) -> dict | None:
    """Set the tuning of `workload` from a table written by ``autotune`` (if
    it exists); returns the entry used, or None (library defaults)."""
    import paper_2404_16517_amd as ss
    path = path or DEFAULT_TABLE
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get("workloads", {}).get(workload)
    if e is None:
        return None
    ss.set_tuning(ss.SS_TUNE_SMALL_MAX, int(e["small_max"]))
    ss.set_tuning(ss.SS_TUNE_TILE, int(e["tile"]))
    ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, int(e["digit_bits"]))
    return {"workload": workload, "small_max": e["small_max"], "tile": e["tile"], "digit_bits": e["digit_bits"]}


def _samples(dev):
    """Samples shaped like the benchmark's uses: per-PE sets of 10^6 D/N
    strings (500 B, long shared prefixes) and of 10^6 text strings, and
    independent sets of 10^3..10^6 strings."""
    import synth
    return {
        "dn": synth.concat([synth.dn_strings(1_000_000, 500, 0.5, seed=s, device=dev) for s in range(4)]),
        "text": synth.concat([synth.text_strings(1_000_000, seed=s, device=dev) for s in range(4)]),
        "sets": synth.random_sets(96, 1e3, 1e6, 8, 256, seed=1, device=dev),
    }


def autotune(reps: int = 3, out: str | None = None) -> dict:
    import torch
    import paper_2404_16517_amd as ss
    dev = torch.device("cuda:0")
    samples = _samples(dev)
    old = (ss.set_tuning(ss.SS_TUNE_SMALL_MAX, 1024), ss.set_tuning(ss.SS_TUNE_TILE, 4096),
           ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, 8))
    table = {"device": torch.cuda.get_device_name(0), "reps": reps, "workloads": {}}
    try:
        for name, (s, bounds) in samples.items():
            so = bounds.to(dev)
            ws = torch.empty(ss.lib().ss_sort_workspace(s.n), dtype=torch.uint8, device=dev)
            timings = {}
            for bits in DIGIT_BITS:
                for sm in SMALL_MAX:
                    for tile in TILES:
                        if not valid(sm, tile, bits):
                            continue
                        ss.set_tuning(ss.SS_TUNE_SMALL_MAX, sm)
                        ss.set_tuning(ss.SS_TUNE_TILE, tile)
                        ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, bits)
                        ss.sort_batch(s.bytes, s.offsets, so, ws=ws)  # warm-up
                        torch.cuda.synchronize()
                        ts = []
                        for _ in range(reps):
                            t0 = time.perf_counter()
                            ss.sort_batch(s.bytes, s.offsets, so, ws=ws)
                            torch.cuda.synchronize()
                            ts.append(time.perf_counter() - t0)
                        timings[f"{bits},{sm},{tile}"] = statistics.median(ts) * 1e3
            best = min(timings, key=timings.get)
            bits, sm, tile = (int(x) for x in best.split(","))
            table["workloads"][name] = {"digit_bits": bits, "small_max": sm, "tile": tile, "ms": timings[best],
                                        "strings": s.n, "bytes": s.N, "ms_all": timings}
    finally:
        ss.set_tuning(ss.SS_TUNE_SMALL_MAX, old[0])
        ss.set_tuning(ss.SS_TUNE_TILE, old[1])
        ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, old[2])
    if out:
        with open(out, "w") as f:
            json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    a = ap.parse_args()
    print(json.dumps(autotune(a.reps, a.out)))
