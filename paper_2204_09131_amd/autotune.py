"""Autotuner of the main kernel's work-list and scheduling choices (its tile
shapes), per window-size bucket, on the device it runs on.

    python -m paper_2204_09131_amd.autotune [--runs N] [--out PATH]

The choices (``wmi_tuning`` in include/wmi.h): windows per local item and
triples per triple item by the largest window of the item, windows per sweep
item by window size (1: runs of equally spaced windows evaluated window by
window instead of one from the other), and the straggler threshold of
windows scanned in x order by window size.  For every choice and bucket the tuner builds a
synthetic workload of that bucket (the multi-scale segment recipe: linear,
quadratic, sine and independent links), times the main kernel (HIP events,
mean over the last runs) for every candidate value with the other choices at
their defaults, and keeps the fastest; a candidate must beat the default by
more than 2% to replace it.  Every candidate has to give bit-identical
results -- all are schedules of the same exact arithmetic, so a difference
would expose a race -- or the tuner stops.  The choices, with every timing
behind them, are written as JSON keyed by the device's architecture
(``tuning/<arch>.json`` beside this file), which ``wmi.Store(tuning="auto")``
loads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_2204_09131_amd import synth, wmi  # noqa: E402

LOCAL_M = (32, 64, 128, 256)          # buckets 0..3 of local_windows (bucket 4 holds one window)
TRIPLE_U = (64, 128, 256, 512)        # union sizes, buckets 1..4 of triples
SWEEP_M = (64, 128, 240)              # sweep_windows buckets 0..2
SPLIT_M = (1024, 2048, 4096)          # stragglers buckets 0..2


def _bucket(m: int, tops) -> int:
    for i, t in enumerate(tops):
        if m <= t:
            return i
    return len(tops) - 1


def workloads(n: int = 1 << 19, seed: int = 91):
    """Queries per (choice, bucket), on one pair of n points (series 0, 1)."""
    out = {}
    for m in LOCAL_M:
        out[("local_windows", _bucket(m, (32, 64, 128, 256, 512)))] = (
            synth.make_queries(0, 1, synth.sliding(n, m, m // 8), m),
            [c for c in (1, 2, 4, 8, 16) if c * ((m + 1) & ~1) <= 512])
    for u in TRIPLE_U:
        d = u // 8
        starts = synth.sliding(n - d, u - d, d)
        out[("triples", _bucket(u, (32, 64, 128, 256, 512)))] = (
            synth.make_queries(0, 1, starts, u - d, d, +1), [c for c in (1, 2, 3, 4, 5) if c * u <= 512])
    for m in SWEEP_M:
        out[("sweep_windows", _bucket(m, (64, 128, 255)))] = (
            synth.make_queries(0, 1, np.arange(0, 16384, dtype=np.uint64), m), [1, 2, 4, 8, 16, 32, 64])
    for m in SPLIT_M:
        out[("stragglers", _bucket(m, (1024, 2048, 4096)))] = (
            synth.make_queries(0, 1, synth.sliding(n, m, m // 8), m), [0, 4, 8, 16, 32, 64])
    return out


def main_ms(st, q, runs: int, k: int = 4):
    b = st.submit(q, k=k, tau=0.05)
    res = b.read()
    for _ in range(runs):
        b.replay(direct=True)
    b.wait()
    t = b.timing()
    b.destroy()
    return t["main_ms"], res


def tune(runs: int = 16, log=print) -> dict:
    import torch
    x, y = synth.cfg2_pair(1 << 19, 91)
    st = wmi.Store(0)
    assert [st.add_series(x), st.add_series(y)] == [0, 1]
    chosen = {f: list(v) for f, v in st.get_tuning().items()}
    measured = {}
    for (field, b), (q, cands) in workloads().items():
        default = chosen[field][b]
        times, ref = {}, None
        for c in sorted(set(cands) | {default}):
            t = dict(chosen)
            t[field] = list(chosen[field])
            t[field][b] = c
            st.set_tuning(t)
            main_ms(st, q, 2)  # warm up
            ms, res = main_ms(st, q, runs)
            if ref is None:
                ref = res
            elif not np.array_equal(ref.view(np.uint8), res.view(np.uint8)):
                raise RuntimeError(f"{field}[{b}] = {c} changed results")
            times[c] = ms
        best = min(times, key=times.get)
        if times[best] < 0.98 * times[default]:
            chosen[field][b] = best
        measured[f"{field}[{b}]"] = {"windows": int(len(q)), "main_ms": {str(c): v for c, v in times.items()},
                                     "chosen": chosen[field][b], "default": default}
        log(f"{field}[{b}]: {len(q)} queries; " + ", ".join(f"{c}: {v:.3f} ms" for c, v in sorted(times.items()))
            + f" -> {chosen[field][b]}")
    st.close()
    props = torch.cuda.get_device_properties(0)
    return {"arch": props.gcnArchName.split(":")[0], "device": props.name,
            "compute_units": props.multi_processor_count, "k": 4, "runs": runs,
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "tuning": chosen, "measured": measured}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=16)
    ap.add_argument("--out", default=None, help="default: tuning/<arch>.json beside this file")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the autotuner needs a GPU"
    out = tune(args.runs, log=lambda s: print(s, flush=True))
    path = args.out or os.path.join(HERE, "tuning", f"{out['arch']}.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
