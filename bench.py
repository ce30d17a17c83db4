"""Benchmark: windowed KSG MI over the multi-scale workload on one MI355X.

Workload (one step): one pair of float32 series, n = 65,536, on the 2^-12
grid, segments of linear / quadratic / sine / independent links with lengths
uniform in [256, 4096]; windows w in {32, 64, ..., 4096} with stride w/8, all
8 scales in one batch (32,584 windows, 4,117,467,936 ordered point pairs),
k = 4, Eq. (2) estimator.  Series are resident in HBM before timing starts.

A step = one run of the batch: descriptor upload, clear, prep kernel (sorted
marginals), persistent main kernel (neighbours, counts, digamma sums, MI),
result download.  Steps are enqueued back to back on one stream (pipelined),
with HIP events around each kernel; `value` is windows / (wall time / step).

Also reported: the same steps as HIP-graph launches, the plain form (one
prep + one main launch per window), end-to-end query latency (fresh submit ->
results on host), the roofline of the main kernel, the serving loop on 1024
resident series of 2^20 points under a Poisson request stream (p50/p99
latency, throughput), the all-pairs noise search (64 x 32,768, 2016 pairs,
8,195,040 noise triples) and the large-search hot path on one pair of 2^24
points (every top-down layer, 4,161,487 windows), and the CPU oracle on the
host's cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "window-MI evals/s and distance ops/s (% FP32 VALU peak); p50/p99 query latency"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz, one 32-bit VALU op per lane per clock
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
OPS_PER_PAIR = 8   # per ordered pair: 2 differences + max (distance), k-th test, 2 x (difference + compare)


# HBM traffic of main_kernel<4> per launch on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch), each scaled by what the
# same counter reads for an elementwise kernel of known traffic (256 MiB read,
# 256 MiB written): FETCH_SIZE x 1.9998, WRITE_SIZE x 1.0.  Valid only for the
# kernel source it was taken on (hash of the kernel and descriptor sources).
TRAFFIC = {"kernel_sha256": "72f4d7cb4ea5e1639cceedfe97c7b030240757839d1d1375b25d23a089fb73dd",
           "fetch_bytes": 78583189, "write_bytes": 46743756}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("wmi_kernels.hip", "wmi_internal.h"):
        with open(os.path.join(ROOT, "paper_2204_09131_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(workload, budget_s: float = 20.0) -> dict:
    """The oracle as it stands, on every host core, over a bounded sample."""
    import oracle
    orc = oracle.load()
    cores = orc.threads(len(os.sched_getaffinity(0)))
    q = workload.queries
    # a strided sample holding every scale; grown until it takes a few seconds
    step = 64
    t_used = 0.0
    while True:
        sub = q[::step]
        t0 = time.perf_counter()
        orc.batch(workload.series, sub, k=workload.k)
        dt = time.perf_counter() - t0
        t_used += dt
        if dt > 3.0 or step == 1 or t_used > budget_s:
            break
        step = max(1, step // 4)
    # whole passes over the sample until about 10 s of work
    reps = max(1, int(10.0 / max(dt, 1e-3)))
    if reps > 1:
        t0 = time.perf_counter()
        for _ in range(reps):
            orc.batch(workload.series, sub, k=workload.k)
        dt = (time.perf_counter() - t0) / reps
    return {"value": len(sub) / dt, "unit": "window-MI evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sub)} of {len(q)} windows (every {step}-th, all scales), "
                      f"{reps} pass(es) of {dt:.2f} s each",
            "pairs_per_s": float(np.sum(sub['len'].astype(np.float64) * (sub['len'] - 1.0))) / dt}


def serve_bench(args, torch, synth, wmi) -> dict:
    """Serving workload: 1024 resident series x 2^20 points (4 GiB, cfg2
    segment recipe, drawn on the device), a Poisson stream of range requests
    (random pair, w log-uniform in [32, 2048], stride w/4, whole series) at
    `rate` per second, continuous batching with arena admission.  Latency of a
    request = results on the host minus its scheduled arrival.  Then the same
    requests submitted at once (saturation throughput)."""
    import threading
    n_series, n = 1024, 1 << 20
    t_gen = time.perf_counter()
    data = synth.cfg2_pairs_device(n_series // 2, n, seed=4, device="cuda")
    torch.cuda.synchronize()
    log(f"serve: generated {n_series} x {n} series in {time.perf_counter() - t_gen:.1f} s")
    t, a, b, w, stride = synth.config4_stream(n_queries=args.serve_queries, n_series=n_series, n=n,
                                              rate=args.serve_rate)
    st = wmi.Store(0)
    ids = [st.add_series(data[i]) for i in range(n_series)]
    assert ids == list(range(n_series))
    pairs_of = w.astype(np.float64) * (w - 1) * ((n - w) // stride + 1)
    wins_of = ((n - w) // stride + 1).astype(np.float64)

    def run_stream(times, srv):
        tickets = [0] * len(times)
        sched = np.zeros(len(times))
        errors = []

        def producer():
            try:
                c0 = srv.clock_us()
                for i in range(len(times)):
                    due = c0 + times[i] * 1e6
                    while True:
                        now = srv.clock_us()
                        if now >= due:
                            break
                        time.sleep(min(0.002, (due - now) * 1e-6))
                    sched[i] = due
                    tickets[i] = srv.submit(int(a[i]), int(b[i]), 0, n, int(w[i]), int(stride[i]))
            except Exception as e:  # reported by the collector below
                errors.append(e)

        th = threading.Thread(target=producer)
        w0 = time.perf_counter()
        th.start()
        lat = np.zeros(len(times))
        done = 0
        while done < len(times):
            while tickets[done] == 0:
                if errors:
                    raise errors[0]
                time.sleep(0.0005)
            srv.wait(tickets[done], 600_000_000)
            if done % 1000 == 999:
                log(f"serve: {done + 1} of {len(times)} requests done")
            res, info = srv.read(tickets[done])
            if not np.all(np.isfinite(res["mi"])):
                raise RuntimeError(f"request {done}: non-finite MI")
            lat[done] = (info["t_complete_us"] - sched[done]) * 1e-3
            done += 1
        th.join()
        return lat, time.perf_counter() - w0

    out = {"workload": f"serving: {n_series} resident series x {n} float32 (cfg2 segment recipe), "
                       "Poisson range requests (random pair, w log-uniform 32..2048, stride w/4, whole series)",
           "k": 4}
    with wmi.Server(st, k=4) as srv:
        # warm up the scheduler and both launch slots
        lat_w, _ = run_stream(np.zeros(8), srv)
        q = args.serve_queries
        lat, wall = run_stream(t[:q], srv)
        stats = srv.stats()
    out["poisson"] = {"rate_qps": args.serve_rate, "queries": int(q), "wall_s": wall,
                      "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "max_ms": float(lat.max()), "throughput_qps": q / wall,
                      "windows_per_s": float(wins_of[:q].sum() / wall),
                      "pairs_per_s": float(pairs_of[:q].sum() / wall),
                      "launches": int(stats["launches"]), "gpu_busy_frac": stats["busy_us"] * 1e-6 / wall,
                      "arena_peak_bytes": int(stats["arena_peak_bytes"]),
                      "queued_peak": int(stats["queued_peak"])}
    log(f"serve poisson: {out['poisson']}")
    # saturation: the first requests of the stream, all arriving at once
    qs = min(args.serve_queries, args.serve_burst)
    with wmi.Server(st, k=4) as srv:
        run_stream(np.zeros(8), srv)
        lat_s, wall_s = run_stream(np.zeros(qs), srv)
        stats = srv.stats()
    out["saturation"] = {"queries": int(qs), "wall_s": wall_s, "throughput_qps": qs / wall_s,
                         "windows_per_s": float(wins_of[:qs].sum() / wall_s),
                         "pairs_per_s": float(pairs_of[:qs].sum() / wall_s),
                         "p50_ms": float(np.percentile(lat_s, 50)), "p99_ms": float(np.percentile(lat_s, 99)),
                         "gpu_busy_frac": stats["busy_us"] * 1e-6 / wall_s, "launches": int(stats["launches"])}
    log(f"serve saturation: {out['saturation']}")
    st.close()
    del data
    torch.cuda.empty_cache()
    return out


def chunked_bench(wmi, torch, w, steps: int) -> dict:
    """A workload too large for one batch: consecutive batches of the whole
    query set (submit_many), series resident; one pass = a direct replay of
    every batch, enqueued back to back (each batch on its own stream)."""
    st = wmi.Store(0, budget_bytes=4 << 30)
    ids = [st.add_series(s) for s in w.series]
    assert ids == list(range(len(w.series)))
    t0 = time.perf_counter()
    batches = st.submit_many(w.queries, k=w.k, tau=w.tau)
    for b in batches:
        b.wait()
    t_submit = time.perf_counter() - t0
    for b in batches:  # warm-up pass
        b.replay(direct=True)
    for b in batches:
        b.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for b in batches:
            b.replay(direct=True)
    for b in batches:
        b.wait()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    main_ms = float(sum(b.timing()["main_ms"] for b in batches))
    evaluated = int(sum(b.count_evals() for b in batches))  # untimed extra pass with counters
    for b in batches:
        b.destroy()
    st.close()
    pairs = w.ordered_pairs
    return {"workload": w.name, "note": w.note, "queries": int(len(w.queries)), "windows": int(w.n_windows),
            "ordered_pairs": int(pairs), "batches": len(batches), "passes": steps, "ms_per_pass": dt * 1e3,
            "windows_per_s": w.n_windows / dt, "pairs_per_s": pairs / dt,
            "distance_ops_frac_valu_peak": pairs * OPS_PER_PAIR / dt / 1e12 / VALU_PEAK_TOPS,
            "main_kernel_ms_sum": main_ms,
            "main_kernel_frac_valu_peak": pairs * OPS_PER_PAIR / (main_ms / 1e3) / 1e12 / VALU_PEAK_TOPS,
            "evaluated_pairs": evaluated,
            "main_kernel_evaluated_frac": evaluated * OPS_PER_PAIR / (main_ms / 1e3) / 1e12 / VALU_PEAK_TOPS,
            "first_submit_s": t_submit}


def td_bench(wmi, torch, w) -> dict:
    """Top-down search (library driver) over the large-search pair with the
    paper's thresholds (normalised sigma = 0.2, tau = sigma / 4), windows 4096
    down to 64, step w/8; without pruning and with pruning after p = 2
    consecutive noise detections, the latter graded by overlap accuracy."""
    from paper_2204_09131_amd.search import overlap_accuracy
    st = wmi.Store(0, budget_bytes=4 << 30)
    a, b = st.add_series(w.series[0]), st.add_series(w.series[1])
    n = len(w.series[0])
    kw = dict(s_max=4096, s_min=64, sigma=0.2, tau=0.05, step_div=8, normalize=True, k=4)
    out = {"workload": f"top-down search, {w.name.split('_td_')[0]} pair of {n} points", "params": kw}
    runs = {}
    for p in (0, 2):
        st.td_search(a, b, 0, min(n, 1 << 20), p=p, **kw)  # warm-up on a prefix
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        found, stats = st.td_search(a, b, 0, n, p=p, **kw)
        dt = time.perf_counter() - t0
        runs[p] = found
        out[f"p{p}"] = {"seconds": dt, "windows_found": int(len(found)),
                        "covered_points": int(found["len"].astype(np.int64).sum()),
                        "pairs_per_s": stats["ordered_pairs"] / dt, **stats}
        log(f"td p={p}: {out[f'p{p}']}")
    ref = [(int(r["start"]), int(r["len"])) for r in runs[0]]
    cand = [(int(r["start"]), int(r["len"])) for r in runs[2]]
    out["pruning_overlap_accuracy"] = overlap_accuracy(ref, cand)
    out["pruning_speedup"] = out["p0"]["seconds"] / out["p2"]["seconds"]
    st.close()
    return out


def bu_bench(wmi, torch, w) -> dict:
    """Bottom-up search (library driver, 1024 walkers over chunks of 16,384
    points) over the large-search pair with the paper's thresholds, windows
    64 to 4096, moving step 32, max idle 2, history 4, directional pruning
    after p = 2 detections; then the integrated selection (Algorithm 3) on 6
    of 64 partitions and the selected search over the whole pair."""
    from paper_2204_09131_amd.search import isycos
    st = wmi.Store(0, budget_bytes=4 << 30)
    a, b = st.add_series(w.series[0]), st.add_series(w.series[1])
    n = len(w.series[0])
    bu = dict(s_min=64, s_max=4096, delta=32, sigma=0.2, max_idle=2, history=4, tau=0.05, p=2, normalize=True,
              chunk=16384, seed=1, k=4)
    td = dict(s_max=4096, s_min=64, sigma=0.2, tau=0.05, p=0, step_div=8, normalize=True, k=4)
    st.bu_search(a, b, 0, 1 << 18, **bu)  # warm-up on a prefix
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    found, stats = st.bu_search(a, b, 0, n, **bu)
    dt = time.perf_counter() - t0
    out = {"workload": f"bottom-up search, large-search pair of {n} points", "params": bu, "seconds": dt,
           "windows_found": int(len(found)), "covered_points": int(found["len"].astype(np.int64).sum()),
           "pairs_per_s": stats["ordered_pairs"] / dt, **stats}
    log(f"bu: {out}")
    r = isycos(st, a, b, 0, n, td, bu, M=64, m=6, alpha=0.5, rho=0.5, seed=7)
    out["isycos"] = {k: v for k, v in r.items() if k not in ("windows", "stats")}
    out["isycos"]["windows_found"] = int(len(r["windows"]))
    log(f"isycos: {out['isycos']}")
    st.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--latency-samples", type=int, default=20)
    ap.add_argument("--serve-queries", type=int, default=3000,
                    help="requests of the Poisson serving stream (20000 = the full stream)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-burst", type=int, default=2000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the all-pairs and large-search workloads")
    ap.add_argument("--large-passes", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(windows are independent; sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_09131_amd import synth, wmi

    if not os.path.exists(wmi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    w = synth.config2()
    n_win = len(w.queries)
    pairs = w.ordered_pairs
    log(f"workload {w.name}: {n_win} windows, {pairs} ordered pairs")

    st = wmi.Store(0)
    ids = [st.add_series(s) for s in w.series]
    q = w.queries.copy()
    q["a"], q["b"] = ids
    b = st.submit(q, k=w.k)
    first = b.read()
    assert np.all(np.isfinite(first["mi_base"]))

    # ---- timed region: pipelined direct runs with per-kernel events --------
    for _ in range(args.warmup):
        b.replay(direct=True)
    b.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.replay(direct=True)
    b.wait()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = b.timing()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = n_win / (ms_step / 1e3)
    again = b.read()
    assert np.array_equal(first.view(np.uint8), again.view(np.uint8)), "replay changed results"
    log(f"direct: {ms_step:.3f} ms/step, main kernel {tim['main_ms']:.3f} ms, prep {tim['prep_ms']:.3f} ms")
    # distances the kernel computes (an extra, untimed run with counters):
    # split windows scan outwards in x order and stop early
    evaluated = b.count_evals()
    log(f"distance evaluations per launch: {evaluated} ({evaluated / pairs:.3f} of the ordered pairs)")

    # ---- the same steps as graph launches -----------------------------------
    b.replay()
    b.wait()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(args.steps):
        b.replay()
    b.wait()
    torch.cuda.synchronize()
    g_ms = (time.perf_counter() - g0) / args.steps * 1e3
    log(f"graph: {g_ms:.3f} ms/step")
    b.destroy()

    # ---- query latency: fresh submit -> results on the host -------------------
    lat = []
    for _ in range(args.latency_samples):
        s0 = time.perf_counter()
        r = st.evaluate(q, k=w.k)
        lat.append((time.perf_counter() - s0) * 1e3)
    lat = np.array(lat)
    log(f"query latency p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms")

    # ---- plain form: one prep + one main launch per window ------------------
    plain = None
    if not args.no_plain:
        bp = st.submit(q, k=w.k, plain=True)
        bp.wait()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        bp.replay()
        bp.wait()
        p_ms = (time.perf_counter() - p0) * 1e3
        pt = bp.timing()
        assert np.array_equal(bp.read()["mi_base"].view(np.uint64), first["mi_base"].view(np.uint64))
        bp.destroy()
        plain = {"ms_per_step": p_ms, "value": n_win / (p_ms / 1e3), "device_ms": pt["total_ms"],
                 "launches": 1 + 2 * n_win}
        log(f"plain: {p_ms:.1f} ms/step")

    if args.copy_calibration:
        # an elementwise kernel of known traffic (reads 256 MiB, writes 256 MiB)
        # that HBM byte counters are scaled by
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()

    st.close()

    achieved = pairs * OPS_PER_PAIR / (tim["main_ms"] / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "window-MI evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "windows": n_win, "ordered_pairs": pairs, "k": w.k,
                   "estimator": "eq2 (per-dimension radii)", "scales": list(synth.CFG2_SCALES),
                   "series_len": len(w.series[0])},
        "pairs_per_s": pairs / (ms_step / 1e3),
        "distance_ops_frac_valu_peak": pairs * OPS_PER_PAIR / (ms_step / 1e3) / 1e12 / VALU_PEAK_TOPS,
        "device_ms_per_step": tim["total_ms"],
        "graph_ms_per_step": g_ms,
        "query_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "samples": int(len(lat)), "what": "fresh submit of the whole batch to results on host"},
        "kernels_ms": {"main": tim["main_ms"], "prep": tim["prep_ms"], "runs": tim["runs"]},
        "roofline": {"bound": "alu", "kernel": "main_kernel<4>", "achieved": achieved,
                     "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": (TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]
                                 if kernel_source_hash() == TRAFFIC["kernel_sha256"] else None),
                     "traffic_unit": "HBM bytes per launch (fetch + write, calibrated counters)",
                     "ops_per_pair": OPS_PER_PAIR, "pairs_per_launch": pairs,
                     "evaluated_pairs_per_launch": evaluated,
                     "evaluated_frac": evaluated * OPS_PER_PAIR / (tim["main_ms"] / 1e3) / 1e12 / VALU_PEAK_TOPS},
        "plain_gpu": plain,
    }
    if not args.no_serve:
        out["serving"] = serve_bench(args, torch, synth, wmi)
    if not args.no_large:
        log("all-pairs noise search (64 x 32768, 2016 pairs, triples) ...")
        out["all_pairs_noise"] = chunked_bench(wmi, torch, synth.config3(), args.large_passes)
        log(f"all-pairs: {out['all_pairs_noise']}")
        log("large-search proxy (one pair of 2^24, 7 dense layers) ...")
        w5 = synth.config5_proxy()
        out["large_search_proxy"] = chunked_bench(wmi, torch, w5, args.large_passes)
        log(f"large-search proxy: {out['large_search_proxy']}")
        log("top-down search over the large-search pair ...")
        out["top_down_search"] = td_bench(wmi, torch, w5)
        log("bottom-up search and selection over the large-search pair ...")
        out["bottom_up_search"] = bu_bench(wmi, torch, w5)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
