"""Benchmark: windowed KSG mutual information on one MI355X.

Headline (`value`, one JSON line on stdout): the all-pairs noise search, the
largest workload that runs in full as one finite batch job: 64 float32 series
of 32,768 points on the 2^-12 grid (8 latent Gaussian factors, half the series
linear mixtures, half quadratic / sine links of one factor, plus noise), all
2016 pairs, every window position of w = 256 at stride 8 evaluated as a noise
triple (248-point overlap, 8 new points, 256-point union; Definition 6.2 with
tau = sigma / 4, sigma = 0.2 ln 256): 8,195,040 triples = 24,585,120 windows
and 1.037e12 ordered point pairs, k = 4, Eq. (2) estimator.  Series are
resident in HBM before timing starts.

A step = one pass over the whole workload: its consecutive batches (each at
most 2^18 queries) replayed back to back, alternating between two streams,
each run = descriptor upload, clear, persistent main kernel (neighbours,
counts, digamma sums, estimates, noise flags), result download.  `value` = windows / (wall time per
step).  The roofline object is for the dominant kernel, main_kernel<4>:
achieved = 8 VALU ops x the distances its neighbour searches compute (per
launch, counted by wmi_batch_count_evals: m (m - 1) per brute-forced window,
fewer for windows scanned in x order with an early stop) / its average launch
duration (HIP events on the launch stream).

Also reported, each in its own object: the multi-scale workload (one pair of
65,536 points, w = 32..4096 at stride w/8, all scales in one persistent
launch) with its HIP-graph form, the plain one-launch-per-window form and
fresh-submit latency; the serving loop on 1024 resident series of 2^20 points
under the full Poisson stream of 20,000 range requests at 200/s (p50/p99
latency, per-stage latency, throughput, device busy time) and a burst at
saturation; the large search on 8 series of 2^24 points (all 28 pairs: the
dense top-down layers, the top-down search with noise pruning, the bottom-up
search, the integrated selection on one pair); and the CPU oracle on the
host's cores over a bounded sample of the headline workload.

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

# HBM traffic of main_kernel<4> per launch, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (KiB per dispatch) over a workload's launches, each
# scaled by what the same counter reads for an elementwise kernel of known
# traffic (256 MiB read, 256 MiB written).  Valid only for the kernel source
# it was taken on (hash of the kernel and descriptor sources) and for the
# launch shape it was taken with (batches per pass); keyed by workload name.
TRAFFIC = {
    "cfg3_allpairs_64x32768_w256_s8_triples": {
        "fetch_bytes": 3557529568, "write_bytes": 9822578728, "batches_per_pass": 8,
        "kernel_sha256": "7dce003a9adfec9fb62e33a0bfc36fcf2625ffbf3836cd028b28f64262bffda2",
        "source": "profiles/main_kernel_cfg3_allpairs_triples.md"},
    "cfg2_multiscale_n65536_w32-4096_s8th": {
        "fetch_bytes": 70279870, "write_bytes": 41440010,
        "kernel_sha256": "7dce003a9adfec9fb62e33a0bfc36fcf2625ffbf3836cd028b28f64262bffda2",
        "source": "profiles/main_kernel_cfg2_multiscale.md"},
}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("wmi_kernels.hip", "wmi_internal.h"):
        with open(os.path.join(ROOT, "paper_2204_09131_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_of(workload: str, batches_per_pass: int = 1):
    t = TRAFFIC.get(workload)
    if not t or t["kernel_sha256"] != kernel_source_hash():
        return None
    if t.get("batches_per_pass", 1) != batches_per_pass:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, budget_s: float = 20.0) -> dict:
    """The oracle as it stands, on every host core, over a bounded sample."""
    import oracle
    orc = oracle.load()
    cores = orc.threads(len(os.sched_getaffinity(0)))
    q = workload.queries
    # a strided sample over all pairs and positions, grown until it takes a
    # few seconds
    step = 1 << 14
    t_used = 0.0
    while True:
        sub = q[::step]
        t0 = time.perf_counter()
        orc.batch(workload.series, sub, k=workload.k, tau=workload.tau)
        dt = time.perf_counter() - t0
        t_used += dt
        if dt > 3.0 or step == 1 or t_used > budget_s:
            break
        step = max(1, step // 4)
    reps = max(1, int(10.0 / max(dt, 1e-3)))
    if reps > 1:
        t0 = time.perf_counter()
        for _ in range(reps):
            orc.batch(workload.series, sub, k=workload.k, tau=workload.tau)
        dt = (time.perf_counter() - t0) / reps
    sw = sample_windows(sub)
    return {"value": sw / dt, "unit": "window-MI evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(sub)} of {len(q)} queries ({sw} windows; every {step}-th query of {workload.name}), "
                      f"{reps} pass(es) of {dt:.2f} s each",
            "pairs_per_s": sample_pairs(sub) / dt}


def sample_windows(q) -> int:
    return int(len(q) + 2 * np.count_nonzero(q["ext_side"] != 0))


def sample_pairs(q) -> float:
    m = q["len"].astype(np.float64)
    tot = float(np.sum(m * (m - 1)))
    t = q["ext_side"] != 0
    me = q["ext_len"][t].astype(np.float64)
    mu = m[t] + me
    return tot + float(np.sum(me * (me - 1)) + np.sum(mu * (mu - 1)))


# batches of the headline pass (runs of whole pairs); alternating streams
HEADLINE_BATCHES = 8


def frac(ops, seconds) -> float:
    return ops / seconds / 1e12 / VALU_PEAK_TOPS


# ---------------------------------------------------------------------------
# headline: the all-pairs noise search
# ---------------------------------------------------------------------------

def headline(args, wmi, torch, w) -> dict:
    st = wmi.Store(0, budget_bytes=8 << 30, tuning="auto")
    ids = [st.add_series(s) for s in w.series]
    assert ids == list(range(len(w.series)))
    # the query list as runs, one per pair (equally spaced triples): the host
    # plans per run and the device writes the descriptors at every run
    q = w.queries
    n_pairs = len(w.series) * (len(w.series) - 1) // 2
    cnt = len(q) // n_pairs
    ab = q[::cnt]
    rg = wmi.make_ranges(ab["a"], ab["b"], int(q["start"][0]), cnt, int(q["start"][1] - q["start"][0]),
                         int(q["len"][0]), int(q["ext_len"][0]), int(q["ext_side"][0]))
    assert np.array_equal(wmi.expand_ranges(rg).view(np.uint8), q.view(np.uint8))
    groups = np.array_split(rg, HEADLINE_BATCHES)
    t0 = time.perf_counter()
    batches = [st.submit_ranges(g, k=w.k, tau=w.tau) for g in groups]
    first = [b.read() for b in batches]
    t_submit = time.perf_counter() - t0
    for r in first:
        assert np.all(np.isfinite(r["mi_base"])) and np.all(np.isfinite(r["mi_union"]))
    log(f"headline: {len(rg)} runs in {len(batches)} batches, first submit {t_submit:.2f} s")
    # consecutive batches alternate between two streams, so that one batch's
    # result download overlaps its neighbour's kernels
    # (--serial: one stream, so that per-dispatch hardware counters see one
    # launch at a time)
    streams = [torch.cuda.Stream()] * 2 if args.serial else [torch.cuda.Stream(), torch.cuda.Stream()]
    for _ in range(max(1, args.warmup)):
        for i, b in enumerate(batches):
            b.replay(stream=streams[i % 2], direct=True)
    for b in batches:
        b.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for i, b in enumerate(batches):
            b.replay(stream=streams[i % 2], direct=True)
    for b in batches:
        b.wait()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    tims = [b.timing() for b in batches]
    main_ms = float(sum(t["main_ms"] for t in tims))
    for b, r in zip(batches, first):
        assert np.array_equal(b.read().view(np.uint8), r.view(np.uint8)), "replay changed results"
    # untimed extra pass with counters (left out of profiling runs, whose
    # kernel statistics should hold the timed launches only)
    evaluated = None if args.no_evals else int(sum(b.count_evals() for b in batches))
    noise = int(sum(np.count_nonzero(r["flags"] & 1) for r in first))
    for b in batches:
        b.destroy()
    st.close()
    pairs = w.ordered_pairs
    launches = len(batches)
    achieved = None if evaluated is None else OPS_PER_PAIR * evaluated / (main_ms / 1e3) / 1e12
    log(f"headline: {dt * 1e3:.1f} ms/pass, main kernels {main_ms:.1f} ms, evaluated {evaluated} of {pairs}")
    return {"dt": dt, "batches": launches, "runs": int(len(rg)), "first_submit_s": t_submit, "main_ms_sum": main_ms,
            "evaluated": evaluated, "pairs": pairs, "noise_triples": noise,
            "roofline": {"bound": "alu", "kernel": "main_kernel<4>", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                         "unit": "TOP/s", "frac": None if achieved is None else achieved / VALU_PEAK_TOPS,
                         "traffic": traffic_of(w.name, HEADLINE_BATCHES),
                         "traffic_unit": "HBM bytes per launch (fetch + write, calibrated counters)",
                         "ops_per_distance": OPS_PER_PAIR, "launches_per_step": launches,
                         "distances_per_launch": None if evaluated is None else evaluated / launches,
                         "ordered_pairs_per_launch": pairs / launches,
                         "avg_launch_ms": main_ms / launches}}


# ---------------------------------------------------------------------------
# the multi-scale workload: one persistent launch over 8 scales
# ---------------------------------------------------------------------------

def multiscale(args, wmi, torch, synth) -> dict:
    w = synth.config2()
    n_win = len(w.queries)
    pairs = w.ordered_pairs
    st = wmi.Store(0, tuning="auto")
    ids = [st.add_series(s) for s in w.series]
    q = w.queries.copy()
    q["a"], q["b"] = ids
    b = st.submit(q, k=w.k)
    first = b.read()
    assert np.all(np.isfinite(first["mi_base"]))
    # a fixed warm-up (about 30 ms of work) so that the number does not
    # depend on --warmup
    for _ in range(48):
        b.replay(direct=True)
    b.wait()
    torch.cuda.synchronize()
    steps = max(args.steps, 16)
    t0 = time.perf_counter()
    for _ in range(steps):
        b.replay(direct=True)
    b.wait()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / steps * 1e3
    tim = b.timing()
    assert np.array_equal(first.view(np.uint8), b.read().view(np.uint8)), "replay changed results"
    evaluated = b.count_evals()
    b.replay()
    b.wait()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(steps):
        b.replay()
    b.wait()
    torch.cuda.synchronize()
    g_ms = (time.perf_counter() - g0) / steps * 1e3
    b.destroy()
    lat = []
    for _ in range(args.latency_samples):
        s0 = time.perf_counter()
        st.evaluate(q, k=w.k)
        lat.append((time.perf_counter() - s0) * 1e3)
    lat = np.array(lat)
    # the same windows as runs (one per scale), expanded on the device
    n = len(w.series[0])
    rg = np.concatenate([wmi.make_ranges(ids[0], ids[1], 0, (n - wl) // (wl // 8) + 1, wl // 8, wl)
                         for wl in synth.CFG2_SCALES])
    assert np.array_equal(wmi.expand_ranges(rg).view(np.uint8), q.view(np.uint8))
    br = st.submit_ranges(rg, k=w.k)
    assert np.array_equal(br.read().view(np.uint8), first.view(np.uint8))
    for _ in range(48):
        br.replay(direct=True)
    br.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        br.replay(direct=True)
    br.wait()
    torch.cuda.synchronize()
    r_ms = (time.perf_counter() - t0) / steps * 1e3
    r_tim = br.timing()
    br.replay()
    br.wait()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(steps):
        br.replay()
    br.wait()
    torch.cuda.synchronize()
    rg_ms = (time.perf_counter() - g0) / steps * 1e3
    br.destroy()
    rlat = []
    for _ in range(args.latency_samples):
        s0 = time.perf_counter()
        bb = st.submit_ranges(rg, k=w.k)
        bb.read()
        rlat.append((time.perf_counter() - s0) * 1e3)
        bb.destroy()
    rlat = np.array(rlat)
    runs = {"runs": int(len(rg)), "ms_per_step": r_ms, "windows_per_s": n_win / (r_ms / 1e3),
            "graph_ms_per_step": rg_ms, "graph_windows_per_s": n_win / (rg_ms / 1e3),
            "device_ms_per_step": r_tim["total_ms"], "main_ms": r_tim["main_ms"],
            "query_latency_ms": {"p50": float(np.percentile(rlat, 50)), "p99": float(np.percentile(rlat, 99)),
                                 "samples": int(len(rlat))}}
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
        plain = {"ms_per_step": p_ms, "windows_per_s": n_win / (p_ms / 1e3), "device_ms": pt["total_ms"],
                 "launches": 1 + 2 * n_win}
    st.close()
    main_s = tim["main_ms"] / 1e3
    out = {"workload": w.name, "windows": n_win, "ordered_pairs": pairs, "k": w.k,
           "scales": list(synth.CFG2_SCALES), "series_len": len(w.series[0]),
           "ms_per_step": ms_step, "windows_per_s": n_win / (ms_step / 1e3),
           "graph_ms_per_step": g_ms, "graph_windows_per_s": n_win / (g_ms / 1e3),
           "device_ms_per_step": tim["total_ms"],
           "kernels_ms": {"main": tim["main_ms"], "prep": tim["prep_ms"], "runs": tim["runs"]},
           "brute_force_pairs_per_s": pairs / (ms_step / 1e3),
           "main_kernel": {"evaluated_distances": int(evaluated), "evaluated_share": evaluated / pairs,
                           "achieved_tops": OPS_PER_PAIR * evaluated / main_s / 1e12,
                           "frac_valu_peak": frac(OPS_PER_PAIR * evaluated, main_s),
                           "hbm_traffic_bytes": traffic_of(w.name)},
           "query_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                "samples": int(len(lat)), "what": "fresh submit of the whole batch to results on host"},
           "as_runs": runs,
           "plain_gpu": plain}
    log(f"multiscale: {out}")
    return out


# ---------------------------------------------------------------------------
# the plain workload: a stride-1 sweep, incremental against window by window
# ---------------------------------------------------------------------------

def plain_sweep(args, wmi, torch, synth) -> dict:
    """One pair of 4096 points, w = 128, stride 1 (3,969 windows): the
    incremental form (each window from the one before, Section 7.1.2) with
    2 .. 16 windows per sweep item, and every window on its own, each timed
    over pipelined direct runs.  The autotuner's choice for this window size
    is reported beside them."""
    w = synth.config1()
    out = {"workload": w.name, "windows": len(w.queries), "ordered_pairs": w.ordered_pairs}
    with wmi.Store(0, tuning="auto") as st0:
        tuned = st0.get_tuning()
    out["autotuned_sweep_windows"] = tuned["sweep_windows"]
    res = {}
    variants = [("window_by_window", tuned, {"no_reuse": True})]
    variants += [(f"incremental_{c}", dict(tuned, sweep_windows=[c, c, c]), {}) for c in (2, 4, 8, 16)]
    for name, tun, kw in variants:
        with wmi.Store(0, tuning=tun) as st:
            ids = [st.add_series(s) for s in w.series]
            q = w.queries.copy()
            q["a"], q["b"] = ids
            b = st.submit(q, k=w.k, **kw)
            res[name] = b.read()
            for _ in range(30):
                b.replay(direct=True)
            b.wait()
            torch.cuda.synchronize()
            steps = max(args.steps, 50)
            t0 = time.perf_counter()
            for _ in range(steps):
                b.replay(direct=True)
            b.wait()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            tim = b.timing()
            ev = b.count_evals()
            b.destroy()
        out[name] = {"ms_per_step": ms, "windows_per_s": len(q) / (ms / 1e3), "main_kernel_ms": tim["main_ms"],
                     "distances": int(ev)}
    for name in res:
        assert np.array_equal(res[name].view(np.uint8), res["window_by_window"].view(np.uint8)), name
    best = min((n for n, _, _ in variants[1:]), key=lambda n: out[n]["main_kernel_ms"])
    out["incremental_best"] = best
    out["kernel_speedup_best"] = out["window_by_window"]["main_kernel_ms"] / out[best]["main_kernel_ms"]
    log(f"plain sweep: {out}")
    return out


# ---------------------------------------------------------------------------
# serving: the full Poisson stream of range requests
# ---------------------------------------------------------------------------

def serve_bench(args, torch, synth, wmi) -> dict:
    """1024 resident series x 2^20 points (4 GiB, the multi-scale segment
    recipe, drawn on the device), a Poisson stream of range requests (random
    pair, w log-uniform in [32, 2048], stride w/4, whole series) at `rate` per
    second, continuous batching with arena admission.  Latency of a request =
    results on the host minus its scheduled arrival.  Then the first requests
    of the stream submitted at once (saturation throughput)."""
    import threading
    n_series, n = 1024, 1 << 20
    t_gen = time.perf_counter()
    data = synth.cfg2_pairs_device(n_series // 2, n, seed=4, device="cuda")
    torch.cuda.synchronize()
    log(f"serve: generated {n_series} x {n} series in {time.perf_counter() - t_gen:.1f} s")
    t, a, b, w, stride = synth.config4_stream(n_queries=args.serve_queries, n_series=n_series, n=n,
                                              rate=args.serve_rate)
    st = wmi.Store(0, tuning="auto")
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
        stage = np.zeros((len(times), 3))
        done = 0
        while done < len(times):
            while tickets[done] == 0:
                if errors:
                    raise errors[0]
                time.sleep(0.0005)
            srv.wait(tickets[done], 600_000_000)
            if done % 2000 == 1999:
                log(f"serve: {done + 1} of {len(times)} requests done")
            res, info = srv.read(tickets[done])
            if not np.all(np.isfinite(res["mi"])):
                raise RuntimeError(f"request {done}: non-finite MI")
            lat[done] = (info["t_complete_us"] - sched[done]) * 1e-3
            stage[done] = [(info["t_admit_us"] - sched[done]) * 1e-3,
                           (info["t_first_launch_us"] - info["t_admit_us"]) * 1e-3,
                           (info["t_complete_us"] - info["t_first_launch_us"]) * 1e-3]
            done += 1
        th.join()
        return lat, stage, time.perf_counter() - w0

    def pct(v):
        return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)), "max": float(v.max())}

    out = {"workload": f"serving: {n_series} resident series x {n} float32 (multi-scale segment recipe), "
                       "Poisson range requests (random pair, w log-uniform 32..2048, stride w/4, whole series)",
           "k": 4}
    with wmi.Server(st, k=4) as srv:
        run_stream(np.zeros(8), srv)  # warm up the scheduler and both launch slots
        s0 = srv.stats()
        q = args.serve_queries
        lat, stage, wall = run_stream(t[:q], srv)
        s1 = srv.stats()
    out["poisson"] = {"rate_qps": args.serve_rate, "queries": int(q), "wall_s": wall,
                      "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "max_ms": float(lat.max()), "throughput_qps": q / wall,
                      "stages_ms": {"arrival_to_admit": pct(stage[:, 0]), "admit_to_first_launch": pct(stage[:, 1]),
                                    "first_launch_to_complete": pct(stage[:, 2])},
                      "windows_per_s": float(wins_of[:q].sum() / wall),
                      "pairs_per_s": float(pairs_of[:q].sum() / wall),
                      "launches": int(s1["launches"] - s0["launches"]),
                      "gpu_busy_frac": (s1["busy_union_us"] - s0["busy_union_us"]) * 1e-6 / wall,
                      "arena_peak_bytes": int(s1["arena_peak_bytes"]),
                      "queued_peak": int(s1["queued_peak"])}
    log(f"serve poisson: {out['poisson']}")
    qs = min(args.serve_queries, args.serve_burst)
    with wmi.Server(st, k=4) as srv:
        run_stream(np.zeros(8), srv)
        s0 = srv.stats()
        lat_s, stage_s, wall_s = run_stream(np.zeros(qs), srv)
        s1 = srv.stats()
    out["saturation"] = {"queries": int(qs), "wall_s": wall_s, "throughput_qps": qs / wall_s,
                         "windows_per_s": float(wins_of[:qs].sum() / wall_s),
                         "pairs_per_s": float(pairs_of[:qs].sum() / wall_s),
                         "p50_ms": float(np.percentile(lat_s, 50)), "p99_ms": float(np.percentile(lat_s, 99)),
                         "gpu_busy_frac": (s1["busy_union_us"] - s0["busy_union_us"]) * 1e-6 / wall_s,
                         "launches": int(s1["launches"] - s0["launches"])}
    log(f"serve saturation: {out['saturation']}")
    st.close()
    del data
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# the large search: 8 series of 2^24 points, all 28 pairs
# ---------------------------------------------------------------------------

def large_search(args, wmi, torch, synth) -> dict:
    from paper_2204_09131_amd.search import isycos, overlap_accuracy
    t_gen = time.perf_counter()
    series = synth.config5_series(5, n_series=8)
    n = len(series[0])
    log(f"large search: generated 8 x {n} series in {time.perf_counter() - t_gen:.1f} s")
    st = wmi.Store(0, budget_bytes=4 << 30, tuning="auto")
    ids = [st.add_series(s) for s in series]
    pairs = [(i, j) for i in range(8) for j in range(i + 1, 8)]
    if args.large_pairs:
        pairs = pairs[:args.large_pairs]
    out = {"workload": f"large search: 8 IoT-like series x {n} float32, {len(pairs)} pairs, w 64..4096, k 4",
           "pairs": len(pairs)}

    # the dense top-down layers (every window of w = 4096 .. 64 at stride w/8)
    rd = np.concatenate([wmi.make_ranges(0, 1, 0, (n - wl) // (wl // 8) + 1, wl // 8, wl) for wl in synth.CFG5_LAYERS])
    n_win = int(rd["count"].sum())
    dense_pairs = float(np.sum(rd["count"] * rd["len"].astype(np.float64) * (rd["len"] - 1.0)))
    t_sum, main_ms, evaluated = 0.0, 0.0, 0
    for i, (a, b) in enumerate(pairs):
        r = rd.copy()
        r["a"], r["b"] = ids[a], ids[b]
        batches = st.submit_ranges_many(r, k=4)
        for bt in batches:
            bt.wait()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for bt in batches:
            bt.replay(direct=True)
        for bt in batches:
            bt.wait()
        torch.cuda.synchronize()
        t_sum += time.perf_counter() - t0
        main_ms += float(sum(bt.timing()["main_ms"] for bt in batches))
        if i == 0:
            evaluated = int(sum(bt.count_evals() for bt in batches))
        for bt in batches:
            bt.destroy()
    out["dense_layers"] = {"windows_per_pair": n_win, "ordered_pairs_per_pair": dense_pairs,
                           "seconds": t_sum, "windows_per_s": n_win * len(pairs) / t_sum,
                           "brute_force_pairs_per_s": dense_pairs * len(pairs) / t_sum,
                           "main_kernel_ms": main_ms,
                           "evaluated_distances_pair0": evaluated,
                           "main_kernel_frac_valu_peak_pair0_rate": frac(OPS_PER_PAIR * evaluated * len(pairs),
                                                                         main_ms / 1e3)}
    log(f"large dense: {out['dense_layers']}")

    td = dict(s_max=4096, s_min=64, sigma=0.2, tau=0.05, step_div=8, normalize=True, k=4)
    bu = dict(s_min=64, s_max=4096, delta=32, sigma=0.2, max_idle=2, history=4, tau=0.05, p=2, normalize=True,
              chunk=16384, seed=1, k=4)
    st.td_search(ids[0], ids[1], 0, 1 << 20, p=2, **td)  # warm-up on a prefix
    st.bu_search(ids[0], ids[1], 0, 1 << 18, **bu)
    torch.cuda.synchronize()
    for name, fn in (("top_down", lambda a, b: st.td_search(a, b, 0, n, p=2, **td)),
                     ("bottom_up_per_pair", lambda a, b: st.bu_search(a, b, 0, n, **bu))):
        agg = {"seconds": 0.0, "windows_found": 0, "windows_evaluated": 0, "ordered_pairs": 0, "batches": 0,
               "noise_skips": 0, "submit_s": 0.0, "wait_s": 0.0}
        for a, b in pairs:
            t0 = time.perf_counter()
            found, stats = fn(ids[a], ids[b])
            agg["seconds"] += time.perf_counter() - t0
            agg["windows_found"] += int(len(found))
            for f in ("windows_evaluated", "ordered_pairs", "batches", "noise_skips"):
                agg[f] += int(stats[f])
            agg["submit_s"] += stats["submit_ms"] / 1e3
            agg["wait_s"] += stats["wait_ms"] / 1e3
        agg["windows_per_s"] = agg["windows_evaluated"] / agg["seconds"]
        agg["pairs_per_s"] = agg["ordered_pairs"] / agg["seconds"]
        out[name] = agg
        log(f"large {name}: {agg}")
    # bottom-up over every pair at once: the walkers of all pairs advance
    # together, one batch per step
    t0 = time.perf_counter()
    found, span, stats = st.bu_search_many([(ids[a], ids[b], 0, n) for a, b in pairs], **bu)
    dt = time.perf_counter() - t0
    out["bottom_up"] = {"seconds": dt, "windows_found": int(len(found)),
                        "windows_evaluated": int(stats["windows_evaluated"]),
                        "ordered_pairs": int(stats["ordered_pairs"]), "batches": int(stats["batches"]),
                        "noise_skips": int(stats["noise_skips"]),
                        "submit_s": stats["submit_ms"] / 1e3, "wait_s": stats["wait_ms"] / 1e3,
                        "windows_per_s": stats["windows_evaluated"] / dt, "pairs_per_s": stats["ordered_pairs"] / dt,
                        "same_as_per_pair": int(len(found)) == out["bottom_up_per_pair"]["windows_found"]}
    log(f"large bottom_up (all pairs together): {out['bottom_up']}")

    # pruning on one pair: p = 0 against p = 2, graded by overlap accuracy
    runs = {}
    for p in (0, 2):
        t0 = time.perf_counter()
        found, stats = st.td_search(ids[0], ids[1], 0, n, p=p, **td)
        runs[p] = (found, time.perf_counter() - t0, stats)
    ref = [(int(r["start"]), int(r["len"])) for r in runs[0][0]]
    cand = [(int(r["start"]), int(r["len"])) for r in runs[2][0]]
    out["td_pruning_pair0"] = {"p0_s": runs[0][1], "p2_s": runs[2][1], "speedup": runs[0][1] / runs[2][1],
                               "p0_pairs": runs[0][2]["ordered_pairs"], "p2_pairs": runs[2][2]["ordered_pairs"],
                               "overlap_accuracy": overlap_accuracy(ref, cand)}
    log(f"large td pruning: {out['td_pruning_pair0']}")
    r = isycos(st, ids[0], ids[1], 0, n, dict(td, p=2), bu, M=64, m=6, alpha=0.5, rho=0.5, seed=7)
    out["isycos_pair0"] = {k: v for k, v in r.items() if k not in ("windows", "stats")}
    out["isycos_pair0"]["windows_found"] = int(len(r["windows"]))
    log(f"large isycos: {out['isycos_pair0']}")
    out["sigma_tau_estimators"] = sigma_tau_sweep(st, ids, n, wmi)
    st.close()
    return out


def sigma_tau_sweep(st, ids, n, wmi) -> dict:
    """The thresholds' meaning under the two estimators: Eq. 2 (KSG-2) and
    Kraskov's first form (KSG-1) on pair 0's first 2^22 points.  The same
    windows of one layer under both (how their values differ), then the
    top-down search (normalised thresholds, tau = sigma / 4, p = 2) for
    several sigma under each, and how far the windows each finds agree."""
    from scipy.stats import spearmanr

    from paper_2204_09131_amd.search import overlap_accuracy
    span = min(n, 1 << 22)
    rr = wmi.make_ranges(ids[0], ids[1], 0, (span - 256) // 32 + 1, 32, 256)
    vals = {}
    for est in (0, 1):
        b = st.submit_ranges(rr, k=4, estimator=est)
        vals[est] = b.read()["mi_base"]
        b.destroy()
    d = vals[1] - vals[0]
    out = {"span": span, "layer_w256": {"windows": int(len(d)), "mean_ksg2": float(np.mean(vals[0])),
                                         "mean_ksg1": float(np.mean(vals[1])), "mean_diff": float(np.mean(d)),
                                         "sd_diff": float(np.std(d)),
                                         "spearman": float(spearmanr(vals[0], vals[1]).statistic)}}
    found, rows = {}, []
    for est in (0, 1):
        for sg in (0.1, 0.2, 0.3, 0.5):
            t0 = time.perf_counter()
            f, stt = st.td_search(ids[0], ids[1], 0, span, s_max=4096, s_min=64, sigma=sg, tau=sg / 4, p=2,
                                  step_div=8, normalize=1, k=4, estimator=est)
            found[(est, sg)] = [(int(r["start"]), int(r["len"])) for r in f]
            rows.append({"estimator": "ksg1" if est else "ksg2", "sigma": sg, "tau": sg / 4, "windows": int(len(f)),
                         "covered_share": float(np.sum(f["len"].astype(np.int64))) / span,
                         "noise_skips": int(stt["noise_skips"]), "seconds": time.perf_counter() - t0})
    out["top_down"] = rows
    out["agreement"] = [{"sigma": sg, "ksg2_found_by_ksg1": overlap_accuracy(found[(0, sg)], found[(1, sg)]),
                         "ksg1_found_by_ksg2": overlap_accuracy(found[(1, sg)], found[(0, sg)])}
                        for sg in (0.1, 0.2, 0.3, 0.5)]
    log(f"sigma/tau across estimators: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--latency-samples", type=int, default=20)
    ap.add_argument("--serve-queries", type=int, default=20000,
                    help="requests of the Poisson serving stream (20000 = the full stream)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-burst", type=int, default=2000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-multiscale", action="store_true")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the headline workload (profiling runs of the other workloads only)")
    ap.add_argument("--no-large", action="store_true", help="skip the large search")
    ap.add_argument("--large-pairs", type=int, default=0, help="first N of the 28 pairs (0: all)")
    ap.add_argument("--no-evals", action="store_true",
                    help="skip the distance-counting pass of the headline (profiling runs)")
    ap.add_argument("--serial", action="store_true",
                    help="headline batches on one stream (for per-dispatch counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB elementwise kernel (HBM counter calibration)")
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

    w = synth.config3()
    log(f"headline {w.name}: {w.n_windows} windows, {w.ordered_pairs} ordered pairs")
    if args.no_headline:
        h = {"dt": float("nan"), "batches": 0, "noise_triples": 0, "roofline": None}
    else:
        h = headline(args, wmi, torch, w)
    out = {
        "metric": METRIC,
        "value": w.n_windows / h["dt"],
        "unit": "window-MI evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "series": len(w.series), "series_len": len(w.series[0]),
                   "pairs": len(w.series) * (len(w.series) - 1) // 2, "window": 256, "stride": 8,
                   "triples": int(len(w.queries)), "windows": w.n_windows, "ordered_pairs": w.ordered_pairs,
                   "k": w.k, "tau": w.tau, "estimator": "eq2 (per-dimension radii)"},
        "pairs_per_s": w.ordered_pairs / h["dt"],
        "distance_ops_per_s": OPS_PER_PAIR * w.ordered_pairs / h["dt"],
        "batches_per_step": h["batches"],
        "noise_triples": h["noise_triples"],
        "roofline": h["roofline"],
    }
    # the work-list choices (tile shapes) in use: the autotuner's file for
    # this architecture when there is one, else the library's defaults
    with wmi.Store(0, tuning="auto") as st:
        tf = wmi.tuning_file(0)
        out["tuning"] = {"source": os.path.relpath(tf, ROOT) if os.path.exists(tf) else "defaults",
                         **st.get_tuning()}
    if args.copy_calibration:
        # an elementwise kernel of known traffic (reads 256 MiB, writes 256 MiB)
        # that HBM byte counters are scaled by
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_multiscale:
        out["multiscale"] = multiscale(args, wmi, torch, synth)
        out["plain_sweep"] = plain_sweep(args, wmi, torch, synth)
    if not args.no_serve:
        out["serving"] = serve_bench(args, torch, synth, wmi)
    if not args.no_large:
        out["large_search"] = large_search(args, wmi, torch, synth)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
