"""The library's top-down driver (wmi_td_search: speculative batches on the
GPU plus a host walk) against the sequential rule of oracle/search.py driven
by the CPU oracle's estimator, window by window: the same correlated windows
(start, length, layer) and their estimates within 1e-9."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import search
from paper_2204_09131_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-9


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def wmi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_09131_amd import wmi as w
    w.lib()
    return w


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def oracle_td(orc, x, y, margin, **kw):
    calls = []

    def mi(t, m):
        v = orc.window_mi(x[t:t + m], y[t:t + m], k=kw.get("k", 4))
        calls.append((t, m, v))
        return v
    args = {k: v for k, v in kw.items() if k != "k"}
    found = search.top_down(mi, **args)
    # decisions taken within 1e-9 of a threshold could go either way on the GPU
    sig, tau, norm = args["sigma"], args.get("tau", 0.0), args.get("normalize", False)
    for t, m, v in calls:
        thr = sig * math.log(m) if norm else sig
        if not math.isnan(v):
            margin.append(abs(v - thr))
    return found


CASES = [
    # (series seed, n, s_max, s_min, sigma, tau, p, step_div, normalize)
    (11, 16384, 1024, 64, 0.30, 0.075, 0, 8, False),
    (12, 16384, 1024, 64, 0.30, 0.075, 2, 8, False),
    (13, 12000, 512, 32, 0.20, 0.05, 1, 8, True),
    (14, 10000, 700, 40, 0.25, 0.06, 2, 3, False),   # steps 233, 116, ... do not divide the windows:
                                                     # off-grid windows in follow-up batches
]


@pytest.mark.parametrize("case", CASES)
def test_td_driver_matches_sequential_rule(wmi, orc, case):
    seed, n, s_max, s_min, sigma, tau, p, div, norm = case
    x, y = synth.cfg2_pair(n, seed)
    st = wmi.Store(0)
    a, b = st.add_series(x), st.add_series(y)
    got, stats = st.td_search(a, b, 0, n, s_max, s_min, sigma, tau=tau, p=p, step_div=div, normalize=norm)
    st.close()
    margin = []
    ref = oracle_td(orc, x, y, margin, begin=0, end=n, s_max=s_max, s_min=s_min, sigma=sigma, tau=tau, p=p,
                    step_div=div, normalize=norm)
    log(f"case {case}: {len(ref)} windows; stats {stats}; closest margin {min(margin):.3g}")
    assert min(margin) > TOL
    assert [(int(s), int(m), int(l)) for s, m, l, _ in ref] == \
        [(int(r["start"]), int(r["len"]), int(r["layer"])) for r in got]
    if len(ref):
        assert np.max(np.abs(np.array([v for *_, v in ref]) - got["mi"])) <= TOL
    if p:
        assert stats["noise_detections"] >= stats["noise_skips"]
    if s_max % max(1, s_max // div):
        assert stats["batches"] > stats["layers"]  # follow-up batches ran


def oracle_bu(orc, x, y, **kw):
    cache = {}

    def mi(s, m):
        key = (s, m)
        if key not in cache:
            cache[key] = orc.window_mi(x[s:s + m], y[s:s + m], k=kw.get("k", 4))
        return cache[key]
    args = {k: v for k, v in kw.items() if k != "k"}
    return search.bottom_up(mi, **args), cache


BU_CASES = [
    # (series seed, n, chunk, s_min, s_max, delta, max_idle, history, sigma, tau, p, normalize, seed)
    (21, 4096, 1024, 32, 256, 16, 2, 4, 0.30, 0.075, 0, False, 7),
    (22, 4096, 2048, 32, 256, 16, 2, 4, 0.30, 0.075, 2, False, 8),
    (23, 6000, 1500, 48, 384, 24, 1, 3, 0.15, 0.04, 1, True, 9),
    (24, 3000, 0, 64, 512, 32, 2, 5, 0.25, 0.06, 2, False, 10),
]


@pytest.mark.parametrize("case", BU_CASES)
def test_bu_driver_matches_sequential_rule(wmi, orc, case):
    seed, n, chunk, s_min, s_max, delta, idle, h, sigma, tau, p, norm, rs = case
    x, y = synth.cfg2_pair(n, seed)
    st = wmi.Store(0)
    a, b = st.add_series(x), st.add_series(y)
    kw = dict(s_min=s_min, s_max=s_max, delta=delta, sigma=sigma, max_idle=idle, history=h, tau=tau, p=p,
              normalize=norm, chunk=chunk, seed=rs)
    got, stats = st.bu_search(a, b, 0, n, **kw)
    st.close()
    ref, cache = oracle_bu(orc, x, y, begin=0, end=n, **kw)
    log(f"bu case {case}: {len(ref)} windows; stats {stats}; {len(cache)} distinct windows on the CPU")
    # comparisons between estimates closer than 1e-9 could go either way
    vals = np.sort(np.array([v for v in cache.values() if not math.isnan(v)]))
    assert np.min(np.diff(np.unique(vals))) > TOL
    assert [(int(s), int(m)) for s, m, _, _ in ref] == [(int(r["start"]), int(r["len"])) for r in got]
    if len(ref):
        assert np.max(np.abs(np.array([v for *_, v in ref]) - got["mi"])) <= TOL


def test_isycos_selection_runs_the_selected_search(wmi):
    from paper_2204_09131_amd.search import isycos
    x, y = synth.cfg2_pair(65536, 31)
    st = wmi.Store(0)
    a, b = st.add_series(x), st.add_series(y)
    td = dict(s_max=1024, s_min=64, sigma=0.2, tau=0.05, p=0, step_div=8, normalize=True)
    bu = dict(s_min=64, s_max=1024, delta=32, sigma=0.2, max_idle=2, history=4, tau=0.05, p=2, normalize=True,
              chunk=4096, seed=3)
    r = isycos(st, a, b, 0, 65536, td, bu, M=16, m=4, alpha=0.5, rho=0.5, seed=5)
    log(f"isycos: selected {r['selected']}, scores {r['nscore_td']:.3f} / {r['nscore_bu']:.3f}, "
        f"{len(r['windows'])} windows")
    ref, _ = (st.td_search(a, b, 0, 65536, **td) if r["selected"] == "top-down"
              else st.bu_search(a, b, 0, 65536, **bu))
    assert np.array_equal(ref, r["windows"])
    assert (r["nscore_td"] > r["nscore_bu"]) == (r["selected"] == "top-down")
    st.close()


def test_bu_many_spans_match_single_calls(wmi):
    """Walkers of several spans in one batch per step: every span gives the
    windows (and bit-identical estimates) of its own call."""
    series = [synth.cfg2_pair(6000, 41)[0], synth.cfg2_pair(6000, 41)[1], synth.cfg2_pair(6000, 42)[1]]
    spans = [(0, 1, 0, 6000), (1, 2, 500, 5500), (0, 2, 0, 4000), (0, 1, 3000, 6000), (2, 0, 100, 100)]
    kw = dict(s_min=48, s_max=384, delta=24, sigma=0.15, max_idle=1, history=3, tau=0.04, p=1, normalize=1,
              chunk=1500, seed=9)
    with wmi.Store(0) as st:
        assert [st.add_series(s) for s in series] == [0, 1, 2]
        got, span, stats = st.bu_search_many(spans, **kw)
        ref, tot = [], 0
        for i, (a, b, s0, e0) in enumerate(spans):
            r, s1 = st.bu_search(a, b, s0, e0, **kw)
            ref.append(r)
            tot += s1["windows_evaluated"]
    for i, r in enumerate(ref):
        mine = got[span == i]
        assert np.array_equal(mine.view(np.uint8), r.view(np.uint8)), i
    assert np.all(np.diff(span.astype(np.int64)) >= 0)
    assert stats["windows_evaluated"] == tot
    log(f"bu many: {len(got)} windows over {len(spans)} spans in {stats['batches']} batches")
