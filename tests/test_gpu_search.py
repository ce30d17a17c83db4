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
