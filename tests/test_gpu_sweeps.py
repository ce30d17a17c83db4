"""Sweep items: runs of equally spaced windows evaluated incrementally (each
window from the one before: points removed and added, influenced regions
of Section 7.1.2) against the same windows evaluated one by one
(WMI_SUBMIT_NO_REUSE) -- bit for bit, both sum the same exact integers --
and against the oracle within 1e-9."""
import sys

import numpy as np
import pytest

import oracle
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
    o = oracle.load()
    o.threads(0)
    return o


def same_bits(a, b):
    assert np.array_equal(a["mi_base"].view(np.uint64), b["mi_base"].view(np.uint64))
    assert np.array_equal(a["flags"], b["flags"])


def test_plain_workload_all_windows(wmi, orc):
    """Every window of the plain workload (n = 4096, w = 128, stride 1)."""
    w = synth.config1()
    with wmi.Store(0) as st:
        ids = [st.add_series(s) for s in w.series]
        q = w.queries.copy()
        q["a"], q["b"] = ids
        b = st.submit(q, k=4)
        inc = b.read()
        ev = b.count_evals()
        b.destroy()
        b = st.submit(q, k=4, no_reuse=True)
        full = b.read()
        ev_full = b.count_evals()
        b.destroy()
    same_bits(inc, full)
    ref = orc.batch(w.series, w.queries, k=4)
    assert float(np.max(np.abs(inc["mi_base"] - ref["mi_base"]))) <= TOL
    assert np.array_equal(inc["flags"], ref["flags"])
    assert ev_full == w.ordered_pairs and ev < ev_full / 3
    log(f"plain workload: {len(q)} windows, incremental == one by one == oracle; "
        f"distances {ev} vs {ev_full} ({ev_full / ev:.1f}x fewer)")


def make_series(kind, n, seed):
    if kind == "segments":
        return synth.cfg2_pair(n, seed)
    if kind == "normal":
        return synth.bivariate_normal(n, 0.6, seed)
    if kind == "ties":
        return synth.grid_points(n, seed, levels=4, scale=1 / 32)
    if kind == "heavy":
        r = synth.rng(seed)
        x = r.standard_normal(n)
        y = r.standard_normal(n) / (r.uniform(0.0, 1.0, n) + 0.02)
        return synth.quantize(x), synth.quantize(y / 8.0)
    if kind == "wide":  # values too spread for 32-bit keys: windows evaluated one by one
        return synth.bivariate_normal(n, 0.6, seed, scale=900.0)
    if kind == "offgrid":
        x, y = synth.bivariate_normal(n, 0.6, seed)
        y = y.copy()
        y[::97] += np.float32(1e-5)  # windows of fewer than 97 points hold one such value or none
        return x, y
    raise ValueError(kind)


CASES = [
    # (kind, m, stride, k, est, run lengths)
    ("segments", 128, 1, 4, 0, (40, 9, 2, 17)),
    ("normal", 64, 2, 4, 1, (33, 8, 5)),
    ("ties", 100, 3, 3, 0, (25, 12)),
    ("heavy", 240, 15, 4, 0, (20, 10)),
    ("normal", 34, 1, 16, 0, (30, 3)),
    ("segments", 200, 12, 8, 1, (18, 9)),
    ("ties", 48, 1, 1, 0, (50,)),
    ("wide", 96, 2, 4, 0, (20,)),
    ("offgrid", 80, 1, 4, 0, (40,)),
]


@pytest.mark.parametrize("kind,m,s,k,est,runs", CASES)
def test_runs_incremental_equal_one_by_one_and_oracle(wmi, orc, kind, m, s, k, est, runs):
    n = 6000
    x, y = make_series(kind, n, 81 + m + s)
    r = np.random.default_rng(82)
    parts, start = [], 0
    for L in runs:
        start += int(r.integers(0, 300))
        parts.append(synth.make_queries(0, 1, start + s * np.arange(L, dtype=np.uint64), m))
        start += s * L + m
        # other queries between the runs: a plain window of another size and a triple
        parts.append(synth.make_queries(0, 1, np.array([start % 3000], dtype=np.uint64), m + 7))
        parts.append(synth.make_queries(0, 1, np.array([100], dtype=np.uint64), 60, 8, +1))
    q = np.concatenate(parts)
    assert int(q["start"].max()) + m + 8 < n
    with wmi.Store(0) as st:
        ids = (st.add_series(x), st.add_series(y))
        qq = q.copy()
        qq["a"], qq["b"] = ids
        inc = st.evaluate(qq, k=k, estimator=est, tau=0.05)
        full = st.evaluate(qq, k=k, estimator=est, tau=0.05, no_reuse=True)
    for f in ("mi_base", "mi_ext", "mi_union"):
        assert np.array_equal(inc[f].view(np.uint64), full[f].view(np.uint64)), f
    assert np.array_equal(inc["flags"], full["flags"])
    ref = orc.batch([x, y], q, k=k, estimator=est, tau=0.05)
    for f in ("mi_base", "mi_ext", "mi_union"):
        a, b = inc[f], ref[f]
        assert np.array_equal(np.isnan(a), np.isnan(b)), f
        ok = ~np.isnan(b)
        if ok.any():
            assert float(np.max(np.abs(a[ok] - b[ok]))) <= TOL, f
    assert np.array_equal(inc["flags"], ref["flags"])
    if kind == "offgrid":
        assert np.any(inc["flags"] & wmi.F_OFFGRID) and not np.all(inc["flags"] & wmi.F_OFFGRID)
    log(f"{kind} m={m} s={s} k={k} est={est}: {len(q)} queries, incremental == one by one == oracle")
