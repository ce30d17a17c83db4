"""Noise triples evaluated through their unions (triple items: the base's and
the extension's neighbour lists come from the union's scan) against the same
triples evaluated window by window (WMI_SUBMIT_NO_REUSE) and against
the oracle.  Both GPU forms sum the same exact integers, so they must agree
bit for bit; the oracle within 1e-9, flags equal outside the 1e-9 margin."""
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


def bits_equal(a, b):
    for f in ("mi_base", "mi_ext", "mi_union"):
        assert np.array_equal(a[f].view(np.uint64), b[f].view(np.uint64)), f
    assert np.array_equal(a["flags"], b["flags"])


def oracle_close(got, ref, tau_eff):
    for f in ("mi_base", "mi_ext", "mi_union"):
        x, r = got[f], ref[f]
        assert np.array_equal(np.isnan(x), np.isnan(r)), f
        ok = ~np.isnan(r)
        if ok.any():
            assert float(np.max(np.abs(x[ok] - r[ok]))) <= TOL, f
    for i in np.nonzero(got["flags"] != ref["flags"])[0]:
        r = ref[i]
        margin = min(abs(r["mi_ext"] - tau_eff[i]), abs(r["mi_union"] - r["mi_base"]), abs(r["mi_base"]))
        assert margin < TOL, (i, got[i], r)


def mixed_triples(ids, n, seed):
    """Triples of many shapes: top-down style (overlap + new part on the
    right), bottom-up style (extensions on the left), parts of 1..k points,
    odd sizes, unions up to 512 points, and a few that do not fit a triple
    item (unions above 512) or are plain windows, interleaved."""
    r = np.random.default_rng(seed)
    a, b = ids
    parts = []
    shapes = [(248, 8, +1), (56, 8, +1), (120, 16, +1), (448, 64, +1), (247, 9, +1), (64, 32, -1),
              (96, 64, -1), (300, 212, -1), (3, 2, +1), (5, 4, +1), (40, 1, -1), (4, 60, +1), (2, 2, -1),
              (200, 200, +1), (511, 1, +1), (17, 33, -1)]
    for base, ext, side in shapes:
        lo = ext if side < 0 else 0
        starts = np.sort(r.choice(np.arange(lo, n - base - ext), 40, replace=False)).astype(np.uint64)
        parts.append(synth.make_queries(a, b, starts, base, ext, side))
    parts.append(synth.make_queries(a, b, np.arange(100, 2000, 97, dtype=np.uint64), 700, 100, +1))  # union 800
    parts.append(synth.make_queries(a, b, np.arange(50, 3000, 61, dtype=np.uint64), 333))           # plain
    q = np.concatenate(parts)
    return q[r.permutation(len(q))]


@pytest.mark.parametrize("kind,k,est,norm", [("grid", 4, 0, 0), ("normal", 4, 0, 1), ("grid", 1, 0, 0),
                                             ("normal", 3, 1, 0), ("grid", 8, 0, 1), ("normal", 16, 1, 0),
                                             ("wide", 4, 0, 0), ("ties", 4, 0, 0)])
def test_fused_triples_equal_separate_and_oracle(wmi, orc, kind, k, est, norm):
    n = 6000
    if kind == "grid":
        x, y = synth.cfg2_pair(n, 71)
    elif kind == "normal":
        x, y = synth.bivariate_normal(n, 0.7, 72)
    elif kind == "wide":  # value ranges too large for 32-bit keys: 64-bit key path
        x, y = synth.bivariate_normal(n, 0.6, 73, scale=300.0)
    else:  # few distinct values: ties at the k-th distance everywhere
        x, y = synth.grid_points(n, 74, levels=5, scale=1 / 64)
    tau = 0.08
    with wmi.Store(0) as st:
        ids = (st.add_series(x), st.add_series(y))
        q = mixed_triples(ids, n, 75)
        fused = st.evaluate(q, k=k, estimator=est, tau=tau, tau_normalize=norm)
        sep = st.evaluate(q, k=k, estimator=est, tau=tau, tau_normalize=norm, no_reuse=True)
    bits_equal(fused, sep)
    qq = q.copy()
    qq["a"], qq["b"] = 0, 1
    pick = np.random.default_rng(76).choice(len(q), 500, replace=False)
    ref = orc.batch([x, y], qq[pick], k=k, estimator=est, tau=tau, tau_normalize=norm)
    tau_eff = np.where(q["ext_side"][pick] != 0, tau * (np.log(np.maximum(q["ext_len"][pick], 1)) if norm else 1.0),
                       tau)
    oracle_close(fused[pick], ref, tau_eff)
    log(f"{kind} k={k} est={est} norm={norm}: {len(q)} queries, fused == separate bit for bit, "
        f"500 against the oracle; noise flags {int(np.count_nonzero(fused['flags'] & 1))}")


def test_all_pairs_positions_fused_equal_separate(wmi):
    """Every position of 12 pairs of the all-pairs workload."""
    w = synth.config3(pairs=[(p, (p * 7 + 5) % 64) for p in range(12)])
    with wmi.Store(0, budget_bytes=2 << 30) as st:
        ids = [st.add_series(s) for s in w.series]
        assert ids == list(range(len(w.series)))
        fused = np.concatenate([b.read() for b in st.submit_many(w.queries, k=4, tau=w.tau)])
        sep = np.concatenate([b.read() for b in st.submit_many(w.queries, k=4, tau=w.tau, no_reuse=True)])
    bits_equal(fused, sep)
    log(f"all-pairs positions: {len(w.queries)} triples fused == separate")


def test_fused_triples_count_only_union_distances(wmi):
    w = synth.config3(pairs=[(0, 40), (3, 9)])
    with wmi.Store(0) as st:
        ids = [st.add_series(s) for s in w.series]
        b = st.submit(w.queries, k=4, tau=w.tau)
        ev = b.count_evals()
        b.destroy()
        b2 = st.submit(w.queries, k=4, tau=w.tau, no_reuse=True)
        ev2 = b2.count_evals()
        b2.destroy()
    m = w.queries["len"].astype(np.int64) + w.queries["ext_len"]
    assert ev == int(np.sum(m * (m - 1)))          # the unions only
    assert ev2 == w.ordered_pairs                    # every window on its own
    log(f"distances: fused {ev}, separate {ev2} ({ev2 / ev:.2f}x)")
