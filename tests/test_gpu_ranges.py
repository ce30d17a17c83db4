"""Queries given as runs (wmi_submit_ranges: descriptors and work queue
written on the device) against the same queries submitted one by one
(wmi_submit): bit-identical results, entropies and distance counts, in every
form a batch runs in, and the oracle on samples."""
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


def mixed_ranges(wmi, n):
    """Every kind of run: small plain windows (local items), small strides
    (sweep items), windows above 512 points (split items), triples whose
    union fits a triple item, larger triples on either side, one-query and
    empty runs."""
    R = [wmi.make_ranges(0, 1, 0, (n - 64) // 8 + 1, 8, 64),            # local
         wmi.make_ranges(1, 0, 17, 300, 1, 200),                        # sweep (stride 1)
         wmi.make_ranges(0, 1, 1000, 200, 3, 96),                       # sweep (stride 3)
         wmi.make_ranges(0, 1, 5, 40, 700, 1500),                       # split
         wmi.make_ranges(0, 1, 0, 3, 9000, 4096),                       # largest windows
         wmi.make_ranges(0, 1, 0, 1500, 8, 248, 8, +1),                 # triple items
         wmi.make_ranges(1, 0, 64, 700, 16, 448, 64, -1),               # triple items, left
         wmi.make_ranges(0, 1, 3000, 30, 97, 1200, 300, +1),            # wide triples
         wmi.make_ranges(0, 1, 2048, 20, 111, 2000, 1024, -1),          # wide, all three split
         wmi.make_ranges(0, 1, 9, 1, 0, 33),                            # one query
         wmi.make_ranges(0, 1, 0, 0, 0, 100),                           # empty run
         wmi.make_ranges(0, 1, 100, 50, 2, 5, 3, +1)]                   # tiny triples (too short)
    return np.concatenate(R)


def same(a, b):
    return np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))


@pytest.mark.parametrize("no_reuse", [False, True])
def test_ranges_match_query_list(wmi, no_reuse):
    n = 40000
    x, y = synth.cfg2_pair(n, 71)
    rg = mixed_ranges(wmi, n)
    q = wmi.expand_ranges(rg)
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        b = st.submit_ranges(rg, k=4, tau=0.05, no_reuse=no_reuse)
        got = b.read()
        s = b.stats()
        for direct in (False, True, False):
            b.replay(direct=direct)
            assert same(b.read(), got)
        ev = b.count_evals()
        b.destroy()
        b2 = st.submit(q, k=4, tau=0.05, no_reuse=no_reuse)
        ref = b2.read()
        s2, ev2 = b2.stats(), b2.count_evals()
        b2.destroy()
    log(f"{len(rg)} runs, {len(q)} queries, {s['windows']} windows, {s['items']} items "
        f"(query list: {s2['items']}); distances {ev} vs {ev2}")
    assert len(got) == len(q)
    assert same(got, ref)
    assert s["windows"] == s2["windows"] and s["ordered_pairs"] == s2["ordered_pairs"]
    assert ev == ev2  # the same windows scanned the same way


def test_ranges_entropy_and_thresholds(wmi):
    n = 20000
    x, y = synth.cfg2_pair(n // 4, 72)
    x, y = np.repeat(x, 4), np.repeat(y, 4)  # held values: ties
    rg = np.concatenate([wmi.make_ranges(0, 1, 0, 500, 16, 248, 8, +1),
                         wmi.make_ranges(0, 1, 3000, 100, 5, 100),
                         wmi.make_ranges(0, 1, 600, 20, 301, 1000, 600, -1)])
    q = wmi.expand_ranges(rg)
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        for tn in (0, 1, 2):
            b = st.submit_ranges(rg, k=4, tau=0.06, tau_normalize=tn, entropy=True)
            r1, h1 = b.read(), b.read_entropy()
            b.replay()
            assert same(b.read(), r1) and same(b.read_entropy(), h1)
            b.destroy()
            b = st.submit(q, k=4, tau=0.06, tau_normalize=tn, entropy=True)
            r2, h2 = b.read(), b.read_entropy()
            b.destroy()
            assert same(r1, r2) and same(h1, h2), tn
            log(f"tau_normalize {tn}: {int(np.sum(r1['flags'] & 1))} noise of {len(q)}")


def test_all_pairs_triples_against_oracle(wmi):
    """The all-pairs noise search shape on 8 series: one run per pair."""
    series = synth.config3_series(3, n_series=8, n=8192)
    pairs = [(a, b) for a in range(8) for b in range(a + 1, 8)]
    cnt = (8192 - 256) // 8 + 1
    rg = np.concatenate([wmi.make_ranges(a, b, 0, cnt, 8, 248, 8, +1) for a, b in pairs])
    q = wmi.expand_ranges(rg)
    tau = 0.2 * np.log(256) / 4
    with wmi.Store(0) as st:
        assert [st.add_series(s) for s in series] == list(range(8))
        got = st.submit_ranges(rg, k=4, tau=tau)
        res = got.read()
        got.destroy()
        ref = st.evaluate(q, k=4, tau=tau)
    assert same(res, ref)
    pick = np.random.default_rng(73).choice(len(q), 300, replace=False)
    o = oracle.load().batch(series, q[pick], k=4, tau=tau)
    for f in ("mi_base", "mi_ext", "mi_union"):
        assert float(np.max(np.abs(res[f][pick] - o[f]))) <= TOL
    margin = np.minimum(np.abs(o["mi_ext"] - tau), np.abs(o["mi_union"] - o["mi_base"]))
    clear = margin > TOL
    assert np.array_equal(res["flags"][pick][clear], o["flags"][clear])
    log(f"{len(pairs)} runs, {len(q)} triples: identical to the query list; 300 match the oracle")


def test_range_errors(wmi):
    x, y = synth.cfg2_pair(5000, 74)
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        bad = [wmi.make_ranges(0, 1, 0, 10, 0, 100),                  # stride 0
               wmi.make_ranges(0, 1, 0, 100, 50, 100),                # last query past the end
               wmi.make_ranges(0, 1, 5, 3, 10, 100, 10, -1),          # first extension before the start
               wmi.make_ranges(0, 7, 0, 3, 10, 100),                  # unknown series
               wmi.make_ranges(0, 1, 0, 3, 10, 4000, 200, +1)]        # union above the maximum
        r = wmi.make_ranges(0, 1, 0, 3, 10, 100)
        r["pad"] = 1
        bad.append(r)
        for rg in bad:
            with pytest.raises(wmi.WmiError):
                st.submit_ranges(rg, k=4)
        b = st.submit_ranges(np.zeros(0, dtype=wmi.RANGE_DTYPE), k=4)  # nothing to do
        assert len(b.read()) == 0
        b.destroy()
