"""Window entropies on the GPU (WMI_SUBMIT_ENTROPY, the denominator of the
normalised MI of Section 5.4) and the thresholds that take them
(tau_normalize 2; normalize 2 in the search drivers), against the oracle's
empirical entropy of the window's pairs.

Inputs with many exact ties (values held for several samples, or drawn from
a few levels) so that H differs from ln m; H within 1e-12 of the oracle
(the device sums ln c in 2^-44 fixed point, the oracle p ln p in double);
flags exact where the extension's estimate is more than 1e-9 away from its
threshold."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import search
from paper_2204_09131_amd import synth

pytestmark = pytest.mark.gpu

H_TOL = 1e-12
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


def held_pair(n, seed, hold):
    """The multi-scale segment pair on n / hold samples, each value held for
    `hold` samples (a sensor read more often than it changes): runs of equal
    pairs, so a window's entropy is near ln(m / hold)."""
    x, y = synth.cfg2_pair(-(-n // hold), seed)
    return np.repeat(x, hold)[:n].copy(), np.repeat(y, hold)[:n].copy()


def level_pair(n, seed, levels):
    """Values from a few grid levels, y partly following x: many repeated
    pairs at any window size."""
    r = np.random.default_rng(seed)
    x = r.integers(0, levels, n)
    y = np.where(r.random(n) < 0.6, x, r.integers(0, levels, n))
    return (x / 8.0).astype(np.float32), (y / 8.0).astype(np.float32)


def window_list(q):
    """(query, slot, start, m) of every window of the queries."""
    out = []
    for i, r in enumerate(q):
        s, m, e, side = int(r["start"]), int(r["len"]), int(r["ext_len"]), int(r["ext_side"])
        out.append((i, 0, s, m))
        if side:
            es = s + m if side > 0 else s - e
            out.append((i, 1, es, e))
            out.append((i, 2, min(s, es), m + e))
    return out


def mixed_queries(n, seed):
    r = np.random.default_rng(seed)
    q = [synth.make_queries(0, 1, np.array([0, 5, n - 4096], dtype=np.uint64), 4096),   # largest windows
         synth.make_queries(0, 1, np.array([3, 100], dtype=np.uint64), 1),               # one point
         synth.make_queries(0, 1, np.array([7], dtype=np.uint64), 2)]
    for m in (17, 64, 129, 500, 1500):
        q.append(synth.make_queries(0, 1, np.sort(r.choice(n - m, 40, replace=False)).astype(np.uint64), m))
    for base, ext, side in ((248, 8, 1), (96, 32, -1), (448, 64, 1), (3000, 1096, 1), (60, 4, -1)):
        lo = ext if side < 0 else 0
        starts = np.sort(r.choice(np.arange(lo, n - base - ext), 30, replace=False)).astype(np.uint64)
        q.append(synth.make_queries(0, 1, starts, base, ext, side))
    return np.concatenate(q)


@pytest.mark.parametrize("kind", ["held", "levels"])
def test_entropies_match_oracle(wmi, orc, kind):
    n = 20000
    x, y = held_pair(n, 41, 4) if kind == "held" else level_pair(n, 42, 5)
    q = mixed_queries(n, 43)
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        b = st.submit(q, k=4, tau=0.05, entropy=True)
        res, h = b.read(), b.read_entropy()
        b.destroy()
        plain = st.evaluate(q, k=4, tau=0.05)
    # the entropy pass leaves the estimates alone
    assert np.array_equal(res.view(np.uint8), plain.view(np.uint8))
    worst, below = 0.0, 0
    for i, slot, s, m in window_list(q):
        ref = orc.window_entropy(x[s:s + m], y[s:s + m])
        worst = max(worst, abs(h[i, slot] - ref))
        below += ref < math.log(m) - 1e-9
    nan_expected = np.array([[False, r["ext_side"] == 0, r["ext_side"] == 0] for r in q])
    assert np.array_equal(np.isnan(h), nan_expected)
    log(f"{kind}: {len(window_list(q))} windows, {below} with ties (H < ln m); max |H - oracle| {worst:.3g}")
    assert worst <= H_TOL
    assert below > len(q) // 2


def test_entropy_threshold_flags(wmi, orc):
    """tau_normalize 2: noise iff I(w_o) > 0, I(w_d) < tau H(w_d) and
    I(w'') < I(w_o); H from ties differs from ln|w_d|, so the flags of the
    two readings part on some triples."""
    n = 40000
    x, y = held_pair(n, 44, 4)
    r = np.random.default_rng(45)
    q = []
    for base, ext, side in ((248, 8, 1), (120, 8, -1), (448, 64, 1), (200, 56, 1)):
        lo = ext if side < 0 else 0
        starts = np.sort(r.choice(np.arange(lo, n - base - ext), 400, replace=False)).astype(np.uint64)
        q.append(synth.make_queries(0, 1, starts, base, ext, side))
    q = np.concatenate(q)
    parted = 0
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        for tau in (0.02, 0.06, 0.15):
            got = st.evaluate(q, k=4, tau=tau, tau_normalize=2)
            ln = st.evaluate(q, k=4, tau=tau, tau_normalize=1)
            ref = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=2)
            for f in ("mi_base", "mi_ext", "mi_union"):
                assert np.max(np.abs(got[f] - ref[f])) <= TOL
            hd = np.array([orc.window_entropy(x[s:s + m], y[s:s + m]) for i, sl, s, m in window_list(q) if sl == 1])
            clear = np.abs(ref["mi_ext"] - tau * hd) > TOL
            assert np.array_equal(got["flags"][clear], ref["flags"][clear])
            parted += int(np.sum((got["flags"] ^ ln["flags"]) & wmi.F_NOISE))
            log(f"tau {tau}: {int(np.sum(ref['flags'] & 1))} noise of {len(q)}; {int(np.sum(~clear))} near the "
                f"threshold; flags differing from tau ln|w_d| so far {parted}")
    assert parted > 0


def test_entropy_replay_plain_and_noalloc(wmi, orc):
    """The entropy pass in every form a batch runs in: graph replays,
    direct replays, the launch-per-window form, and the allocation-free
    entry point (thresholds only)."""
    import torch
    n = 12000
    x, y = held_pair(n, 46, 3)
    q = mixed_queries(n, 47)
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        b = st.submit(q, k=4, tau=0.07, tau_normalize=2, entropy=True)
        r0, h0 = b.read(), b.read_entropy()
        for direct in (False, False, True, False):
            b.replay(direct=direct)
            st.evaluate(q[:50], k=4)  # other work between the runs
            r1, h1 = b.read(), b.read_entropy()
            assert np.array_equal(r1.view(np.uint8), r0.view(np.uint8))
            assert np.array_equal(h1.view(np.uint64), h0.view(np.uint64))
        b.destroy()
        bp = st.submit(q, k=4, tau=0.07, tau_normalize=2, entropy=True, plain=True)
        assert np.array_equal(bp.read().view(np.uint8), r0.view(np.uint8))
        assert np.array_equal(bp.read_entropy().view(np.uint64), h0.view(np.uint64))
        bp.destroy()
        d = torch.zeros(len(q) * 4, dtype=torch.float64, device="cuda")
        st.submit_noalloc(q, d.data_ptr(), k=4, tau=0.07, tau_normalize=2)
        got = d.cpu().numpy().view(wmi.RESULT_DTYPE)
        assert np.array_equal(got.view(np.uint8), r0.view(np.uint8))
        b = st.submit(q[:10], k=4)
        with pytest.raises(wmi.WmiError):
            b.read_entropy()  # not asked for
        b.destroy()
        with pytest.raises(wmi.WmiError):
            st.submit(q[:10], k=4, tau_normalize=3)
    ref = orc.batch([x, y], q, k=4, tau=0.07, tau_normalize=2)
    assert np.max(np.abs(r0["mi_union"] - ref["mi_union"])[~np.isnan(ref["mi_union"])]) <= TOL


def oracle_with_entropy(orc, x, y, k=4):
    """The oracle's estimate and entropy of a window, cached.  Held values
    repeat whole windows' structure, so distinct windows can have equal
    estimates; the oracle's double sums leave them a few ulps apart in an
    order-dependent way, while the device's exact fixed-point sums make them
    bit-equal.  The estimates are therefore rounded to 2^-40 here, so that
    a comparison between equal estimates is a tie on both sides."""
    cache_mi, cache_h = {}, {}

    def mi(s, m):
        if (s, m) not in cache_mi:
            v = orc.window_mi(x[s:s + m], y[s:s + m], k=k)
            cache_mi[(s, m)] = v if math.isnan(v) else round(v * 2.0 ** 40) / 2.0 ** 40
        return cache_mi[(s, m)]

    def ent(s, m):
        if (s, m) not in cache_h:
            cache_h[(s, m)] = orc.window_entropy(x[s:s + m], y[s:s + m])
        return cache_h[(s, m)]
    return mi, ent, cache_mi, cache_h


@pytest.mark.parametrize("case", [
    # (seed, n, hold, s_max, s_min, sigma, tau, p, step_div)
    (51, 12000, 4, 512, 64, 0.25, 0.06, 0, 8),
    (52, 12000, 3, 512, 32, 0.20, 0.05, 1, 8),
])
def test_td_driver_entropy_thresholds(wmi, orc, case):
    seed, n, hold, s_max, s_min, sigma, tau, p, div = case
    x, y = held_pair(n, seed, hold)
    with wmi.Store(0) as st:
        a, b = st.add_series(x), st.add_series(y)
        got, stats = st.td_search(a, b, 0, n, s_max, s_min, sigma, tau=tau, p=p, step_div=div, normalize=2)
        got1, _ = st.td_search(a, b, 0, n, s_max, s_min, sigma, tau=tau, p=p, step_div=div, normalize=1)
    mi, ent, cm, ch = oracle_with_entropy(orc, x, y)
    ref = search.top_down(mi, 0, n, s_max, s_min, sigma, tau=tau, p=p, step_div=div, normalize=2, entropy=ent)
    # decisions within 1e-9 of a threshold could go either way
    margins = [min(abs(v - sigma * ch[(s, m)]), abs(v - tau * ch[(s, m)])) for (s, m), v in cm.items()
               if (s, m) in ch and not math.isnan(v)]
    log(f"td case {case}: {len(ref)} windows (ln-normalised: {len(got1)}); stats {stats}; "
        f"closest margin {min(margins):.3g}")
    assert min(margins) > TOL
    assert [(int(s), int(m), int(l)) for s, m, l, _ in ref] == \
        [(int(r["start"]), int(r["len"]), int(r["layer"])) for r in got]
    if len(ref):
        assert np.max(np.abs(np.array([v for *_, v in ref]) - got["mi"])) <= TOL


@pytest.mark.parametrize("case", [
    # (seed, n, hold, chunk, s_min, s_max, delta, max_idle, history, sigma, tau, p, rng seed)
    (61, 4096, 4, 1024, 32, 256, 16, 2, 4, 0.25, 0.06, 2, 3),
    (62, 6000, 2, 1500, 48, 384, 24, 1, 3, 0.12, 0.04, 1, 4),
])
def test_bu_driver_entropy_thresholds(wmi, orc, case):
    seed, n, hold, chunk, s_min, s_max, delta, idle, h, sigma, tau, p, rs = case
    x, y = held_pair(n, seed, hold)
    kw = dict(s_min=s_min, s_max=s_max, delta=delta, sigma=sigma, max_idle=idle, history=h, tau=tau, p=p,
              normalize=2, chunk=chunk, seed=rs)
    with wmi.Store(0) as st:
        a, b = st.add_series(x), st.add_series(y)
        got, stats = st.bu_search(a, b, 0, n, **kw)
    mi, ent, cm, ch = oracle_with_entropy(orc, x, y)
    ref = search.bottom_up(mi, 0, n, entropy=ent, **kw)
    vals = np.sort(np.array([v for v in cm.values() if not math.isnan(v)]))
    assert np.min(np.diff(np.unique(vals))) > TOL
    log(f"bu case {case}: {len(ref)} windows; stats {stats}")
    assert [(int(s), int(m)) for s, m, _, _ in ref] == [(int(r["start"]), int(r["len"])) for r in got]
    if len(ref):
        assert np.max(np.abs(np.array([v for *_, v in ref]) - got["mi"])) <= TOL
