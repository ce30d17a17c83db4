"""GPU tests of the serving loop (wmi_server_*): continuous batching of range
requests.

Every window a request covers is compared with the batch entry point on the
same windows (bit-identical: both paths use the same exact integer sums) and
a sample with the CPU oracle (within 1e-9).  A request's results must not
depend on what else was in flight: alone vs. in a mix, cut across launches
or not, admitted at once or after waiting for arena space.
"""
import sys
import threading
import time

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
    return oracle.load()


N = 65536
N_SERIES = 6


@pytest.fixture(scope="module")
def series():
    out = []
    for p in range(N_SERIES // 2):
        x, y = synth.cfg2_pair(N, 40 + p)
        out += [x, y]
    return out


@pytest.fixture(scope="module")
def store(wmi, series):
    s = wmi.Store(0)
    ids = [s.add_series(v) for v in series]
    assert ids == list(range(N_SERIES))
    yield s
    s.close()


def windows_of(req):
    a, b, start, end, w, stride = req
    if end - start < w:
        return np.zeros(0, dtype=np.uint64)
    return np.arange(start, end - w + 1, stride, dtype=np.uint64)


def batch_reference(store, req, k=4, estimator=0):
    a, b, start, end, w, stride = req
    st = windows_of(req)
    if len(st) == 0:
        return np.zeros(0), np.zeros(0, dtype=np.uint32)
    r = store.evaluate(synth.make_queries(a, b, st, w), k=k, estimator=estimator)
    return r["mi_base"], r["flags"]


def same(got, ref_mi, ref_fl):
    assert len(got) == len(ref_mi)
    assert np.array_equal(got["flags"], ref_fl)
    assert np.array_equal(np.isnan(got["mi"]), np.isnan(ref_mi))
    ok = ~np.isnan(ref_mi)
    assert np.array_equal(got["mi"][ok], ref_mi[ok])  # bit-identical


def run_requests(server, reqs):
    tickets = [server.submit(*r) for r in reqs]
    out = []
    for t in tickets:
        server.wait(t, 60_000_000)
        out.append(server.read(t))
    return out


MIX = [
    # (a, b, start, end, w, stride)
    (0, 1, 0, N, 128, 16),
    (2, 3, 1000, 40000, 32, 8),
    (1, 4, 0, N, 4096, 512),
    (5, 0, 7, 30007, 513, 64),
    (3, 2, 12345, 50000, 2048, 256),
    (4, 5, 0, 3000, 4, 1),        # w <= k: NaN, TOO_SHORT
    (0, 3, 500, 600, 200, 1),     # range shorter than w: no windows
    (2, 5, 0, N, 1, 4096),        # one-point windows
    (1, 1, 100, 20000, 511, 37),  # a series with itself
    (3, 4, 0, N, 512, 1000),
    (4, 2, 60000, N, 64, 1),
    (0, 5, 0, N, 1000, 333),
]


def test_server_matches_batch_and_oracle(wmi, store, series, orc):
    with wmi.Server(store, k=4) as srv:
        res = run_requests(srv, MIX)
        st = srv.stats()
    log(f"server stats {st}")
    assert st["requests_done"] == len(MIX)
    for req, (got, info) in zip(MIX, res):
        log(f"request {req}: {info['windows']} windows over {info['launches']} launches")
        assert info["windows"] == len(windows_of(req)) and info["state"] == 2
        ref_mi, ref_fl = batch_reference(store, req)
        same(got, ref_mi, ref_fl)
        # oracle on a sample of windows
        a, b, start, end, w, stride = req
        starts = windows_of(req)
        if len(starts) == 0:
            continue
        pick = np.unique(np.linspace(0, len(starts) - 1, 3).astype(int))
        for i in pick:
            s0 = int(starts[i])
            mi = orc.window_mi(series[a][s0:s0 + w], series[b][s0:s0 + w], k=4)
            if np.isnan(mi):
                assert np.isnan(got["mi"][i]) and got["flags"][i] == wmi.F_TOO_SHORT
            else:
                assert abs(got["mi"][i] - mi) <= TOL, (req, i, got["mi"][i], mi)
                assert got["flags"][i] == 0


def test_alone_vs_mix(wmi, store):
    """Each request alone on an idle server, then all of them submitted
    together (overlapping on the device, several per launch, cut across
    launches): results bit-identical."""
    with wmi.Server(store, k=4) as srv:
        alone = []
        for r in MIX:
            alone += run_requests(srv, [r])
    with wmi.Server(store, k=4, max_launch_windows=3000) as srv:
        mixed = run_requests(srv, MIX[::-1])[::-1]
        st = srv.stats()
    log(f"mix stats {st}")
    multi = 0
    for req, (g1, i1), (g2, i2) in zip(MIX, alone, mixed):
        assert np.array_equal(g1["flags"], g2["flags"]), req
        assert np.array_equal(g1["mi"].view(np.uint64), g2["mi"].view(np.uint64)), req
        multi += i2["launches"] > 1
    assert multi >= 3  # long requests were cut across launches


def test_arrivals_while_busy(wmi, store):
    """Requests submitted from another thread while launches run join later
    launches; every result still equals the batch entry point's."""
    rng = np.random.default_rng(7)
    reqs = []
    for _ in range(60):
        w = int(np.exp(rng.uniform(np.log(32), np.log(2048))))
        a = int(rng.integers(0, N_SERIES))
        b = int((a + rng.integers(1, N_SERIES)) % N_SERIES)
        start = int(rng.integers(0, N // 2))
        reqs.append((a, b, start, N, w, max(w // 8, 1)))
    tickets = [None] * len(reqs)
    with wmi.Server(store, k=4, max_launch_windows=8192) as srv:
        def producer():
            for i, r in enumerate(reqs):
                tickets[i] = srv.submit(*r)
                time.sleep(0.0001 * (i % 3))

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        res = []
        for t in tickets:
            srv.wait(t, 60_000_000)
            res.append(srv.read(t))
        st = srv.stats()
    log(f"arrival stats {st}")
    assert st["requests_done"] == len(reqs)
    overlap = 0
    for i, (req, (got, info)) in enumerate(zip(reqs, res)):
        ref_mi, ref_fl = batch_reference(store, req)
        same(got, ref_mi, ref_fl)
        assert info["t_arrival_us"] <= info["t_admit_us"] <= info["t_first_launch_us"] <= info["t_complete_us"]
        overlap += any(o["t_arrival_us"] < info["t_arrival_us"] < o["t_complete_us"]
                       for _, o in res[:i])
    # launches each request would need on its own (cut at the launch cap);
    # sharing launches can only lower the count (how much depends on timing)
    alone = sum(-(-len(got) // 8192) for got, _ in res)
    log(f"{overlap} requests arrived while an earlier one was still running; "
        f"{st['launches']} launches against {alone} for the requests one by one")
    assert overlap > 0
    assert st["launches"] <= alone


def test_admission_by_arena(wmi, store):
    """A 256 KiB arena holds few requests at once: the rest wait in arrival
    order, and the results are unchanged."""
    reqs = [(i % N_SERIES, (i + 1) % N_SERIES, 0, N, 64, 8) for i in range(12)]  # 8185 windows, 128 KiB each
    with wmi.Server(store, k=4, hbm_budget_bytes=256 << 10) as srv:
        res = run_requests(srv, reqs)
        st = srv.stats()
    log(f"admission stats {st}")
    assert st["queued_peak"] >= 1
    assert st["arena_peak_bytes"] <= st["arena_bytes"] == 256 << 10
    admits = [info["t_admit_us"] for _, info in res]
    assert admits == sorted(admits)  # first come, first admitted
    for req, (got, _) in zip(reqs, res):
        ref_mi, ref_fl = batch_reference(store, req)
        same(got, ref_mi, ref_fl)


def test_other_estimator_and_k(wmi, store, series, orc):
    req = (2, 3, 5000, 25000, 300, 97)
    for k, est in ((1, 0), (7, 1), (16, 0)):
        with wmi.Server(store, k=k, estimator=est) as srv:
            (got, info), = run_requests(srv, [req])
        ref_mi, ref_fl = batch_reference(store, req, k=k, estimator=est)
        same(got, ref_mi, ref_fl)
        s0 = int(windows_of(req)[5])
        mi = orc.window_mi(series[2][s0:s0 + 300], series[3][s0:s0 + 300], k=k, estimator=est)
        assert abs(got["mi"][5] - mi) <= TOL


def test_errors(wmi, store):
    W = wmi
    with W.Server(store, k=4, hbm_budget_bytes=64 << 10) as srv:
        bad = [
            ((0, 99, 0, 100, 10, 1), W.WMI_EINVAL),      # unknown series
            ((0, 1, 0, 100, 0, 1), W.WMI_EINVAL),        # w = 0
            ((0, 1, 0, 10000, 4097, 1), W.WMI_EINVAL),   # w > 4096
            ((0, 1, 0, 100, 10, 0), W.WMI_EINVAL),       # stride 0
            ((0, 1, 0, N + 1, 10, 1), W.WMI_EINVAL),     # end beyond the series
            ((0, 1, 50, 40, 10, 1), W.WMI_EINVAL),       # end before start
            ((0, 1, 0, N, 32, 1), W.WMI_ENOMEM),         # 65505 windows > 64 KiB arena
        ]
        for req, code in bad:
            with pytest.raises(W.WmiError) as e:
                srv.submit(*req)
            assert e.value.code == code, (req, e.value)
        with pytest.raises(W.WmiError) as e:
            srv.info(12345)
        assert e.value.code == W.WMI_EINVAL
        # a pending request's series cannot be removed
        extra = store.add_series(np.zeros(N, dtype=np.float32) + 0.25)
        t = srv.submit(extra, 1, 0, N, 4096, 64)
        try:
            store.remove_series(extra)
            removed = True
        except W.WmiError as err:
            removed = False
            assert err.code == W.WMI_EBUSY
        srv.wait(t, 60_000_000)
        got, info = srv.read(t)
        assert info["windows"] == len(got) == (N - 4096) // 64 + 1
        if not removed:
            store.remove_series(extra)  # finished: no longer pinned
        with pytest.raises(W.WmiError):
            srv.read(t)  # ticket forgotten after read


def test_two_hundred_requests_alone_mix_oracle(wmi, store, series, orc):
    """The serving workload's request shape (random pair, w log-uniform in
    [32, 2048], stride w/4) on resident series: 200 requests, each alone on an
    idle server and all of them in flight together, bit-identical; every
    window equal to the batch entry point's; one window of each against the
    oracle."""
    r = np.random.default_rng(404)
    reqs = []
    for _ in range(200):
        w = int(np.rint(np.exp(r.uniform(np.log(32), np.log(2048)))))
        a = int(r.integers(0, N_SERIES))
        b = int((a + r.integers(1, N_SERIES)) % N_SERIES)
        start = int(r.integers(0, N // 4))
        reqs.append((a, b, start, N, w, max(w // 4, 1)))
    with wmi.Server(store, k=4) as srv:
        alone = [run_requests(srv, [q])[0] for q in reqs]
    with wmi.Server(store, k=4, max_launch_windows=16384) as srv:
        mixed = run_requests(srv, reqs)
        st = srv.stats()
    log(f"200-request mix: {st}")
    assert st["launches"] < len(reqs)
    # the batch entry point on every window of every request, in one batch
    qs = [synth.make_queries(q[0], q[1], windows_of(q), q[4]) for q in reqs]
    ref = store.evaluate(np.concatenate(qs), k=4)
    off = 0
    for i, (req, (g1, _), (g2, _)) in enumerate(zip(reqs, alone, mixed)):
        assert np.array_equal(g1["mi"].view(np.uint64), g2["mi"].view(np.uint64)), req
        assert np.array_equal(g1["flags"], g2["flags"]), req
        n = len(g1)
        same(g1, ref["mi_base"][off:off + n], ref["flags"][off:off + n])
        off += n
        j = int(r.integers(0, n))
        s0 = int(windows_of(req)[j])
        mi = orc.window_mi(series[req[0]][s0:s0 + req[4]], series[req[1]][s0:s0 + req[4]], k=4)
        assert abs(g1["mi"][j] - mi) <= TOL, (req, j, g1["mi"][j], mi)
