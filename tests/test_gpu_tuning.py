"""The same workloads under several work-list choices (wmi_tuning: windows
per local item, triples per triple item, windows per sweep item, straggler
thresholds), including the autotuner's file when there is one: results must
be bit-identical across choices (every choice is a schedule of the same exact
arithmetic, so a difference would expose a race between work items) and
match the oracle on samples."""
import json
import os
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


SMALL = {"local_windows": [1, 1, 1, 1, 1], "triples": [1, 1, 1, 1, 1], "sweep_windows": [2, 2, 2],
         "stragglers": [0, 0, 0]}
MIXED = {"local_windows": [3, 5, 2, 2, 1], "triples": [2, 4, 3, 1, 1], "sweep_windows": [3, 37, 13],
         "stragglers": [64, 1, 128]}


def tunings(wmi):
    out = [("default", None), ("small", SMALL), ("mixed", MIXED)]
    path = wmi.tuning_file(0)
    if os.path.exists(path):
        out.append(("autotuned", json.load(open(path))["tuning"]))
    return out


def workload():
    """A mix of every item kind: the multi-scale windows (local and split
    items), noise triples of several shapes (triple items), stride-1 and
    stride-2 runs (sweep items)."""
    w2 = synth.config2()
    q = [w2.queries]
    r = np.random.default_rng(95)
    for base, ext, side in ((248, 8, +1), (56, 8, +1), (96, 32, -1), (448, 64, +1)):
        lo = ext if side < 0 else 0
        starts = np.sort(r.choice(np.arange(lo, 60000 - base - ext), 300, replace=False)).astype(np.uint64)
        q.append(synth.make_queries(0, 1, starts, base, ext, side))
    q.append(synth.make_queries(0, 1, np.arange(1000, 3000, dtype=np.uint64), 128))
    q.append(synth.make_queries(0, 1, np.arange(7000, 9000, 2, dtype=np.uint64), 64))
    q.append(synth.make_queries(0, 1, np.arange(20000, 21500, 3, dtype=np.uint64), 200))
    return w2.series, np.concatenate(q)


def test_results_identical_under_every_tuning(wmi):
    series, q = workload()
    results = {}
    for name, t in tunings(wmi):
        with wmi.Store(0, tuning=t) as st:
            assert [st.add_series(s) for s in series] == [0, 1]
            if t is not None:
                got = st.get_tuning()
                for f, v in t.items():
                    assert got[f] == list(v), (name, f)
            results[name] = st.evaluate(q, k=4, tau=0.05)
        log(f"tuning {name}: {len(q)} queries evaluated")
    ref = results["default"]
    for name, r in results.items():
        assert np.array_equal(r.view(np.uint8), ref.view(np.uint8)), name
    pick = np.random.default_rng(96).choice(len(q), 400, replace=False)
    orc = oracle.load()
    o = orc.batch(series, q[pick], k=4, tau=0.05)
    for f in ("mi_base", "mi_ext", "mi_union"):
        a, b = ref[f][pick], o[f]
        assert np.array_equal(np.isnan(a), np.isnan(b))
        ok = ~np.isnan(b)
        assert float(np.max(np.abs(a[ok] - b[ok]))) <= TOL
    log(f"{len(results)} tunings bit-identical; 400 queries match the oracle")


def test_server_under_other_tuning(wmi):
    x, y = synth.cfg2_pair(65536, 97)
    reqs = [(0, 1, 0, 65536, 32, 8), (1, 0, 100, 60000, 700, 175), (0, 1, 5, 50000, 2048, 512)]
    with wmi.Store(0, tuning=MIXED) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        with wmi.Server(st, k=4) as srv:
            tickets = [srv.submit(*r) for r in reqs]
            got = []
            for t in tickets:
                srv.wait(t, 60_000_000)
                got.append(srv.read(t)[0])
    with wmi.Store(0) as st:
        assert [st.add_series(x), st.add_series(y)] == [0, 1]
        for r, g in zip(reqs, got):
            a, b, s0, e0, w, sd = r
            ref = st.evaluate(synth.make_queries(a, b, np.arange(s0, e0 - w + 1, sd, dtype=np.uint64), w), k=4)
            assert np.array_equal(g["mi"].view(np.uint64), ref["mi_base"].view(np.uint64))


def test_bad_tuning_rejected(wmi):
    with wmi.Store(0) as st:
        for bad in ({"local_windows": [0, 1, 1, 1, 1]}, {"triples": [6, 1, 1, 1, 1]},
                    {"sweep_windows": [0, 2, 2]}, {"sweep_windows": [2, 2, 256]}, {"stragglers": [0, 0, 129]}):
            with pytest.raises(wmi.WmiError):
                st.set_tuning(bad)
        st.set_tuning(None)
        assert st.get_tuning()["local_windows"] == [16] * 5


def test_kernel_variants_agree(wmi):
    """Queues of local and triple items run on the lighter compilation of the
    main kernel (more workgroups per CU); adding one large window moves the
    same queries onto the general one.  Results must be bit-identical."""
    series, q = workload()
    small = q[(q["len"] + q["ext_len"]) <= 512]
    small = small[small["ext_side"] != 0][:3000]
    small = np.concatenate([small, q[(q["ext_side"] == 0) & (q["len"] <= 256)][:3000]])
    big = synth.make_queries(0, 1, np.array([100], dtype=np.uint64), 2000)
    with wmi.Store(0) as st:
        assert [st.add_series(s) for s in series] == [0, 1]
        for k in (4, 3):
            b1 = st.submit(small, k=k, tau=0.05)
            r1, s1 = b1.read(), b1.stats()
            b1.destroy()
            b2 = st.submit(np.concatenate([small, big]), k=k, tau=0.05)
            r2, s2 = b2.read(), b2.stats()
            b2.destroy()
            assert np.array_equal(r1.view(np.uint8), r2[:len(small)].view(np.uint8))
            assert s1["wg_per_cu"] > s2["wg_per_cu"], (s1["wg_per_cu"], s2["wg_per_cu"])
            log(f"k={k}: {len(small)} queries, {s1['wg_per_cu']} vs {s2['wg_per_cu']} workgroups per CU, identical")
