"""The allocation-free entry point (wmi_submit_noalloc) against wmi_submit on
the same queries: two calls in a row through the C-ABI, the second smaller,
each result bit-identical (both paths sum the same exact integers), plus the
size limit of its static scratch array."""
import sys

import numpy as np
import pytest

from paper_2204_09131_amd import synth

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_09131_amd import wmi
    wmi.lib()
    st = wmi.Store(0)
    w2 = synth.config2()
    w1 = synth.config1()
    ids2 = [st.add_series(s) for s in w2.series]
    ids1 = [st.add_series(s) for s in w1.series]
    yield wmi, st, w2, ids2, w1, ids1
    st.close()


def noalloc(wmi, st, q, **kw):
    import torch
    out = torch.empty(len(q) * wmi.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    out.fill_(0xA5)  # results must overwrite whatever was there
    st.submit_noalloc(q, out.data_ptr(), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(wmi.RESULT_DTYPE)


def same(a, b):
    assert np.array_equal(a.view(np.uint8).reshape(len(a), -1)[:, :28], b.view(np.uint8).reshape(len(b), -1)[:, :28])


def test_noalloc_matches_submit_two_calls(env):
    wmi, st, w2, ids2, w1, ids1 = env
    # call 1: every window of the multi-scale workload (32,584 windows, 875 of
    # them above 512 points), k = 4
    q1 = w2.queries.copy()
    q1["a"], q1["b"] = ids2
    log(f"noalloc call 1: {len(q1)} queries")
    got1 = noalloc(wmi, st, q1, k=4)
    same(got1, st.evaluate(q1, k=4))
    # call 2, smaller: noise triples of the plain workload, k = 3, normalised tau
    q2 = np.concatenate([synth.make_queries(ids1[0], ids1[1], np.arange(200, 3600, 17, dtype=np.uint64), 120, 8, +1),
                         synth.make_queries(ids1[0], ids1[1], np.arange(100, 3400, 23, dtype=np.uint64), 600, 40, -1)])
    log(f"noalloc call 2: {len(q2)} queries")
    got2 = noalloc(wmi, st, q2, k=3, tau=0.05, tau_normalize=1)
    ref2 = st.evaluate(q2, k=3, tau=0.05, tau_normalize=1)
    same(got2, ref2)
    assert np.any(ref2["flags"] & wmi.F_NOISE) or np.any(~np.isnan(ref2["mi_union"]))
    log("noalloc: both calls bit-identical with wmi_submit")


def test_noalloc_rejects_calls_beyond_its_scratch(env):
    wmi, st, w2, ids2, _, _ = env
    # 1600 windows of 4096 points need 12 B per point of sorted data: 79 MB
    q = synth.make_queries(ids2[0], ids2[1], np.arange(1600, dtype=np.uint64) * 37, 4096)
    with pytest.raises(wmi.WmiError) as e:
        st.submit_noalloc(q, 1 << 40)  # never dereferenced: the size check comes first
    assert e.value.code == wmi.WMI_ENOMEM
    # and the store is still usable
    q3 = synth.make_queries(ids2[0], ids2[1], np.arange(10, dtype=np.uint64) * 999, 700)
    got = noalloc(wmi, st, q3, k=4)
    same(got, st.evaluate(q3, k=4))
