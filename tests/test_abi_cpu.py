"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
header declares, its host-built digamma table agrees with the oracle's
independent construction, and it fails cleanly without a GPU.  No compute
call is made here."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wmi.h")


@pytest.fixture(scope="module")
def wmi():
    from paper_2204_09131_amd import wmi as w
    if not os.path.exists(w.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return w


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wmi_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported(wmi):
    names = header_functions()
    assert len(names) >= 17
    lib = wmi.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(wmi.EXPORTS) == names


def test_version(wmi):
    assert wmi.version() == (0, 1)


def test_psi_table_matches_oracle(wmi, orc):
    n = 8192
    lib_tab = wmi.psi_table(n)
    ora_tab = orc.psi_table(n)
    assert np.max(np.abs(lib_tab - ora_tab)) <= 1e-14


def test_psi_table_bounds(wmi):
    with pytest.raises(wmi.WmiError) as e:
        wmi.psi_table(8193)
    assert e.value.code == wmi.WMI_EINVAL


def test_query_layout_matches_generator(wmi):
    from paper_2204_09131_amd import synth
    assert synth.QUERY_DTYPE.itemsize == wmi.QUERY_DTYPE.itemsize == 32
    assert synth.QUERY_DTYPE.descr == wmi.QUERY_DTYPE.descr


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_store_create_without_gpu(wmi):
    with pytest.raises(wmi.WmiError) as e:
        wmi.Store(0)
    assert e.value.code in (wmi.WMI_EHIP, wmi.WMI_EINVAL)


def test_missing_library_fails_loudly(wmi, monkeypatch):
    monkeypatch.setattr(wmi, "_lib", None)
    monkeypatch.setattr(wmi, "LIB_PATH", "/nonexistent/libwmi.so")
    with pytest.raises(ImportError):
        wmi.lib()


def test_product_path_does_not_touch_oracle():
    pkg = os.path.join(ROOT, "paper_2204_09131_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ksg_oracle" not in text, f
