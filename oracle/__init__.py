"""CPU oracle for windowed KSG mutual information -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it, and
it shares no code with the GPU path: the arithmetic lives in ``ksg_oracle.c``
(plain C, double precision, no fast-math), loaded here through ctypes.

Parity status of each function (what pins it is in ``tests/test_oracle_pins.py``):
  psi_table      pinned: exact rational harmonic numbers, scipy digamma
  window_counts  pinned: the worked example of Section 7.1.1, brute force with a
                 full sort, scipy's k-d tree on tie-free data, closed forms
  window_mi      pinned: closed form for y = x, bivariate-normal closed form
                 within sampling error, independence, scikit-learn's
                 first-estimator KSG (estimator 1), symmetry and invariances
  batch          pinned: equals window_mi per window; noise flag by the
                 constructed cases of Definition 6.2
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ksg_oracle.c")
LIB = os.path.join(HERE, "libksg_oracle.so")

FLAG_NOISE = 1
FLAG_TOO_SHORT = 2
FLAG_NONPOS_BASE = 4
FLAG_OFFGRID = 8

RESULT_DTYPE = np.dtype([("mi_base", "<f8"), ("mi_ext", "<f8"), ("mi_union", "<f8"),
                         ("flags", "<u4"), ("pad", "<u4")])


def compile_oracle(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile the oracle with gcc (no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        lib.oracle_psi.restype = ctypes.c_double
        lib.oracle_psi.argtypes = [ctypes.c_long]
        lib.oracle_psi_table.restype = ctypes.c_int
        lib.oracle_psi_table.argtypes = [ctypes.c_int, P(ctypes.c_double)]
        lib.oracle_window_counts.restype = ctypes.c_int
        lib.oracle_window_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
        lib.oracle_window_mi.restype = ctypes.c_double
        lib.oracle_window_mi.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int]
        lib.oracle_batch.restype = ctypes.c_int
        lib.oracle_window_entropy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_window_entropy.restype = ctypes.c_double
        lib.oracle_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_void_p]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
        self.lib = lib
        self.path = path

    # -- psi --------------------------------------------------------------
    def psi(self, n: int) -> float:
        return self.lib.oracle_psi(int(n))

    def psi_table(self, n_max: int) -> np.ndarray:
        out = np.empty(n_max, dtype=np.float64)
        rc = self.lib.oracle_psi_table(int(n_max), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if rc != 0:
            raise ValueError("n_max out of range")
        return out

    # -- one window -------------------------------------------------------
    def window_counts(self, x, y, k: int = 4, estimator: int = 0) -> dict:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        m = x.shape[0]
        assert y.shape[0] == m
        nx = np.zeros(m, dtype=np.uint32)
        ny = np.zeros(m, dtype=np.uint32)
        ex = np.zeros(m, dtype=np.float64)
        ey = np.zeros(m, dtype=np.float64)
        nbr = np.zeros((m, max(k, 1)), dtype=np.int32)
        rc = self.lib.oracle_window_counts(x.ctypes.data, y.ctypes.data, m, k, estimator,
                                           nx.ctypes.data, ny.ctypes.data, ex.ctypes.data,
                                           ey.ctypes.data, nbr.ctypes.data)
        if rc != 0:
            raise ValueError("window too short or k out of range")
        return {"nx": nx, "ny": ny, "eps_x": ex, "eps_y": ey, "nbr": nbr}

    def window_mi(self, x, y, k: int = 4, estimator: int = 0) -> float:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        return self.lib.oracle_window_mi(x.ctypes.data, y.ctypes.data, x.shape[0], k, estimator)

    def window_entropy(self, x, y) -> float:
        """Empirical entropy of the window's pairs (Section 5.4), natural log."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        assert x.shape == y.shape
        return self.lib.oracle_window_entropy(x.ctypes.data, y.ctypes.data, x.shape[0])

    # -- batches ----------------------------------------------------------
    def batch(self, series, queries, k: int = 4, estimator: int = 0, tau: float = 0.0,
              tau_normalize: int = 0, threads: int = 0) -> np.ndarray:
        series = [np.ascontiguousarray(s, dtype=np.float32) for s in series]
        ptrs = (ctypes.c_void_p * len(series))(*[s.ctypes.data for s in series])
        q = np.ascontiguousarray(queries)
        assert q.dtype.itemsize == 32
        for name in ("a", "b"):
            if len(q) and int(q[name].max()) >= len(series):
                raise ValueError("series id out of range")
        out = np.zeros(len(q), dtype=RESULT_DTYPE)
        if threads:
            self.lib.oracle_threads(int(threads))
        rc = self.lib.oracle_batch(ptrs, q.ctypes.data, len(q), k, estimator, float(tau),
                                   int(tau_normalize), out.ctypes.data)
        if rc != 0:
            raise ValueError("k or tau_normalize out of range")
        return out

    def threads(self, n: int = 0) -> int:
        return self.lib.oracle_threads(int(n))


def load(rebuild: bool = False) -> Oracle:
    global _lib
    if _lib is not None and not rebuild:
        return _lib
    if rebuild or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_oracle()
    _lib = Oracle(LIB)
    return _lib
