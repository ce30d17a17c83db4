"""Thin ctypes binding to libwmi.so (include/wmi.h).  Argument marshalling only:
every step of the computation runs in the library's HIP kernels.

There is no fallback: if libwmi.so is missing or cannot load, every entry
point raises.  PyTorch is optional and only used to pass device memory and
streams (``Store.add_series`` accepts a CUDA/HIP tensor; ``stream=`` accepts a
``torch.cuda.Stream``).
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwmi.so")

WMI_OK = 0
WMI_EINVAL = -1
WMI_ENOMEM = -2
WMI_EBUSY = -3
WMI_ETIMEDOUT = -4
WMI_EHIP = -5
WMI_ESTATE = -6
ERRNAMES = {0: "WMI_OK", -1: "WMI_EINVAL", -2: "WMI_ENOMEM", -3: "WMI_EBUSY", -4: "WMI_ETIMEDOUT",
            -5: "WMI_EHIP", -6: "WMI_ESTATE"}

F_NOISE = 1
F_TOO_SHORT = 2
F_NONPOS_BASE = 4
F_OFFGRID = 8

STORE_STRICT_GRID = 1
SUBMIT_NONBLOCKING = 1
SUBMIT_PLAIN = 2
SUBMIT_NO_REUSE = 4
SUBMIT_ENTROPY = 8
MAX_WINDOW = 4096
MAX_K = 16

QUERY_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("start", "<u8"), ("len", "<u4"),
                        ("ext_len", "<u4"), ("ext_side", "<i4"), ("pad", "<u4")])
RANGE_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("start", "<u8"), ("count", "<u4"), ("stride", "<u4"),
                        ("len", "<u4"), ("ext_len", "<u4"), ("ext_side", "<i4"), ("pad", "<u4")])
RESULT_DTYPE = np.dtype([("mi_base", "<f8"), ("mi_ext", "<f8"), ("mi_union", "<f8"),
                         ("flags", "<u4"), ("pad", "<u4")])
REQUEST_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("start", "<u8"), ("end", "<u8"), ("w", "<u4"),
                          ("stride", "<u4")])
WINDOW_RESULT_DTYPE = np.dtype([("mi", "<f8"), ("flags", "<u4"), ("pad", "<u4")])
SPAN_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("begin", "<u8"), ("end", "<u8")])
WINDOW_DTYPE = np.dtype([("start", "<u8"), ("len", "<u4"), ("layer", "<u4"), ("mi", "<f8")])

# the symbols include/wmi.h declares
EXPORTS = ("wmi_version", "wmi_last_error", "wmi_store_create", "wmi_store_destroy", "wmi_store_set_tuning",
           "wmi_store_get_tuning",
           "wmi_series_add", "wmi_series_add_device", "wmi_series_remove", "wmi_series_length",
           "wmi_submit", "wmi_submit_ranges", "wmi_submit_noalloc", "wmi_wait", "wmi_done", "wmi_read", "wmi_read_entropy",
           "wmi_batch_replay", "wmi_batch_timing",
           "wmi_batch_stats_get", "wmi_batch_count_evals", "wmi_batch_destroy", "wmi_debug_window", "wmi_psi_table",
           "wmi_server_create", "wmi_server_submit", "wmi_server_wait", "wmi_server_info",
           "wmi_server_read", "wmi_server_stats_get", "wmi_server_clock_us", "wmi_server_destroy",
           "wmi_td_search", "wmi_bu_search", "wmi_bu_search_many")
REPLAY_DIRECT = 1


class WmiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class _StoreDesc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("flags", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_uint64)]


class _Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("estimator", ctypes.c_uint32), ("tau", ctypes.c_double),
                ("tau_normalize", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class _Timing(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_uint32), ("mode", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("prep_ms", ctypes.c_double), ("main_ms", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("windows", ctypes.c_uint64), ("ordered_pairs", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("device_ms", ctypes.c_double),
                ("items", ctypes.c_uint32), ("grid", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("cus", ctypes.c_uint32)]


class _ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("k", ctypes.c_uint32), ("estimator", ctypes.c_uint32),
                ("max_launch_windows", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("windows", ctypes.c_uint64), ("t_arrival_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_first_launch_us", ctypes.c_double), ("t_complete_us", ctypes.c_double),
                ("state", ctypes.c_int32), ("launches", ctypes.c_uint32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("local_windows", ctypes.c_uint32 * 5), ("triples", ctypes.c_uint32 * 5),
                ("sweep_windows", ctypes.c_uint32 * 3), ("stragglers", ctypes.c_uint32 * 3)]


TUNING_FIELDS = {"local_windows": 5, "triples": 5, "sweep_windows": 3, "stragglers": 3}
TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


def tuning_file(device: int = 0) -> str:
    """The autotuner's choices for the device's architecture (may not exist)."""
    import torch
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    return os.path.join(TUNING_DIR, f"{arch}.json")


class _ServerStats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_uint64), ("windows_done", ctypes.c_uint64),
                ("ordered_pairs_done", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("busy_us", ctypes.c_double), ("arena_bytes", ctypes.c_uint64),
                ("arena_peak_bytes", ctypes.c_uint64), ("queued_peak", ctypes.c_uint64),
                ("busy_union_us", ctypes.c_double)]


class _TdParams(ctypes.Structure):
    _fields_ = [("s_max", ctypes.c_uint32), ("s_min", ctypes.c_uint32), ("step_div", ctypes.c_uint32),
                ("p", ctypes.c_uint32), ("sigma", ctypes.c_double), ("tau", ctypes.c_double),
                ("normalize", ctypes.c_uint32), ("k", ctypes.c_uint32), ("estimator", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class _BuParams(ctypes.Structure):
    _fields_ = [("s_min", ctypes.c_uint32), ("s_max", ctypes.c_uint32), ("delta", ctypes.c_uint32),
                ("max_idle", ctypes.c_uint32), ("history", ctypes.c_uint32), ("p", ctypes.c_uint32),
                ("sigma", ctypes.c_double), ("tau", ctypes.c_double), ("normalize", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("estimator", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _SearchStats(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_uint64), ("windows_visited", ctypes.c_uint64),
                ("windows_evaluated", ctypes.c_uint64), ("ordered_pairs", ctypes.c_uint64),
                ("noise_detections", ctypes.c_uint64), ("noise_skips", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("wall_ms", ctypes.c_double), ("submit_ms", ctypes.c_double),
                ("wait_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libwmi.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python -m paper_2204_09131_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "wmi_version": ([], ctypes.c_int),
        "wmi_last_error": ([], ctypes.c_char_p),
        "wmi_store_create": ([P(_StoreDesc), P(vp)], ctypes.c_int),
        "wmi_store_destroy": ([vp], ctypes.c_int),
        "wmi_store_set_tuning": ([vp, P(_Tuning)], ctypes.c_int),
        "wmi_store_get_tuning": ([vp, P(_Tuning)], ctypes.c_int),
        "wmi_series_add": ([vp, vp, u64, P(u32)], ctypes.c_int),
        "wmi_series_add_device": ([vp, vp, u64, vp, P(u32)], ctypes.c_int),
        "wmi_series_remove": ([vp, u32], ctypes.c_int),
        "wmi_series_length": ([vp, u32, P(u64)], ctypes.c_int),
        "wmi_submit": ([vp, vp, u64, P(_Params), vp, P(vp)], ctypes.c_int),
        "wmi_submit_ranges": ([vp, vp, u64, P(_Params), vp, P(vp)], ctypes.c_int),
        "wmi_submit_noalloc": ([vp, vp, u64, P(_Params), vp, vp], ctypes.c_int),
        "wmi_wait": ([vp, i64], ctypes.c_int),
        "wmi_done": ([vp], ctypes.c_int),
        "wmi_read": ([vp, vp], ctypes.c_int),
        "wmi_read_entropy": ([vp, vp], ctypes.c_int),
        "wmi_batch_replay": ([vp, vp, u32], ctypes.c_int),
        "wmi_batch_timing": ([vp, P(_Timing)], ctypes.c_int),
        "wmi_batch_stats_get": ([vp, P(_Stats)], ctypes.c_int),
        "wmi_batch_count_evals": ([vp, P(ctypes.c_uint64)], ctypes.c_int),
        "wmi_batch_destroy": ([vp], ctypes.c_int),
        "wmi_debug_window": ([vp, vp, P(_Params), vp, vp, vp, vp], ctypes.c_int),
        "wmi_psi_table": ([u32, vp], ctypes.c_int),
        "wmi_server_create": ([vp, P(_ServerDesc), P(vp)], ctypes.c_int),
        "wmi_server_submit": ([vp, vp, P(u64)], ctypes.c_int),
        "wmi_server_wait": ([vp, u64, i64], ctypes.c_int),
        "wmi_server_info": ([vp, u64, P(_RequestInfo)], ctypes.c_int),
        "wmi_server_read": ([vp, u64, vp, u64, P(_RequestInfo)], ctypes.c_int),
        "wmi_server_stats_get": ([vp, P(_ServerStats)], ctypes.c_int),
        "wmi_server_clock_us": ([vp], ctypes.c_double),
        "wmi_server_destroy": ([vp], ctypes.c_int),
        "wmi_td_search": ([vp, u32, u32, u64, u64, P(_TdParams), vp, u64, P(u64), P(_SearchStats)], ctypes.c_int),
        "wmi_bu_search": ([vp, u32, u32, u64, u64, P(_BuParams), vp, u64, P(u64), P(_SearchStats)], ctypes.c_int),
        "wmi_bu_search_many": ([vp, vp, u64, P(_BuParams), vp, vp, u64, P(u64), P(_SearchStats)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != WMI_OK:
        raise WmiError(rc, lib().wmi_last_error().decode(errors="replace"))


def version() -> tuple:
    v = lib().wmi_version()
    return (v >> 16, v & 0xFFFF)


def psi_table(n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _check(lib().wmi_psi_table(n, out.ctypes.data))
    return out


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _params(k, estimator, tau, tau_normalize, flags) -> _Params:
    return _Params(int(k), int(estimator), float(tau), int(tau_normalize), int(flags))


def as_queries(q) -> np.ndarray:
    q = np.ascontiguousarray(q)
    if q.dtype != QUERY_DTYPE:
        if q.dtype.names and set(QUERY_DTYPE.names) <= set(q.dtype.names) and q.dtype.itemsize == 32:
            q = q.view(QUERY_DTYPE) if q.dtype.descr == QUERY_DTYPE.descr else q.astype(QUERY_DTYPE)
        else:
            raise TypeError("queries must be a structured array with the wmi_query layout")
    return q


def make_ranges(a, b, start, count, stride, length, ext_len=0, ext_side=0) -> np.ndarray:
    """Runs of equally spaced queries (RANGE_DTYPE); arguments broadcast."""
    cols = np.broadcast_arrays(*(np.asarray(v) for v in (a, b, start, count, stride, length, ext_len, ext_side)))
    r = np.zeros(cols[0].shape, dtype=RANGE_DTYPE)
    for f, v in zip(("a", "b", "start", "count", "stride", "len", "ext_len", "ext_side"), cols):
        r[f] = v
    return r.reshape(-1)


def expand_ranges(ranges) -> np.ndarray:
    """The query list (QUERY_DTYPE) a run list stands for, in batch order."""
    r = np.ascontiguousarray(ranges, dtype=RANGE_DTYPE)
    cnt = r["count"].astype(np.int64)
    q = np.zeros(int(cnt.sum()), dtype=QUERY_DTYPE)
    idx = np.repeat(np.arange(len(r)), cnt)
    pos = np.arange(len(q)) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    for f in ("a", "b", "len", "ext_side"):
        q[f] = r[f][idx]
    q["ext_len"] = np.where(r["ext_side"][idx] != 0, r["ext_len"][idx], 0)
    q["start"] = r["start"][idx] + pos.astype(np.uint64) * r["stride"][idx].astype(np.uint64)
    return q


class Batch:
    def __init__(self, store: "Store", handle: int, count: int):
        self.store = store
        self.h = ctypes.c_void_p(handle)
        self.count = count

    def wait(self, timeout_us: int = -1):
        _check(lib().wmi_wait(self.h, int(timeout_us)))

    def done(self) -> bool:
        return bool(lib().wmi_done(self.h))

    def read(self) -> np.ndarray:
        out = np.zeros(self.count, dtype=RESULT_DTYPE)
        _check(lib().wmi_read(self.h, out.ctypes.data if self.count else None))
        return out

    def read_entropy(self) -> np.ndarray:
        """Window entropies (count x 3: base, extension, union; NaN where a
        query has no such window) of a batch submitted with entropy=True."""
        out = np.zeros((self.count, 3), dtype=np.float64)
        _check(lib().wmi_read_entropy(self.h, out.ctypes.data if self.count else None))
        return out

    def replay(self, stream=None, direct: bool = False):
        """Enqueue another run (graph launch, or kernel by kernel if direct)."""
        _check(lib().wmi_batch_replay(self.h, _stream_handle(stream), REPLAY_DIRECT if direct else 0))

    def timing(self) -> dict:
        t = _Timing()
        _check(lib().wmi_batch_timing(self.h, ctypes.byref(t)))
        return {"runs": t.runs, "mode": t.mode, "total_ms": t.total_ms, "prep_ms": t.prep_ms,
                "main_ms": t.main_ms}

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().wmi_batch_stats_get(self.h, ctypes.byref(s)))
        return {"windows": s.windows, "ordered_pairs": s.ordered_pairs, "launches": s.launches,
                "device_ms": s.device_ms, "items": s.items, "grid": s.grid, "wg_per_cu": s.wg_per_cu,
                "cus": s.cus}

    def count_evals(self) -> int:
        """(query point, candidate) distances the neighbour searches compute
        (one extra run of the kernels; synchronous)."""
        n = ctypes.c_uint64(0)
        _check(lib().wmi_batch_count_evals(self.h, ctypes.byref(n)))
        return n.value

    def destroy(self):
        if self.h:
            _check(lib().wmi_batch_destroy(self.h))
            self.h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            if self.h and self.store.h:
                lib().wmi_batch_destroy(self.h)
        except Exception:
            pass


class Store:
    """A set of resident series on one device."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, strict_grid: bool = False, tuning=None):
        """tuning: None (the library's defaults), a dict of wmi_tuning fields,
        or "auto": the autotuner's file for this device's architecture when
        there is one (tuning_file), else the defaults."""
        d = _StoreDesc(int(device), STORE_STRICT_GRID if strict_grid else 0, int(budget_bytes))
        h = ctypes.c_void_p()
        _check(lib().wmi_store_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.device = device
        self._borrowed = {}
        if tuning == "auto":
            path = tuning_file(device)
            tuning = json.load(open(path))["tuning"] if os.path.exists(path) else None
        if tuning is not None:
            self.set_tuning(tuning)

    def set_tuning(self, tuning=None):
        """Set the work-list choices (dict of wmi_tuning fields; missing
        fields keep the defaults; None: all defaults)."""
        if tuning is None:
            _check(lib().wmi_store_set_tuning(self.h, None))
            return
        cur = _Tuning()
        _check(lib().wmi_store_set_tuning(self.h, None))
        _check(lib().wmi_store_get_tuning(self.h, ctypes.byref(cur)))
        for f, n in TUNING_FIELDS.items():
            if f in tuning:
                v = list(tuning[f])
                if len(v) != n:
                    raise ValueError(f"tuning field {f} needs {n} values")
                setattr(cur, f, (ctypes.c_uint32 * n)(*[int(x) for x in v]))
        _check(lib().wmi_store_set_tuning(self.h, ctypes.byref(cur)))

    def get_tuning(self) -> dict:
        cur = _Tuning()
        _check(lib().wmi_store_get_tuning(self.h, ctypes.byref(cur)))
        return {f: list(getattr(cur, f)) for f in TUNING_FIELDS}

    def close(self):
        if self.h:
            _check(lib().wmi_store_destroy(self.h))
            self.h = ctypes.c_void_p(None)
            self._borrowed.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self.h:
                lib().wmi_store_destroy(self.h)
        except Exception:
            pass

    def add_series(self, values, stream=None) -> int:
        """Host array: copied.  Device tensor (torch, float32, contiguous): borrowed."""
        sid = ctypes.c_uint32()
        if hasattr(values, "is_cuda") and values.is_cuda:
            import torch
            if values.dtype != torch.float32 or not values.is_contiguous():
                raise TypeError("device series must be a contiguous float32 tensor")
            s = _stream_handle(stream if stream is not None else torch.cuda.current_stream(values.device))
            _check(lib().wmi_series_add_device(self.h, values.data_ptr(), values.numel(), s,
                                               ctypes.byref(sid)))
            self._borrowed[sid.value] = values
        else:
            v = np.ascontiguousarray(values, dtype=np.float32)
            _check(lib().wmi_series_add(self.h, v.ctypes.data, v.shape[0], ctypes.byref(sid)))
        return sid.value

    def remove_series(self, sid: int):
        _check(lib().wmi_series_remove(self.h, int(sid)))
        self._borrowed.pop(sid, None)

    def series_length(self, sid: int) -> int:
        n = ctypes.c_uint64()
        _check(lib().wmi_series_length(self.h, int(sid), ctypes.byref(n)))
        return n.value

    def submit(self, queries, k: int = 4, estimator: int = 0, tau: float = 0.0, tau_normalize: int = 0,
               plain: bool = False, nonblocking: bool = False, no_reuse: bool = False,
               entropy: bool = False, stream=None) -> Batch:
        q = as_queries(queries)
        flags = ((SUBMIT_PLAIN if plain else 0) | (SUBMIT_NONBLOCKING if nonblocking else 0)
                 | (SUBMIT_NO_REUSE if no_reuse else 0) | (SUBMIT_ENTROPY if entropy else 0))
        p = _params(k, estimator, tau, tau_normalize, flags)
        h = ctypes.c_void_p()
        _check(lib().wmi_submit(self.h, q.ctypes.data if len(q) else None, len(q), ctypes.byref(p),
                                _stream_handle(stream), ctypes.byref(h)))
        return Batch(self, h.value, len(q))

    def submit_ranges(self, ranges, k: int = 4, estimator: int = 0, tau: float = 0.0, tau_normalize: int = 0,
                      nonblocking: bool = False, no_reuse: bool = False, entropy: bool = False,
                      stream=None) -> Batch:
        """wmi_submit_ranges: queries given as runs (RANGE_DTYPE), expanded on
        the device; results in the order of expand_ranges(ranges)."""
        r = np.ascontiguousarray(ranges, dtype=RANGE_DTYPE)
        flags = ((SUBMIT_NONBLOCKING if nonblocking else 0) | (SUBMIT_NO_REUSE if no_reuse else 0)
                 | (SUBMIT_ENTROPY if entropy else 0))
        p = _params(k, estimator, tau, tau_normalize, flags)
        h = ctypes.c_void_p()
        _check(lib().wmi_submit_ranges(self.h, r.ctypes.data if len(r) else None, len(r), ctypes.byref(p),
                                       _stream_handle(stream), ctypes.byref(h)))
        return Batch(self, h.value, int(np.sum(r["count"], dtype=np.uint64)))

    def submit_ranges_many(self, ranges, max_queries: int = 1 << 20, max_points: int = 1 << 26, **kw) -> list:
        """Submit runs as consecutive batches of at most max_queries queries
        and (once a batch holds one) max_points window points, cutting runs
        where needed; results concatenate to those of expand_ranges(ranges)."""
        r = np.ascontiguousarray(ranges, dtype=RANGE_DTYPE)
        per = (r["len"].astype(np.int64) +
               np.where(r["ext_side"] != 0, r["len"].astype(np.int64) + 2 * r["ext_len"].astype(np.int64), 0))
        out, cur, cq, cp = [], [], 0, 0
        for i in range(len(r)):
            left, start = int(r["count"][i]), int(r["start"][i])
            while left > 0:
                room = min(max_queries - cq, max(0 if cq else 1, (max_points - cp) // max(int(per[i]), 1)))
                take = min(left, room)
                if take <= 0:
                    out.append(self.submit_ranges(np.array(cur, dtype=RANGE_DTYPE), **kw))
                    cur, cq, cp = [], 0, 0
                    continue
                g = r[i].copy()
                g["start"], g["count"] = start, take
                cur.append(g)
                cq += take
                cp += take * int(per[i])
                start += take * int(r["stride"][i])
                left -= take
                if cq >= max_queries or cp >= max_points:
                    out.append(self.submit_ranges(np.array(cur, dtype=RANGE_DTYPE), **kw))
                    cur, cq, cp = [], 0, 0
        if cur:
            out.append(self.submit_ranges(np.array(cur, dtype=RANGE_DTYPE), **kw))
        return out

    def submit_many(self, queries, max_queries: int = 1 << 18, max_points: int = 1 << 26, **kw) -> list:
        """Submit a large query set as consecutive batches, each of at most
        max_queries queries and (once it holds one) max_points window points;
        a query and its windows stay together."""
        q = as_queries(queries)
        pts = q["len"].astype(np.int64) + np.where(q["ext_side"] != 0, q["len"] + 2 * q["ext_len"].astype(np.int64), 0)
        cum = np.concatenate([[0], np.cumsum(pts)])
        out, i = [], 0
        while i < len(q):
            j = int(np.searchsorted(cum, cum[i] + max_points, side="right")) - 1
            j = min(max(j, i + 1), i + max_queries, len(q))
            out.append(self.submit(q[i:j], **kw))
            i = j
        return out

    def submit_noalloc(self, queries, d_results: int, k: int = 4, estimator: int = 0, tau: float = 0.0,
                       tau_normalize: int = 0, stream=None):
        """wmi_submit_noalloc: results (32 bytes per query) written to the
        device address d_results; returns once they are there."""
        q = as_queries(queries)
        p = _params(k, estimator, tau, tau_normalize, 0)
        _check(lib().wmi_submit_noalloc(self.h, q.ctypes.data if len(q) else None, len(q), ctypes.byref(p),
                                        _stream_handle(stream), int(d_results) if d_results else None))

    def evaluate(self, queries, **kw) -> np.ndarray:
        b = self.submit(queries, **kw)
        try:
            return b.read()
        finally:
            b.destroy()

    def td_search(self, a: int, b: int, begin: int, end: int, s_max: int, s_min: int, sigma: float,
                  tau: float = 0.0, p: int = 0, step_div: int = 8, normalize: int = 0, k: int = 4,
                  estimator: int = 0):
        """Top-down search (wmi_td_search): correlated windows (WINDOW_DTYPE,
        ascending start) and the search counters."""
        prm = _TdParams(int(s_max), int(s_min), int(step_div), int(p), float(sigma), float(tau),
                        int(normalize), int(k), int(estimator), 0)
        cap = max(1, (int(end) - int(begin)) // max(int(s_min), 1) + 1)
        out = np.zeros(cap, dtype=WINDOW_DTYPE)
        n = ctypes.c_uint64()
        st = _SearchStats()
        _check(lib().wmi_td_search(self.h, int(a), int(b), int(begin), int(end), ctypes.byref(prm),
                                   out.ctypes.data, cap, ctypes.byref(n), ctypes.byref(st)))
        return out[:n.value].copy(), {f: getattr(st, f) for f, _ in _SearchStats._fields_}

    def bu_search(self, a: int, b: int, begin: int, end: int, s_min: int, s_max: int, delta: int, sigma: float,
                  max_idle: int = 2, history: int = 4, tau: float = 0.0, p: int = 0, normalize: int = 0,
                  chunk: int = 0, seed: int = 0, k: int = 4, estimator: int = 0):
        """Bottom-up search (wmi_bu_search): correlated windows (WINDOW_DTYPE,
        ascending start) and the search counters."""
        prm = _BuParams(int(s_min), int(s_max), int(delta), int(max_idle), int(history), int(p), float(sigma),
                        float(tau), int(normalize), int(k), int(estimator), int(chunk),
                        int(seed) & 0xFFFFFFFFFFFFFFFF, 0, 0)
        cap = max(1, (int(end) - int(begin)) // max(int(s_min), 1) + 1)
        out = np.zeros(cap, dtype=WINDOW_DTYPE)
        n = ctypes.c_uint64()
        st = _SearchStats()
        _check(lib().wmi_bu_search(self.h, int(a), int(b), int(begin), int(end), ctypes.byref(prm),
                                   out.ctypes.data, cap, ctypes.byref(n), ctypes.byref(st)))
        return out[:n.value].copy(), {f: getattr(st, f) for f, _ in _SearchStats._fields_}

    def bu_search_many(self, spans, s_min: int, s_max: int, delta: int, sigma: float, max_idle: int = 2,
                       history: int = 4, tau: float = 0.0, p: int = 0, normalize: int = 0, chunk: int = 0,
                       seed: int = 0, k: int = 4, estimator: int = 0):
        """wmi_bu_search_many over spans [(a, b, begin, end), ...]: the
        correlated windows (WINDOW_DTYPE, by span then start), the span of
        each, and the search counters summed over the spans."""
        sp = np.zeros(len(spans), dtype=SPAN_DTYPE)
        for i, (a, b, begin, end) in enumerate(spans):
            sp[i] = (a, b, begin, end)
        prm = _BuParams(int(s_min), int(s_max), int(delta), int(max_idle), int(history), int(p), float(sigma),
                        float(tau), int(normalize), int(k), int(estimator), int(chunk),
                        int(seed) & 0xFFFFFFFFFFFFFFFF, 0, 0)
        cap = max(1, int(np.sum((sp["end"].astype(np.int64) - sp["begin"].astype(np.int64)) // max(int(s_min), 1) + 1)))
        out = np.zeros(cap, dtype=WINDOW_DTYPE)
        span = np.zeros(cap, dtype=np.uint32)
        n = ctypes.c_uint64()
        st = _SearchStats()
        _check(lib().wmi_bu_search_many(self.h, sp.ctypes.data if len(sp) else None, len(sp), ctypes.byref(prm),
                                        out.ctypes.data, span.ctypes.data, cap, ctypes.byref(n), ctypes.byref(st)))
        return out[:n.value].copy(), span[:n.value].copy(), {f: getattr(st, f) for f, _ in _SearchStats._fields_}

    def debug_window(self, a: int, b: int, start: int, length: int, k: int = 4, estimator: int = 0) -> dict:
        q = np.zeros(1, dtype=QUERY_DTYPE)
        q["a"], q["b"], q["start"], q["len"] = a, b, start, length
        nx = np.zeros(length, dtype=np.uint32)
        ny = np.zeros(length, dtype=np.uint32)
        ex = np.zeros(length, dtype=np.float32)
        ey = np.zeros(length, dtype=np.float32)
        p = _params(k, estimator, 0.0, 0, 0)
        _check(lib().wmi_debug_window(self.h, q.ctypes.data, ctypes.byref(p), nx.ctypes.data,
                                      ny.ctypes.data, ex.ctypes.data, ey.ctypes.data))
        return {"nx": nx, "ny": ny, "eps_x": ex, "eps_y": ey}


def _info_dict(i: _RequestInfo) -> dict:
    return {"windows": i.windows, "t_arrival_us": i.t_arrival_us, "t_admit_us": i.t_admit_us,
            "t_first_launch_us": i.t_first_launch_us, "t_complete_us": i.t_complete_us,
            "state": i.state, "launches": i.launches}


class Server:
    """Continuous batching of range requests over a store's series."""

    def __init__(self, store: Store, k: int = 4, estimator: int = 0, hbm_budget_bytes: int = 0,
                 max_launch_windows: int = 0):
        d = _ServerDesc(int(hbm_budget_bytes), int(k), int(estimator), int(max_launch_windows), 0)
        h = ctypes.c_void_p()
        _check(lib().wmi_server_create(store.h, ctypes.byref(d), ctypes.byref(h)))
        self.store = store
        self.h = h
        self._windows = {}

    def submit(self, a: int, b: int, start: int, end: int, w: int, stride: int = 1) -> int:
        r = np.zeros(1, dtype=REQUEST_DTYPE)
        r["a"], r["b"], r["start"], r["end"], r["w"], r["stride"] = a, b, start, end, w, stride
        t = ctypes.c_uint64()
        _check(lib().wmi_server_submit(self.h, r.ctypes.data, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        _check(lib().wmi_server_wait(self.h, int(ticket), int(timeout_us)))

    def info(self, ticket: int) -> dict:
        i = _RequestInfo()
        _check(lib().wmi_server_info(self.h, int(ticket), ctypes.byref(i)))
        return _info_dict(i)

    def read(self, ticket: int):
        """Results (WINDOW_RESULT_DTYPE, window order) and timing of a completed request."""
        n = self.info(ticket)["windows"]
        out = np.zeros(n, dtype=WINDOW_RESULT_DTYPE)
        i = _RequestInfo()
        _check(lib().wmi_server_read(self.h, int(ticket), out.ctypes.data if n else None, n, ctypes.byref(i)))
        return out, _info_dict(i)

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib().wmi_server_stats_get(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _ServerStats._fields_}

    def clock_us(self) -> float:
        return lib().wmi_server_clock_us(self.h)

    def close(self):
        # a closed store has already destroyed its servers
        if self.h and self.store.h:
            _check(lib().wmi_server_destroy(self.h))
        self.h = ctypes.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self.h and self.store.h:
                lib().wmi_server_destroy(self.h)
        except Exception:
            pass
