"""Seeded synthetic inputs for the windowed-MI path.

This module only draws numbers and lays out windows: it holds none of the
estimator's arithmetic, so both the CPU oracle and the GPU path can be fed from
it without sharing any method code.

Every series value is put on the 2^-12 grid with magnitude below 2^11
(``quantize``).  On that grid every coordinate difference is an exact FP32
number, which is what makes neighbour distances and counts exact on both sides.

Workloads (stand-ins for the paper's NYC / energy data, which are not public):

* ``config1``  one pair, n=4096, 512-sample segments cycling through linear,
  quadratic, sinusoidal and independent links; windows w=128, stride 1.
* ``config2``  one pair, n=65536, segment lengths uniform in [256, 4096];
  windows w in {32..4096}, stride w/8, all scales in one batch.
* ``config3``  64 series x 32768 from an 8-factor latent model, half linear
  in the factors, half with quadratic / sine links; all 2016 pairs, w=256,
  stride 8, every position a noise triple (248-sample overlap + 8 new samples).
* ``config4``  serving: cfg2-style pairs, a Poisson stream of queries.
* ``config5``  IoT-like seasonal + AR(1) series with injected bursts;
  ``config5_proxy``: one pair, every top-down layer (w = 4096 .. 64,
  stride w/8) evaluated densely.

The relation types of the paper's synthetic-data table (Section 8.3.1) are
available through ``relation`` for qualitative tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GRID = 4096.0                     # 2^12 grid steps per unit
QMAX = (1 << 23) - 1              # |v| * 2^12 <= 2^23 - 1  =>  |v| < 2^11

SEG_TYPES = ("linear", "quadratic", "sine", "independent")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def quantize(v) -> np.ndarray:
    """Round to the 2^-12 grid, clip to |v| < 2^11, return float32."""
    q = np.clip(np.rint(np.asarray(v, dtype=np.float64) * GRID), -QMAX, QMAX)
    return (q / GRID).astype(np.float32)


def on_grid(v) -> bool:
    a = np.asarray(v, dtype=np.float64)
    s = a * GRID
    return bool(np.all(np.isfinite(a)) and np.all(s == np.rint(s)) and np.all(np.abs(s) <= QMAX))


def _link(kind: str, x: np.ndarray, e: np.ndarray) -> np.ndarray:
    if kind == "linear":
        return 0.8 * x + 0.6 * e
    if kind == "quadratic":
        return x * x + 0.3 * e
    if kind == "sine":
        return np.sin(3.0 * x) + 0.3 * e
    if kind == "independent":
        return e.copy()
    raise ValueError(kind)


def segmented_pair(n: int, seg_lengths, seed_rng: np.random.Generator):
    """x ~ N(0,1); y follows the segment's link to x (types cycle)."""
    x = quantize(seed_rng.standard_normal(n))
    e = quantize(seed_rng.standard_normal(n))
    xd = x.astype(np.float64)
    ed = e.astype(np.float64)
    y = np.empty(n, dtype=np.float64)
    types = np.empty(n, dtype=np.int8)
    pos = 0
    seg = 0
    for L in seg_lengths:
        if pos >= n:
            break
        end = min(n, pos + int(L))
        kind = SEG_TYPES[seg % 4]
        y[pos:end] = _link(kind, xd[pos:end], ed[pos:end])
        types[pos:end] = seg % 4
        pos = end
        seg += 1
    assert pos == n
    return x, quantize(y), types


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    series: list            # list of float32 arrays
    queries: np.ndarray     # structured array, see QUERY_DTYPE
    k: int = 4
    tau: float = 0.0
    note: str = ""

    @property
    def n_windows(self) -> int:
        q = self.queries
        return int(len(q) + 2 * np.count_nonzero(q["ext_side"] != 0))

    @property
    def ordered_pairs(self) -> int:
        q = self.queries
        m = q["len"].astype(np.int64)
        tot = int(np.sum(m * (m - 1)))
        t = q["ext_side"] != 0
        if np.any(t):
            me = q["ext_len"][t].astype(np.int64)
            mu = m[t] + me
            tot += int(np.sum(me * (me - 1)) + np.sum(mu * (mu - 1)))
        return tot


QUERY_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("start", "<u8"), ("len", "<u4"),
                        ("ext_len", "<u4"), ("ext_side", "<i4"), ("pad", "<u4")])
assert QUERY_DTYPE.itemsize == 32


def make_queries(a, b, start, length, ext_len=0, ext_side=0) -> np.ndarray:
    start = np.atleast_1d(np.asarray(start, dtype=np.uint64))
    q = np.zeros(start.shape[0], dtype=QUERY_DTYPE)
    q["a"] = a
    q["b"] = b
    q["start"] = start
    q["len"] = length
    q["ext_len"] = ext_len
    q["ext_side"] = ext_side
    return q


def sliding(n: int, w: int, stride: int) -> np.ndarray:
    return np.arange(0, n - w + 1, stride, dtype=np.uint64)


def config1(seed: int = 1) -> Workload:
    n = 4096
    x, y, _ = segmented_pair(n, [512] * 8, rng(seed))
    q = make_queries(0, 1, sliding(n, 128, 1), 128)
    return Workload("cfg1_plain_n4096_w128_s1", [x, y], q, k=4,
                    note="one pair, n=4096, w=128, stride 1, k=4")


CFG2_SCALES = (32, 64, 128, 256, 512, 1024, 2048, 4096)


def cfg2_pair(n: int, seed: int):
    r = rng(seed)
    lens = r.integers(256, 4096, size=n // 256 + 2, endpoint=True)
    x, y, _ = segmented_pair(n, lens, r)
    return x, y


def multiscale_queries(a: int, b: int, n: int, scales=CFG2_SCALES) -> np.ndarray:
    parts = [make_queries(a, b, sliding(n, w, w // 8), w) for w in scales]
    return np.concatenate(parts)


def config2(seed: int = 2, n: int = 65536) -> Workload:
    x, y = cfg2_pair(n, seed)
    q = multiscale_queries(0, 1, n)
    return Workload(f"cfg2_multiscale_n{n}_w32-4096_s8th", [x, y], q, k=4,
                    note="one pair, n=65536, w in 32..4096, stride w/8, k=4")


def config3_series(seed: int = 3, n_series: int = 64, n: int = 32768):
    r = rng(seed)
    F = r.standard_normal((n, 8))
    L = r.uniform(-1.0, 1.0, size=(n_series, 8))
    out = []
    half = n_series // 2
    block = np.arange(n) // 4096
    for s in range(n_series):
        noise = 0.3 * r.standard_normal(n)
        if s < half:
            v = F @ L[s] / np.linalg.norm(L[s]) + noise
        else:
            f = F[:, s % 8]
            v = np.where(block % 2 == 0, f * f, np.sin(3.0 * f)) + noise
        out.append(quantize(v))
    return out


def config3(seed: int = 3, n_series: int = 64, n: int = 32768, pairs=None,
            w: int = 256, delta: int = 8, stride: int = 8) -> Workload:
    series = config3_series(seed, n_series, n)
    if pairs is None:
        pairs = [(a, b) for a in range(n_series) for b in range(a + 1, n_series)]
    starts = sliding(n, w, stride)
    parts = [make_queries(a, b, starts, w - delta, delta, +1) for a, b in pairs]
    sigma = 0.2 * math.log(w)
    return Workload(f"cfg3_allpairs_{n_series}x{n}_w{w}_s{stride}_triples", series,
                    np.concatenate(parts), k=4, tau=sigma / 4.0,
                    note="latent-factor series, all pairs, noise triples")


def config4_pair(pair_id: int, n: int = 1 << 20):
    return cfg2_pair(n, 4 + pair_id)


def _quantize_torch(v):
    import torch
    q = torch.clamp(torch.round(v * GRID), -QMAX, QMAX)
    return (q / GRID).to(torch.float32)


def cfg2_pairs_device(n_pairs: int, n: int, seed: int, device, chunk: int = 16):
    """The cfg2 segment recipe drawn with torch's generator on `device`: a
    (2 * n_pairs, n) float32 tensor, rows (x0, y0, x1, y1, ...).  Used where
    host generation would take minutes (the serving store: 512 pairs of 2^20
    points).  Deterministic for a seed on a given device and torch build; not
    the same numbers as ``cfg2_pair``."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((2 * n_pairs, n), dtype=torch.float32, device=device)
    nseg = n // 256 + 2
    pos = torch.arange(n, device=device)
    for p0 in range(0, n_pairs, chunk):
        c = min(chunk, n_pairs - p0)
        x = _quantize_torch(torch.randn((c, n), generator=g, device=device, dtype=torch.float64))
        e = _quantize_torch(torch.randn((c, n), generator=g, device=device, dtype=torch.float64))
        lens = torch.randint(256, 4097, (c, nseg), generator=g, device=device)
        ends = torch.cumsum(lens, dim=1)
        kind = torch.searchsorted(ends, pos.expand(c, n).contiguous(), right=True) % 4
        xd, ed = x.double(), e.double()
        y = torch.where(kind == 0, 0.8 * xd + 0.6 * ed,
                        torch.where(kind == 1, xd * xd + 0.3 * ed,
                                    torch.where(kind == 2, torch.sin(3.0 * xd) + 0.3 * ed, ed)))
        out[2 * p0:2 * (p0 + c):2] = x
        out[2 * p0 + 1:2 * (p0 + c):2] = _quantize_torch(y)
        del x, e, xd, ed, y, kind, lens, ends
    return out


def config4_stream(n_queries: int = 20000, n_series: int = 1024, n: int = 1 << 20,
                   rate: float = 200.0, wmin: int = 32, wmax: int = 2048, seed: int = 4):
    """Poisson arrivals; each query = (a, b, w, stride=w//4) over the full series."""
    r = rng(seed + 1_000_000)
    gaps = r.exponential(1.0 / rate, size=n_queries)
    t = np.cumsum(gaps) - gaps[0]
    a = r.integers(0, n_series, size=n_queries)
    b = (a + r.integers(1, n_series, size=n_queries)) % n_series
    w = np.rint(np.exp(r.uniform(math.log(wmin), math.log(wmax), size=n_queries))).astype(np.int64)
    return t, a.astype(np.uint32), b.astype(np.uint32), w, np.maximum(w // 4, 1)


def config5_series(seed: int = 5, n_series: int = 8, n: int = 1 << 24):
    r = rng(seed)
    t = np.arange(n, dtype=np.float64)
    out = []
    base = []
    for s in range(n_series):
        ph1, ph2 = r.uniform(0, 2 * math.pi, size=2)
        innov = r.standard_normal(n) * math.sqrt(0.19)
        ar = _ar1(innov, 0.9)          # AR(1), phi = 0.9, unit stationary variance
        v = np.sin(2 * math.pi * t / 1440.0 + ph1) + 0.5 * np.sin(2 * math.pi * t / 10080.0 + ph2) + ar
        base.append(v)
    for s in range(n_series):
        v = base[s].copy()
        for _ in range(16):
            L = int(round(math.exp(r.uniform(math.log(1024), math.log(65536)))))
            st = int(r.integers(0, n - L))
            src = int(r.integers(0, n_series - 1))
            src = src if src < s else src + 1
            kind = int(r.integers(0, 3))
            u = base[src][st:st + L]
            if kind == 0:
                seg = 1.5 * u
            elif kind == 1:
                seg = u * u
            else:
                seg = np.exp(np.clip(u, -20.0, 7.0))
            v[st:st + L] = seg + 0.1 * r.standard_normal(L)
        out.append(quantize(v))
    return out


CFG5_LAYERS = (4096, 2048, 1024, 512, 256, 128, 64)


def config5_proxy(seed: int = 5, n: int = 1 << 24) -> Workload:
    """The hot path of the large search on one series pair: every layer of a
    top-down sweep evaluated densely (w = 4096, 2048, ..., 64, stride w/8)
    over the whole pair.  The pair is the config5 recipe with two series
    (each one's bursts copied from the other)."""
    series = config5_series(seed, n_series=2, n=n)
    q = np.concatenate([make_queries(0, 1, sliding(n, w, w // 8), w) for w in CFG5_LAYERS])
    return Workload(f"cfg5_td_dense_pair_n{n}_w64-4096_s8th", series, q, k=4,
                    note="IoT-like pair, 7 halving layers, stride w/8, k=4")


def _ar1(innov: np.ndarray, phi: float) -> np.ndarray:
    from scipy.signal import lfilter
    return lfilter([1.0], [1.0, -phi], innov)


# --------------------------------------------------------------------------
# relation types of the paper's synthetic-data table (Section 8.3.1)
# --------------------------------------------------------------------------

RELATIONS = ("independent", "linear", "exponential", "quadratic", "diamond", "circle",
             "sine", "cross", "quartic", "sqrt")


def relation(kind: str, m: int, seed: int):
    """Draw m samples (x, y) of one relation type; u ~ U(0,1) additive noise."""
    r = rng(seed)
    u = r.uniform(0.0, 1.0, m)
    if kind == "independent":
        x = r.normal(3.0, 5.0, m)
        y = r.normal(0.0, 1.0, m)
    elif kind == "linear":
        x = r.uniform(0, 10, m)
        y = 2 * x + u
    elif kind == "exponential":
        x = r.uniform(-10, 10, m)
        y = 0.01 ** ((x + u) / 10.0)          # rescaled exponent keeps |y| < 2^11
    elif kind == "quadratic":
        x = r.uniform(-4, 4, m)
        y = x * x + u
    elif kind == "diamond":
        x = r.uniform(4, 8, m)
        c = r.integers(0, 4, m)
        y = np.choose(c, [x + u, 8 - x + u, -4 + x + u, 12 - x + u])
    elif kind == "circle":
        x = r.uniform(-3, 3, m)
        sgn = np.where(r.integers(0, 2, m) == 0, -1.0, 1.0)
        y = sgn * np.sqrt(np.maximum(9.0 - x * x + u, 0.0))
    elif kind == "sine":
        x = r.uniform(0, 10, m)
        y = 2 * np.sin(x) + u
    elif kind == "cross":
        x = r.uniform(-5, 5, m)
        sgn = np.where(r.integers(0, 2, m) == 0, -1.0, 1.0)
        y = sgn * x + u
    elif kind == "quartic":
        x = r.uniform(-1, 3, m)
        y = x ** 4 - 4 * x ** 3 + 4 * x ** 2 + x + u
    elif kind == "sqrt":
        x = r.uniform(0, 25, m)
        y = np.sqrt(x) + 0.1 * u
    else:
        raise ValueError(kind)
    return quantize(x), quantize(y)


def bivariate_normal(m: int, rho: float, seed: int, scale: float = 1.0):
    r = rng(seed)
    z1 = r.standard_normal(m)
    z2 = r.standard_normal(m)
    x = z1
    y = rho * z1 + math.sqrt(1.0 - rho * rho) * z2
    return quantize(scale * x), quantize(scale * y)


def grid_points(m: int, seed: int, levels: int = 8, scale: float = 1.0 / 4096):
    """Tie-heavy points: coordinates drawn from a handful of grid levels."""
    r = rng(seed)
    x = r.integers(-levels, levels + 1, m) * scale
    y = r.integers(-levels, levels + 1, m) * scale
    return quantize(x), quantize(y)
