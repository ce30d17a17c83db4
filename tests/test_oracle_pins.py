"""Pins for the CPU oracle: each test checks it against something other than
itself -- the paper's worked example, closed forms, library routines that
implement the same definition by other means, brute force with a different
algorithm on tiny inputs, sampling-theory bounds, and exact invariances.

The arithmetic under test is in oracle/ksg_oracle.c.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.special import digamma

from paper_2204_09131_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Euler-Mascheroni constant to 40 digits (a mathematical constant, not the
# oracle's); used for exact rational harmonic-number checks.
GAMMA_40 = Fraction("0.5772156649015328606065120900824024310422")


# ---------------------------------------------------------------------------
# psi at integers
# ---------------------------------------------------------------------------

def test_psi_exact_harmonic(orc):
    """psi(n) = H_{n-1} - gamma, with H computed as an exact rational."""
    h = Fraction(0)
    for n in range(1, 301):
        exact = float(h - GAMMA_40)
        got = orc.psi(n)
        assert abs(got - exact) <= 2.0 ** -52 * max(1.0, abs(exact)), n
        h += Fraction(1, n)


def test_psi_against_scipy(orc):
    n = np.arange(1, 65537)
    tab = orc.psi_table(65536)
    assert np.max(np.abs(tab - digamma(n.astype(np.float64)))) < 1e-13
    assert tab[0] == pytest.approx(-0.5772156649015329, abs=1e-16)
    assert tab[1] == pytest.approx(1 - 0.5772156649015329, abs=1e-16)


def test_psi_asymptotic(orc):
    """Large-n asymptotic series: psi(n) ~ ln n - 1/(2n) - 1/(12 n^2) + 1/(120 n^4)."""
    for n in (1000, 4096, 65536):
        a = math.log(n) - 1 / (2 * n) - 1 / (12 * n * n) + 1 / (120 * n ** 4)
        assert abs(orc.psi(n) - a) < 1e-14


# ---------------------------------------------------------------------------
# the worked example of Section 7.1.1
# ---------------------------------------------------------------------------

def test_worked_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "worked_example_7pt.json")))
    names = g["order"]
    pts = np.array([g["points"][n] for n in names], dtype=np.float32)
    r = orc.window_counts(pts[:, 0], pts[:, 1], k=g["k"], estimator=0)
    i = names.index(g["query"])
    ex = g["expected"]
    assert sorted(names[j] for j in r["nbr"][i]) == sorted(ex["neighbours"])
    assert r["nx"][i] == ex["n_x"]
    assert r["ny"][i] == ex["n_y"]
    # membership, recomputed from the radii the oracle returned
    dx = np.abs(pts[:, 0] - pts[i, 0]).astype(np.float64)
    dy = np.abs(pts[:, 1] - pts[i, 1]).astype(np.float64)
    mx = {names[j] for j in range(len(names)) if j != i and dx[j] <= r["eps_x"][i]}
    my = {names[j] for j in range(len(names)) if j != i and dy[j] <= r["eps_y"][i]}
    assert mx == set(ex["n_x_members"])
    assert my == set(ex["n_y_members"])


# ---------------------------------------------------------------------------
# brute force with a full sort (a different algorithm) on tiny windows
# ---------------------------------------------------------------------------

def brute(x, y, k, estimator):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m = len(x)
    nx, ny, ex, ey = [], [], [], []
    for i in range(m):
        order = sorted((max(abs(x[i] - x[j]), abs(y[i] - y[j])), j) for j in range(m) if j != i)
        nb = [j for _, j in order[:k]]
        if estimator == 0:
            rx = max(abs(x[i] - x[j]) for j in nb)
            ry = max(abs(y[i] - y[j]) for j in nb)
            cx = sum(1 for j in range(m) if j != i and abs(x[i] - x[j]) <= rx)
            cy = sum(1 for j in range(m) if j != i and abs(y[i] - y[j]) <= ry)
        else:
            rx = ry = order[k - 1][0]
            cx = sum(1 for j in range(m) if j != i and abs(x[i] - x[j]) < rx)
            cy = sum(1 for j in range(m) if j != i and abs(y[i] - y[j]) < ry)
        nx.append(cx); ny.append(cy); ex.append(rx); ey.append(ry)
    return np.array(nx), np.array(ny), np.array(ex), np.array(ey)


def brute_mi(x, y, k, estimator):
    nx, ny, _, _ = brute(x, y, k, estimator)
    m = len(x)
    if estimator == 0:
        return float(digamma(k) - 1.0 / k + digamma(m) - np.mean(digamma(nx) + digamma(ny)))
    return float(digamma(k) + digamma(m) - np.mean(digamma(nx + 1) + digamma(ny + 1)))


@settings(max_examples=150, deadline=None)
@given(m=st.integers(2, 16), k=st.integers(1, 6), levels=st.integers(1, 6),
       seed=st.integers(0, 2 ** 31 - 1), est=st.integers(0, 1))
def test_brute_force_tiny_tie_heavy(orc, m, k, levels, seed, est):
    if m <= k:
        with pytest.raises(ValueError):
            orc.window_counts(np.zeros(m), np.zeros(m), k=k, estimator=est)
        assert math.isnan(orc.window_mi(np.zeros(m), np.zeros(m), k, est))
        return
    x, y = synth.grid_points(m, seed, levels=levels, scale=0.25)
    r = orc.window_counts(x, y, k=k, estimator=est)
    nx, ny, ex, ey = brute(x, y, k, est)
    np.testing.assert_array_equal(r["nx"], nx)
    np.testing.assert_array_equal(r["ny"], ny)
    np.testing.assert_array_equal(r["eps_x"], ex)
    np.testing.assert_array_equal(r["eps_y"], ey)
    assert orc.window_mi(x, y, k, est) == pytest.approx(brute_mi(x, y, k, est), abs=1e-12)


# ---------------------------------------------------------------------------
# scipy's k-d tree (max norm) on tie-free windows
# ---------------------------------------------------------------------------

def tie_free_window(m, seed, span=1 << 20):
    r = np.random.Generator(np.random.PCG64(seed))
    x = synth.quantize(r.integers(-span, span, m) / 4096.0)
    y = synth.quantize(r.integers(-span, span, m) / 4096.0)
    return x, y


@pytest.mark.parametrize("m,k,seed", [(64, 4, 0), (200, 4, 1), (300, 1, 2), (257, 8, 3), (500, 16, 4)])
def test_kdtree_counts(orc, m, k, seed):
    from scipy.spatial import cKDTree
    x, y = tie_free_window(m, seed)
    pts = np.stack([x, y], 1).astype(np.float64)
    d, idx = cKDTree(pts).query(pts, k=k + 2, p=np.inf)
    r = orc.window_counts(x, y, k=k, estimator=0)
    sx = np.sort(x.astype(np.float64))
    sy = np.sort(y.astype(np.float64))
    checked = 0
    for i in range(m):
        # column 0 is the point itself; skip points with a tie at the k-th distance
        if d[i, k] == d[i, k + 1] or d[i, 0] != 0.0:
            continue
        nb = idx[i, 1:k + 1]
        rx = np.max(np.abs(pts[nb, 0] - pts[i, 0]))
        ry = np.max(np.abs(pts[nb, 1] - pts[i, 1]))
        cx = np.searchsorted(sx, pts[i, 0] + rx, "right") - np.searchsorted(sx, pts[i, 0] - rx, "left") - 1
        cy = np.searchsorted(sy, pts[i, 1] + ry, "right") - np.searchsorted(sy, pts[i, 1] - ry, "left") - 1
        assert set(r["nbr"][i]) == set(nb.tolist())
        assert r["eps_x"][i] == rx and r["eps_y"][i] == ry
        assert r["nx"][i] == cx and r["ny"][i] == cy
        checked += 1
    assert checked > 0.9 * m


# ---------------------------------------------------------------------------
# scikit-learn's first-estimator KSG (estimator 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,m,k,seed", [("linear", 300, 3, 0), ("quadratic", 400, 4, 1),
                                           ("sine", 500, 5, 2), ("circle", 350, 4, 3)])
def test_sklearn_ksg1(orc, kind, m, k, seed):
    from sklearn.feature_selection._mutual_info import _compute_mi_cc
    x, y = synth.relation(kind, m, seed)
    ref = _compute_mi_cc(x.astype(np.float64), y.astype(np.float64), k)
    got = orc.window_mi(x, y, k, 1)
    assert ref > 0.05
    assert got == pytest.approx(ref, abs=1e-12)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

SURVEY_CLOSED = {32: 1.943911862103, 128: 3.342001259256, 256: 4.037105379484, 4096: 6.811526423008}


@pytest.mark.parametrize("m", [32, 128, 256, 4096])
def test_closed_form_identity_ramp(orc, m):
    """x = y = ramp: every point has n_x = n_y = k, so I = psi(m) - psi(k) - 1/k."""
    x = (np.arange(m) / 4096.0).astype(np.float32)
    got = orc.window_mi(x, x, 4, 0)
    assert got == pytest.approx(digamma(m) - digamma(4) - 0.25, abs=1e-12)
    assert got == pytest.approx(SURVEY_CLOSED[m], abs=1e-11)


@pytest.mark.parametrize("m,k,seed,scale", [(100, 4, 0, 1.0), (333, 3, 1, 4.0), (1000, 6, 2, 2.0),
                                             (700, 1, 3, 1.0)])
def test_closed_form_functional(orc, m, k, seed, scale):
    """y = 2^j x (j >= 0) on tie-free x: KSG-2 gives psi(m)-psi(k)-1/k for any j;
    KSG-1 gives psi(m)-psi(k) for y = x (its joint radius is not per-dimension)."""
    for attempt in range(50):
        x, _ = tie_free_window(m, seed + 1000 * attempt, span=1 << 20)
        # no tie at the k-th neighbour in 1-D
        d = np.abs(x[:, None].astype(np.float64) - x[None, :])
        np.fill_diagonal(d, np.inf)
        ds = np.sort(d, 1)
        if np.all(ds[:, k - 1] < ds[:, k]):
            break
    else:
        pytest.fail("no tie-free draw")
    y = synth.quantize(x.astype(np.float64) * scale)
    assert orc.window_mi(x, y, k, 0) == pytest.approx(digamma(m) - digamma(k) - 1.0 / k, abs=1e-12)
    if scale == 1.0:
        assert orc.window_mi(x, y, k, 1) == pytest.approx(digamma(m) - digamma(k), abs=1e-12)


# ---------------------------------------------------------------------------
# sampling-theory bounds: Gaussian closed form and independence
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rho", [0.0, 0.5, 0.8, 0.95])
def test_gaussian_closed_form(orc, rho):
    m, seeds = 1024, 32
    vals = []
    for s in range(seeds):
        x, y = synth.bivariate_normal(m, rho, 1000 + s)
        vals.append(orc.window_mi(x, y, 4, 0))
    vals = np.array(vals)
    truth = -0.5 * math.log(1 - rho * rho)
    sd = vals.std(ddof=1)
    # KSG-2 bias for Gaussians at m=1024, k=4 is a few 1e-3 nats (Kraskov et al. 2004)
    assert abs(vals.mean() - truth) <= 3 * sd / math.sqrt(seeds) + 0.01, (vals.mean(), truth, sd)


def test_independent_near_zero(orc):
    vals = []
    for s in range(32):
        x, y = synth.relation("independent", 512, 2000 + s)
        vals.append(orc.window_mi(x, y, 4, 0))
    vals = np.array(vals)
    assert abs(vals.mean()) <= 3 * vals.std(ddof=1) / math.sqrt(32) + 0.01


def test_dependence_ranks_above_independence(orc):
    """Every relation type of the synthetic-data table scores well above noise."""
    noise = max(orc.window_mi(*synth.relation("independent", 512, s), 4, 0) for s in range(8))
    for kind in synth.RELATIONS:
        if kind == "independent":
            continue
        mi = orc.window_mi(*synth.relation(kind, 512, 7), 4, 0)
        assert mi > noise + 0.3, kind


# ---------------------------------------------------------------------------
# exact symmetry and invariances
# ---------------------------------------------------------------------------

@settings(max_examples=60, deadline=None)
@given(m=st.integers(5, 80), levels=st.integers(1, 40), seed=st.integers(0, 2 ** 31 - 1),
       est=st.integers(0, 1), k=st.integers(1, 4))
def test_symmetry_bit_exact(orc, m, levels, seed, est, k):
    x, y = synth.grid_points(m, seed, levels=levels, scale=1 / 64)
    assert orc.window_mi(x, y, k, est) == orc.window_mi(y, x, k, est)


@settings(max_examples=40, deadline=None)
@given(m=st.integers(6, 80), levels=st.integers(1, 40), seed=st.integers(0, 2 ** 31 - 1),
       shift=st.integers(-1000, 1000), j=st.integers(-3, 3))
def test_translation_and_scaling_bit_exact(orc, m, levels, seed, shift, j):
    x, y = synth.grid_points(m, seed, levels=levels, scale=1 / 64)
    base = orc.window_mi(x, y, 4, 0)
    xs = synth.quantize(x.astype(np.float64) + shift / 64.0)
    assert orc.window_mi(xs, y, 4, 0) == base
    xs = synth.quantize(x.astype(np.float64) * 2.0 ** j)
    ys = synth.quantize(y.astype(np.float64) * 2.0 ** j)
    assert orc.window_mi(xs, ys, 4, 0) == base


def test_permutation_invariance_tie_free(orc):
    x, y = tie_free_window(400, 9)
    p = np.random.Generator(np.random.PCG64(1)).permutation(400)
    assert orc.window_mi(x[p], y[p], 4, 0) == pytest.approx(orc.window_mi(x, y, 4, 0), abs=1e-12)


# ---------------------------------------------------------------------------
# batches and the noise flag (Definition 6.2)
# ---------------------------------------------------------------------------

def test_batch_matches_windows(orc):
    w = synth.config1()
    x, y = w.series
    q = w.queries[::97]
    res = orc.batch(w.series, q, k=4)
    for r, qq in zip(res, q):
        s, m = int(qq["start"]), int(qq["len"])
        assert r["mi_base"] == orc.window_mi(x[s:s + m], y[s:s + m], 4, 0)
        assert math.isnan(r["mi_ext"]) and r["flags"] == 0


def _triple(orc, x, y, start, length, ext, side, tau):
    q = synth.make_queries(0, 1, start, length, ext, side)
    return orc.batch([x, y], q, k=4, tau=tau)[0]


def test_noise_flag_constructed():
    import oracle
    orc = oracle.load()
    r = synth.rng(77)
    n = 1024
    x = r.standard_normal(n)
    e = r.standard_normal(n)
    y_lin = 0.9 * x + 0.1 * e
    y_mix = y_lin.copy()
    y_mix[512:] = r.standard_normal(n - 512)          # independent extension
    xq, ylq, ymq = synth.quantize(x), synth.quantize(y_lin), synth.quantize(y_mix)
    tau = 0.1
    # base [0,512) linear, extension [512, 768) independent noise
    res = _triple(orc, xq, ymq, 0, 512, 256, +1, tau)
    assert res["mi_base"] > 1.0 and res["mi_ext"] < tau and res["mi_union"] < res["mi_base"]
    assert res["flags"] & oracle.FLAG_NOISE
    # same relation continues: not noise
    res = _triple(orc, xq, ylq, 0, 512, 256, +1, tau)
    assert not (res["flags"] & oracle.FLAG_NOISE) and res["mi_ext"] > tau
    # left extension: base [512, 768) of the linear series, extension of noise on the left
    y_left = y_lin.copy()
    y_left[:512] = r.standard_normal(512)
    res = _triple(orc, xq, synth.quantize(y_left), 512, 256, 256, -1, tau)
    assert res["flags"] & oracle.FLAG_NOISE
    # each component equals the standalone window
    assert res["mi_ext"] == orc.window_mi(xq[256:512], synth.quantize(y_left)[256:512], 4, 0)
    assert res["mi_union"] == orc.window_mi(xq[256:768], synth.quantize(y_left)[256:768], 4, 0)


def test_noise_flag_nonpositive_base_and_short():
    import oracle
    orc = oracle.load()
    x, y = synth.relation("independent", 600, 5)
    found = False
    for s in range(0, 500, 10):
        res = _triple(orc, x, y, s, 64, 8, +1, 10.0)
        if res["mi_base"] <= 0:
            assert res["flags"] & oracle.FLAG_NONPOS_BASE and not res["flags"] & oracle.FLAG_NOISE
            found = True
        else:
            assert not res["flags"] & oracle.FLAG_NONPOS_BASE
    assert found
    res = _triple(orc, x, y, 100, 64, 4, +1, 10.0)        # extension of 4 points with k = 4
    assert res["flags"] & oracle.FLAG_TOO_SHORT and not res["flags"] & oracle.FLAG_NOISE
    assert math.isnan(res["mi_ext"])


def test_offgrid_flag():
    import oracle
    orc = oracle.load()
    x, y = synth.relation("linear", 64, 3)
    y = y.copy()
    y[5] += np.float32(1e-5)
    res = orc.batch([x, y], synth.make_queries(0, 1, 0, 64), k=4)
    assert res[0]["flags"] & oracle.FLAG_OFFGRID


# ---------------------------------------------------------------------------
# the normalised noise threshold: tau * ln|w_d| (Eq. normalizedMI with the
# entropy of |w_d| distinct samples, applied to Definition 6.2's new part)
# ---------------------------------------------------------------------------

def _x_shape_triple():
    """A 16-point ramp (y = x) followed by an 8-point anti-diagonal over the
    same x range.  Each part alone is a tie-free scaled ramp, so by the closed
    form I(w_o) = psi(16) - psi(4) - 1/4 = 1.23490 and
    I(w_d) = psi(8) - psi(4) - 1/4 = 0.50952; the union is an X, whose
    estimate (0.27023 by the full-sort brute force) is far below I(w_o)."""
    u = 1.0 / 4096.0
    j = np.arange(8)
    x = np.concatenate([np.arange(16) * u, 2 * j * u]).astype(np.float32)
    y = np.concatenate([np.arange(16) * u, (15 - 2 * j) * u]).astype(np.float32)
    return x, y


def test_x_shape_triple_parts_by_closed_form_and_brute_force():
    x, y = _x_shape_triple()
    assert brute_mi(x[:16], y[:16], 4, 0) == pytest.approx(digamma(16) - digamma(4) - 0.25, abs=1e-12)
    assert brute_mi(x[16:], y[16:], 4, 0) == pytest.approx(digamma(8) - digamma(4) - 0.25, abs=1e-12)
    assert brute_mi(x, y, 4, 0) == pytest.approx(0.2702282595235883, abs=1e-12)


# tau, expected noise bit with tau * ln|w_d|; the readings a slip could take
# instead (ln|w_o|, ln|w''|, log2|w_d|, log10|w_d|, no normalisation) give
# the opposite bit in at least one of the two cases, which the test asserts.
@pytest.mark.parametrize("tau,noise", [(0.22, False), (0.30, True)])
def test_noise_flag_normalized_threshold(orc, tau, noise):
    import oracle
    x, y = _x_shape_triple()
    i_o = digamma(16) - digamma(4) - 0.25
    i_d = digamma(8) - digamma(4) - 0.25
    # the case sits well clear of its threshold under the paper's reading
    assert abs(i_d - tau * math.log(8)) > 0.04
    assert (i_d < tau * math.log(8)) == noise
    # and the wrong readings are told apart by the pair of cases
    wrong = {"ln|w_o|": tau * math.log(16), "ln|w''|": tau * math.log(24), "log2": tau * 3.0,
             "log10": tau * math.log10(8), "raw": tau}
    flips = {name for name, thr in wrong.items() if (i_d < thr) != noise}
    assert flips == ({"ln|w_o|", "ln|w''|", "log2"} if not noise else {"log10", "raw"})
    q = synth.make_queries(0, 1, 0, 16, 8, +1)
    r = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=1)[0]
    assert r["mi_base"] == pytest.approx(i_o, abs=1e-12)
    assert r["mi_ext"] == pytest.approx(i_d, abs=1e-12)
    assert r["mi_union"] == pytest.approx(0.2702282595235883, abs=1e-12)
    assert bool(r["flags"] & oracle.FLAG_NOISE) == noise
    assert not r["flags"] & oracle.FLAG_NONPOS_BASE
    # without normalisation the raw threshold decides: never noise here
    r = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=0)[0]
    assert not r["flags"] & oracle.FLAG_NOISE


# --------------------------------------------------------------------------
# window entropy H_w (Section 5.4, the denominator of the normalised MI),
# read as the entropy of the window's empirical distribution of pairs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 7, 256, 4096])
def test_entropy_all_distinct_is_ln_m(orc, m):
    x = (np.arange(m) / 4096.0).astype(np.float32)
    y = np.random.default_rng(m).permutation(x)
    assert orc.window_entropy(x, y) == pytest.approx(math.log(m), abs=1e-12)


@pytest.mark.parametrize("m", [1, 5, 300])
def test_entropy_constant_window_is_zero(orc, m):
    v = np.full(m, 0.75, dtype=np.float32)
    assert orc.window_entropy(v, -v) == 0.0


def test_entropy_two_equal_clusters_is_ln2(orc):
    x = np.array([0.5] * 6 + [0.25] * 6, dtype=np.float32)
    y = np.array([1.0] * 6 + [2.0] * 6, dtype=np.float32)
    assert orc.window_entropy(x, y) == pytest.approx(math.log(2), abs=1e-15)


def test_entropy_pairs_not_coordinates(orc):
    """Pairs that agree in one coordinate only are distinct: the grid
    {0,1} x {0,1}, each cell twice, has entropy ln 4 (ln 2 per coordinate)."""
    x = np.array([0, 0, 1, 1, 0, 0, 1, 1], dtype=np.float32)
    y = np.array([0, 1, 0, 1, 1, 0, 1, 0], dtype=np.float32)
    assert orc.window_entropy(x, y) == pytest.approx(math.log(4), abs=1e-15)
    assert orc.window_entropy(x, np.zeros(8, np.float32)) == pytest.approx(math.log(2), abs=1e-15)
    # unequal multiplicities: (0,0) once, (0,1) twice, (1,0) once
    x = np.array([0, 0, 0, 1], dtype=np.float32)
    y = np.array([0, 1, 1, 0], dtype=np.float32)
    assert orc.window_entropy(x, y) == pytest.approx(1.5 * math.log(2), abs=1e-15)


def test_entropy_signed_zero_is_one_value(orc):
    x = np.array([0.0, -0.0, 0.0, -0.0], dtype=np.float32)
    assert orc.window_entropy(x, x) == 0.0


@pytest.mark.parametrize("seed", range(5))
def test_entropy_against_scipy(orc, seed):
    """Multiplicities drawn at random; scipy's entropy of the count vector
    is the same quantity."""
    from scipy.stats import entropy
    r = np.random.default_rng(seed)
    counts = r.integers(1, 40, size=r.integers(1, 30))
    vals = r.permutation(np.arange(len(counts)))
    x = np.repeat(vals, counts).astype(np.float32) / 8.0
    y = np.repeat(vals % 3, counts).astype(np.float32)
    perm = r.permutation(len(x))
    assert orc.window_entropy(x[perm], y[perm]) == pytest.approx(entropy(counts), abs=1e-12)


def _x_shape_tied_triple():
    """The X-shaped triple with a tie-heavy extension: 16-point ramp, then 4
    anti-diagonal points each taken twice, so H(w_d) = ln 4 against ln 8."""
    u = 1.0 / 4096.0
    j = np.repeat(np.arange(4), 2)
    x = np.concatenate([np.arange(16) * u, 4 * j * u]).astype(np.float32)
    y = np.concatenate([np.arange(16) * u, (15 - 4 * j) * u]).astype(np.float32)
    return x, y


# tau, expected noise bit under tau * H(w_d) (the empirical entropy, ln 4
# here); tau * ln|w_d| = tau ln 8 decides the first case the other way.
@pytest.mark.parametrize("tau,noise", [(0.0055, False), (0.0080, True)])
def test_noise_flag_entropy_threshold(orc, tau, noise):
    import oracle
    x, y = _x_shape_tied_triple()
    i_o = brute_mi(x[:16], y[:16], 4, 0)
    i_d = brute_mi(x[16:], y[16:], 4, 0)
    i_u = brute_mi(x, y, 4, 0)
    assert i_o > 0 and i_u < i_o and i_d > 0
    assert (i_d < tau * math.log(4)) == noise
    assert abs(i_d - tau * math.log(4)) > 0.001
    q = synth.make_queries(0, 1, 0, 16, 8, +1)
    r = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=2)[0]
    assert r["mi_ext"] == pytest.approx(i_d, abs=1e-12)
    assert bool(r["flags"] & oracle.FLAG_NOISE) == noise
    r1 = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=1)[0]
    assert bool(r1["flags"] & oracle.FLAG_NOISE) == (i_d < tau * math.log(8))
    if not noise:
        assert r1["flags"] & oracle.FLAG_NOISE  # the two readings part here


def test_entropy_threshold_equals_log_threshold_when_distinct(orc):
    """Tie-free extensions: the entropy reading reduces to tau * ln|w_d|."""
    x, y = synth.cfg2_pair(4096, 7)
    starts = np.arange(0, 3000, 37, dtype=np.uint64)
    q = synth.make_queries(0, 1, starts, 256, 64, +1)
    for tau in (0.01, 0.05, 0.2):
        a = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=1)
        b = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=2)
        for s in starts:
            e0 = int(s) + 256
            assert len(set(zip(x[e0:e0 + 64].tolist(), y[e0:e0 + 64].tolist()))) == 64
        assert np.array_equal(a["flags"], b["flags"])
