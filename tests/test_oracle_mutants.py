"""Plant plausible mistakes in copies of the oracle source, on the CPU, and
check that the pins catch every one of them (a dropped term, a wrong sign or
index, a transposed operand, a flipped comparison, a wrong tie-break).

The unmutated source must pass the same compact pin suite.
"""
import json
import math
import os
import shutil
import tempfile

import numpy as np
import pytest
from scipy.special import digamma

import oracle
from paper_2204_09131_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MUTANTS = {
    "strict_count": ("<= rx) ++cx;", "< rx) ++cx;"),
    "count_self": ("""            for (int j = 0; j < m; ++j) {
                if (j == i)
                    continue;
                if (fabs((double)x[i] - (double)x[j]) <= rx)""",
                   """            for (int j = 0; j < m; ++j) {
                if (fabs((double)x[i] - (double)x[j]) <= rx)"""),
    "sign_of_1_over_k": ("psi(k) - 1.0 / (double)k + psi(m)", "psi(k) + 1.0 / (double)k + psi(m)"),
    "dropped_1_over_k": ("psi(k) - 1.0 / (double)k + psi(m)", "psi(k) + psi(m)"),
    "psi_m_index": ("- 1.0 / (double)k + psi(m))", "- 1.0 / (double)k + psi(m - 1))"),
    "min_norm": ("return dx > dy ? dx : dy;", "return dx < dy ? dx : dy;"),
    "transposed_eps": ("double dx = fabs((double)x[i] - (double)x[chosen[r]]);",
                       "double dx = fabs((double)y[i] - (double)y[chosen[r]]);"),
    "tie_break_reversed": ("(d == best_d && j < best_j)", "(d == best_d && j > best_j)"),
    "mean_over_m_minus_1": ("- s / (double)m;\n    } else", "- s / (double)(m - 1);\n    } else"),
    "ksg1_le": ("< dk) ++cx;", "<= dk) ++cx;"),
    "psi_recurrence_off_by_one": ("acc += 1.0L / (long double)n;", "acc += 1.0L / (long double)(n + 1);"),
    "psi_table_shift": ("""        psi_tab[n] = (double)acc;
        acc += 1.0L / (long double)n;""", """        acc += 1.0L / (long double)n;
        psi_tab[n] = (double)acc;"""),
    "k_minus_one_neighbours": ("for (int r = 0; r < k; ++r) {\n            int best_j", "for (int r = 0; r < k - 1; ++r) {\n            int best_j"),
    "noise_ext_compare": ("r.mi_ext < tau_eff && r.mi_union < r.mi_base", "r.mi_ext < tau_eff && r.mi_union > r.mi_base"),
    "noise_ext_side_swapped": ("q->start + q->len : q->start - q->ext_len", "q->start - q->ext_len : q->start + q->len"),
    # the normalised threshold tau * ln|w_d| of the new part
    "tau_norm_log2": ("tau_eff = tau * log((double)q->ext_len);", "tau_eff = tau * log2((double)q->ext_len);"),
    "tau_norm_union": ("tau_eff = tau * log((double)q->ext_len);",
                       "tau_eff = tau * log((double)(q->len + q->ext_len));"),
    "tau_norm_base": ("tau_eff = tau * log((double)q->ext_len);", "tau_eff = tau * log((double)q->len);"),
    "tau_norm_ignored": ("tau_eff = tau * log((double)q->ext_len);", "tau_eff = tau;"),
    # the window entropy of Section 5.4 and the threshold tau * H(w_d)
    "entropy_sign": ("h -= p * log(p);", "h += p * log(p);"),
    "entropy_log2": ("h -= p * log(p);", "h -= p * log2(p);"),
    "entropy_x_only": ("""            if (x[j] == x[i] && y[j] == y[i])
                ++c;""", """            if (x[j] == x[i])
                ++c;"""),
    "entropy_every_point": ("""        if (!first)
            continue;""", ""),
    "entropy_over_m_minus_1": ("(double)c / (double)m;", "(double)c / (double)(m - 1);"),
    "tau_entropy_of_base": ("oracle_window_entropy(series[q->a] + ext_start, series[q->b] + ext_start,\n"
                            "                                                          (int)q->ext_len)",
                            "oracle_window_entropy(series[q->a] + q->start, series[q->b] + q->start,\n"
                            "                                                          (int)q->len)"),
    "tau_entropy_as_ln": ("tau_eff = tau * oracle_window_entropy(", "tau_eff = tau * 0.0 + tau * log((double)q->ext_len) + 0.0 * oracle_window_entropy("),
}


def pin_suite(orc):
    """A compact subset of the pins; raises AssertionError on the first miss."""
    # psi against scipy
    tab = orc.psi_table(5000)
    assert np.max(np.abs(tab - digamma(np.arange(1, 5001.0)))) < 1e-13
    # worked example
    g = json.load(open(os.path.join(GOLDEN, "worked_example_7pt.json")))
    pts = np.array([g["points"][n] for n in g["order"]], dtype=np.float32)
    r = orc.window_counts(pts[:, 0], pts[:, 1], k=2, estimator=0)
    assert (r["nx"][0], r["ny"][0]) == (3, 3)
    # closed form
    for m in (32, 256):
        x = (np.arange(m) / 4096.0).astype(np.float32)
        assert abs(orc.window_mi(x, x, 4, 0) - (digamma(m) - digamma(4) - 0.25)) < 1e-12
    # brute force with a full sort, tie-heavy
    from test_oracle_pins import brute
    for seed in range(6):
        for k in (1, 2, 4):
            x, y = synth.grid_points(13, seed, levels=3, scale=0.25)
            rr = orc.window_counts(x, y, k=k, estimator=0)
            nx, ny, ex, ey = brute(x, y, k, 0)
            assert np.array_equal(rr["nx"], nx) and np.array_equal(rr["ny"], ny)
            assert np.array_equal(rr["eps_x"], ex) and np.array_equal(rr["eps_y"], ey)
            assert np.array_equal(rr["nbr"][:, :k], np.array([
                [j for _, j in sorted((max(abs(float(x[i]) - float(x[j])), abs(float(y[i]) - float(y[j]))), j)
                                      for j in range(13) if j != i)[:k]] for i in range(13)]))
            rr = orc.window_counts(x, y, k=k, estimator=1)
            nx, ny, _, _ = brute(x, y, k, 1)
            assert np.array_equal(rr["nx"], nx) and np.array_equal(rr["ny"], ny)
    # scikit-learn's first estimator
    from sklearn.feature_selection._mutual_info import _compute_mi_cc
    x, y = synth.relation("quadratic", 300, 1)
    assert abs(orc.window_mi(x, y, 4, 1) - _compute_mi_cc(x.astype(float), y.astype(float), 4)) < 1e-12
    # noise flag, both sides
    rg = synth.rng(77)
    n = 1024
    xs = rg.standard_normal(n)
    yl = 0.9 * xs + 0.1 * rg.standard_normal(n)
    ym = yl.copy()
    ym[512:] = rg.standard_normal(n - 512)
    q = synth.make_queries(0, 1, 0, 512, 256, +1)
    res = orc.batch([synth.quantize(xs), synth.quantize(ym)], q, k=4, tau=0.1)[0]
    assert res["flags"] & oracle.FLAG_NOISE
    yleft = yl.copy()
    yleft[:512] = rg.standard_normal(512)
    xq, yq = synth.quantize(xs), synth.quantize(yleft)
    q = synth.make_queries(0, 1, 512, 256, 256, -1)
    res = orc.batch([xq, yq], q, k=4, tau=0.1)[0]
    assert res["mi_ext"] == orc.window_mi(xq[256:512], yq[256:512], 4, 0)
    assert res["flags"] & oracle.FLAG_NOISE
    # normalised threshold tau * ln|w_d| on the X-shaped triple (closed forms
    # I(w_d) = psi(8) - psi(4) - 1/4 = 0.5095 against tau ln 8)
    from test_oracle_pins import _x_shape_triple
    x, y = _x_shape_triple()
    q = synth.make_queries(0, 1, 0, 16, 8, +1)
    for tau, noise in ((0.22, False), (0.30, True)):
        res = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=1)[0]
        assert bool(res["flags"] & oracle.FLAG_NOISE) == noise
    # window entropy: closed forms, counts, and the threshold tau * H(w_d)
    m = 7
    v = (np.arange(m) / 4096.0).astype(np.float32)
    assert abs(orc.window_entropy(v, v[::-1].copy()) - math.log(m)) < 1e-12
    xg = np.array([0, 0, 0, 1], dtype=np.float32)
    yg = np.array([0, 1, 1, 0], dtype=np.float32)
    assert abs(orc.window_entropy(xg, yg) - 1.5 * math.log(2)) < 1e-12
    from scipy.stats import entropy
    counts = np.array([3, 9, 1, 5])
    xc = np.repeat(np.arange(4), counts).astype(np.float32)
    assert abs(orc.window_entropy(xc, xc) - entropy(counts)) < 1e-12
    from test_oracle_pins import _x_shape_tied_triple
    x, y = _x_shape_tied_triple()
    for tau, noise in ((0.0055, False), (0.0080, True)):
        res = orc.batch([x, y], q, k=4, tau=tau, tau_normalize=2)[0]
        assert bool(res["flags"] & oracle.FLAG_NOISE) == noise


@pytest.fixture(scope="module")
def tmpdir_mod():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _build(src_text, tmpdir, name):
    src = os.path.join(tmpdir, name + ".c")
    with open(src, "w") as f:
        f.write(src_text)
    lib = oracle.compile_oracle(src, os.path.join(tmpdir, "lib" + name + ".so"))
    return oracle.Oracle(lib)


def test_unmutated_passes(tmpdir_mod):
    pin_suite(_build(open(oracle.SRC).read(), tmpdir_mod, "clean"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmpdir_mod, name):
    old, new = MUTANTS[name]
    text = open(oracle.SRC).read()
    assert text.count(old) >= 1, name
    orc = _build(text.replace(old, new, 1), tmpdir_mod, name)
    with pytest.raises(AssertionError):
        pin_suite(orc)
