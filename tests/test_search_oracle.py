"""Pins of the sequential search rules in oracle/search.py, on constructed
estimate functions whose outcome can be worked out by hand from Algorithm 1
(Section 5.1) and the pruning rule of Section 6.2."""
import math

import pytest

from oracle import search


def test_everything_correlated_tiles_each_layer():
    # sigma = -inf: every examined window is correlated.  Layer 0 tiles
    # [0, 1000) with 256-point windows from 0; the 232-point tail goes down to
    # 128, then its 104-point tail to 64; 40 points are left.
    found = search.top_down(lambda t, m: 0.0, 0, 1000, 256, 64, -math.inf)
    assert [(s, m, l) for s, m, l, _ in found] == [
        (0, 256, 0), (256, 256, 0), (512, 256, 0), (768, 128, 1), (896, 64, 2)]


def test_nothing_correlated_slides_every_layer_over_everything():
    trace = []
    found = search.top_down(lambda t, m: 0.0, 0, 1000, 256, 64, math.inf, trace=trace)
    assert found == []
    # steps 32, 16, 8: starts 0..744, 0..872, 0..936
    assert len(trace) == (744 // 32 + 1) + (872 // 16 + 1) + (936 // 8 + 1) == 197
    assert trace[:3] == [(0, 0), (0, 32), (0, 64)] and trace[-1] == (2, 936)


def test_planted_block():
    # I = 1 for windows inside [300, 700), else 0.  Layer 0 (256, step 32)
    # finds [320, 576); layer 1 (128, step 16) fits nothing inside either
    # remaining partition; layer 2 (64, step 8) finds [576, 640) in
    # [576, 1000) and nothing in [0, 320).
    def mi(t, m):
        return 1.0 if (t >= 300 and t + m <= 700) else 0.0
    found = search.top_down(mi, 0, 1000, 256, 64, 0.5)
    assert [(s, m, l) for s, m, l, _ in found] == [(320, 256, 0), (576, 64, 2)]


def test_noise_pruning_cancels_shifts_after_p_detections():
    # Every shifted 64-point window is noise w.r.t. its overlap (I_o = 0.4 > 0,
    # I_d = 0 < tau, I = 0.3 < I_o) and nothing is correlated.  With p = 2:
    # 0 (not shifted) -> 8 (1st detection) -> 16 (2nd: skip) -> 80 -> 88 ->
    # 96 (skip) -> 160, which no longer fits in [0, 200).
    def mi(t, m):
        return {64: 0.3, 56: 0.4, 8: 0.0}[m]
    trace = []
    found = search.top_down(mi, 0, 200, 64, 64, 0.5, tau=0.1, p=2, trace=trace)
    assert found == []
    assert [t for _, t in trace] == [0, 8, 16, 80, 88, 96]
    # without pruning every step is taken
    trace = []
    search.top_down(mi, 0, 200, 64, 64, 0.5, tau=0.1, p=0, trace=trace)
    assert [t for _, t in trace] == list(range(0, 137, 8))


@pytest.mark.parametrize("case", ["nonpositive_base", "union_not_lower", "new_part_informative"])
def test_noise_needs_all_three_conditions(case):
    # Definition 6.2: I(w_o) > 0, I(w_d) < tau and I(w'') < I(w_o); break one
    # condition and no shift is ever cancelled.
    vals = {"nonpositive_base": {64: 0.3, 56: 0.0, 8: 0.0},
            "union_not_lower": {64: 0.45, 56: 0.4, 8: 0.0},
            "new_part_informative": {64: 0.3, 56: 0.4, 8: 0.2}}[case]
    trace = []
    search.top_down(lambda t, m: vals[m], 0, 200, 64, 64, 0.5, tau=0.1, p=1, trace=trace)
    assert [t for _, t in trace] == list(range(0, 137, 8))


def test_detections_must_be_consecutive():
    # Noise only on shifted windows starting at multiples of 16: detections
    # never come twice in a row, so p = 2 cancels nothing, while p = 1 jumps
    # after the first detection (8 is not noise, 16 is).
    def mi(t, m):
        if m == 64:
            return 0.3
        if m == 56:
            return 0.4
        return 0.0 if (t - 56) % 16 == 0 else 0.2
    trace = []
    search.top_down(mi, 0, 200, 64, 64, 0.5, tau=0.1, p=2, trace=trace)
    assert [t for _, t in trace] == list(range(0, 137, 8))
    trace = []
    search.top_down(mi, 0, 200, 64, 64, 0.5, tau=0.1, p=1, trace=trace)
    assert [t for _, t in trace] == [0, 8, 16, 80, 88, 96]


def test_normalized_thresholds():
    # normalize: correlated iff I >= sigma ln|w|.  I = 0.45 ln 64 meets
    # sigma = 0.45 exactly at 64 points and falls short at 128 (ln 128 > ln 64)
    v = 0.45 * math.log(64)
    found = search.top_down(lambda t, m: v, 0, 128, 128, 64, 0.45, normalize=True)
    assert [(s, m) for s, m, _, _ in found] == [(0, 64), (64, 64)]


def test_splitmix64_reference_value():
    # first output of SplitMix64 seeded with 0 (the published reference
    # generator's value): mix(0 + golden)
    assert search.splitmix64(0 + search.GOLDEN64) == 0xE220A8397B1DCDAF


def test_bottom_up_hill_climb_by_hand():
    # I = |w| / 1000, one history entry (plain hill climbing), s_min 64,
    # s_max 128, step 16, max_idle 1 on [0, 300): each climb grows its end to
    # 128 points, then two rings bring nothing larger; climbs start at 0 and
    # 128, and 44 points are left.
    found = search.bottom_up(lambda s, m: m / 1000.0, 0, 300, 64, 128, 16, 0.1, max_idle=1, history=1)
    assert [(s, m) for s, m, _, _ in found] == [(0, 128), (128, 128)]
    # below the threshold nothing is reported
    assert search.bottom_up(lambda s, m: m / 1000.0, 0, 300, 64, 128, 16, 0.2, max_idle=1, history=1) == []


def test_bottom_up_first_largest_wins_and_climbs_stay_in_their_chunk():
    trace = []
    found = search.bottom_up(lambda s, m: m / 1000.0, 0, 600, 64, 128, 16, 0.1, max_idle=1, history=1,
                             chunk=300, trace=trace)
    assert [(s, m) for s, m, _, _ in found] == [(0, 128), (128, 128), (300, 128), (428, 128)]
    assert all(e <= 300 or s >= 300 for s, e in trace)


def test_bottom_up_left_pruning_by_hand():
    # I = start / 1000 for windows of 32 points or more, 0 below: moving right
    # pays, and every pure left extension is noise (its 16 new points score
    # 0 < tau, the union scores below w, and I(w) > 0 once w left 0), while no
    # right extension is (its union scores the same as w).  Range [0, 96),
    # s_min 32, s_max 64, step 16, max_idle 0, one history entry, p = 1: the
    # left side closes in the second ring, and the climb ends at [64, 96).
    def mi(s, m):
        return s / 1000.0 if m >= 32 else 0.0
    trace = []
    found = search.bottom_up(mi, 0, 96, 32, 64, 16, 0.05, max_idle=0, history=1, tau=0.1, p=1, trace=trace)
    assert [(s, m) for s, m, _, _ in found] == [(64, 32)]
    assert trace == [(0, 32),
                     (0, 48), (16, 48),                               # ring of [0, 32)
                     (0, 32), (0, 48), (0, 64), (16, 64), (32, 64),   # ring of [16, 48): left noise
                     (32, 80), (48, 80),                              # ring of [32, 64), left closed
                     (48, 96), (64, 96)]                              # ring of [48, 80); [64, 96)'s is empty
    trace0 = []
    search.bottom_up(mi, 0, 96, 32, 64, 16, 0.05, max_idle=0, history=1, tau=0.1, p=0, trace=trace0)
    assert trace0[8:11] == [(16, 48), (16, 64), (16, 80)]  # without pruning the left side stays open


# ---------------------------------------------------------------------------
# normalised thresholds: sigma ln|w| for a correlated window, tau ln|w_d| for
# the new part of a shifted or extended window (Eq. normalizedMI with the
# entropy of |w| distinct samples)
# ---------------------------------------------------------------------------

def td_normalized_noise_case(srch, v):
    """Top-down, one layer of 64-point windows, step 8, p = 1, tau = 0.1,
    nothing correlated (sigma ln 64 = 41.6).  The new part scores v against
    tau ln 8 = 0.2079: v = 0.15 is noise (and would not be under the raw
    threshold 0.1 or 0.1 log10 8 = 0.090), v = 0.25 is not (and would be
    under 0.1 log2 8 = 0.3, 0.1 ln 64 = 0.416 or 0.1 ln 56 = 0.403)."""
    vals = {64: 0.3, 56: 0.4, 8: v}
    trace = []
    srch.top_down(lambda t, m: vals[m], 0, 200, 64, 64, 10.0, tau=0.1, p=1, normalize=True, trace=trace)
    return [t for _, t in trace]


def bu_normalized_noise_case(srch, v):
    """The left-pruning climb below with normalised thresholds: windows of 32
    points or more score start / 1000, the 16-point new parts score v against
    tau ln 16 = 0.2773 (tau = 0.1).  v = 0.2 is noise, so the left side closes
    in the ring of [16, 48); v = 0.3 is not, so it stays open.  The raw
    threshold (0.1) would keep it open at 0.2; 0.1 log2 16 = 0.4, 0.1 ln 48
    (the union) = 0.387 and 0.1 ln 32 (the base) = 0.347 would close it at
    0.3.  sigma ln 32 = 0.0347 reports the final [64, 96) (I = 0.064)."""
    def mi(s, m):
        return s / 1000.0 if m >= 32 else v
    trace = []
    found = srch.bottom_up(mi, 0, 96, 32, 64, 16, 0.01, max_idle=0, history=1, tau=0.1, p=1, normalize=True,
                           trace=trace)
    return found, trace


def bu_normalized_report_case(srch, sigma):
    """Hill climb of I = |w| / 1000 ending at 128-point windows (I = 0.128):
    reported iff 0.128 >= sigma ln 128, i.e. for sigma = 0.026 (0.1262) and
    not for sigma = 0.027 (0.1310); sigma log2 128 = 0.182 would report
    neither, the raw sigma both."""
    found = srch.bottom_up(lambda s, m: m / 1000.0, 0, 300, 64, 128, 16, sigma, max_idle=1, history=1,
                           normalize=True)
    return [(s, m) for s, m, _, _ in found]


PRUNED_LEFT_TRACE = [(0, 32), (0, 48), (16, 48), (0, 32), (0, 48), (0, 64), (16, 64), (32, 64), (32, 80),
                     (48, 80), (48, 96), (64, 96)]


def td_entropy_noise_case(srch):
    """normalize=2: the thresholds take the window entropy H(start, length)
    given by the caller.  The 64-point layer of the first case with the new
    part scoring 0.15 and H = ln|w| except for the window starting at 64,
    whose entropy is halved (ties): tau H = 0.104 there, so the first shift
    (new part [64, 72)) is not noise and the second ([72, 80)) is."""
    vals = {64: 0.3, 56: 0.4, 8: 0.15}
    ent = lambda s, m: math.log(m) * (0.5 if s == 64 else 1.0)  # noqa: E731
    trace = []
    srch.top_down(lambda t, m: vals[m], 0, 200, 64, 64, 10.0, tau=0.1, p=1, normalize=2, trace=trace, entropy=ent)
    return [t for _, t in trace]


def bu_entropy_cases(srch):
    """normalize=2 with every window's entropy half of ln|w|: the left
    extensions' new parts (0.2) stay above tau H = 0.139, so the left side
    stays open; the climb of I = |w| / 1000 to 128 points (0.128) is reported
    for sigma = 0.05 (sigma H = 0.121) and not for 0.054 (0.131)."""
    ent = lambda s, m: 0.5 * math.log(m)  # noqa: E731
    trace = []
    srch.bottom_up(lambda s, m: s / 1000.0 if m >= 32 else 0.2, 0, 96, 32, 64, 16, 0.01, max_idle=0, history=1,
                   tau=0.1, p=1, normalize=2, trace=trace, entropy=ent)
    rep = [[(s, m) for s, m, _, _ in srch.bottom_up(lambda s, m: m / 1000.0, 0, 300, 64, 128, 16, sg, max_idle=1,
                                                     history=1, normalize=2, entropy=ent)] for sg in (0.05, 0.054)]
    return trace, rep


def td_report_case(srch, normalize):
    """64-point windows score 0.3, new parts 0.25 (never noise), sigma 0.1:
    0.3 < sigma ln 64 = 0.416, so nothing is correlated with normalize=1,
    though the raw sigma would report every window; with normalize=2 and the
    window at 0 of entropy ln 64 / 2 (sigma H = 0.208) that one is."""
    vals = {64: 0.3, 56: 0.4, 8: 0.25}
    ent = lambda s, m: math.log(m) * (0.5 if s == 0 else 1.0)  # noqa: E731
    trace = []
    srch.top_down(lambda t, m: vals[m], 0, 200, 64, 64, 0.1, tau=0.1, p=1, normalize=normalize, trace=trace,
                  entropy=ent)
    return [t for _, t in trace]


def normalized_pin_suite(srch):
    assert td_report_case(srch, 1) == list(range(0, 137, 8))
    assert td_report_case(srch, 2) == [0] + list(range(64, 137, 8))
    assert td_entropy_noise_case(srch) == [0, 8, 16, 80, 88]
    trace, rep = bu_entropy_cases(srch)
    assert trace[8:11] == [(16, 48), (16, 64), (16, 80)]
    assert rep == [[(0, 128), (128, 128)], []]
    assert td_normalized_noise_case(srch, 0.15) == [0, 8, 72, 80]
    assert td_normalized_noise_case(srch, 0.25) == list(range(0, 137, 8))
    found, trace = bu_normalized_noise_case(srch, 0.2)
    assert trace == PRUNED_LEFT_TRACE and [(s, m) for s, m, _, _ in found] == [(64, 32)]
    found, trace = bu_normalized_noise_case(srch, 0.3)
    assert trace[8:11] == [(16, 48), (16, 64), (16, 80)]
    assert bu_normalized_report_case(srch, 0.026) == [(0, 128), (128, 128)]
    assert bu_normalized_report_case(srch, 0.027) == []


def test_normalized_noise_and_report_thresholds():
    normalized_pin_suite(search)


SEARCH_MUTANTS = {
    "scale_log2": ("return math.log(length) if normalize else 1.0", "return math.log2(length) if normalize else 1.0"),
    "scale_entropy_ignored": ("""    if normalize == 2:
        return entropy(start, length)
""", ""),
    "td_corr_raw": ("if I >= sigma * _scale(normalize, entropy, t, s_w):", "if I >= sigma:"),
    "td_noise_window": ("tau * _scale(normalize, entropy, t + s_w - delta, delta)", "tau * _scale(normalize, entropy, t, s_w)"),
    "td_noise_overlap": ("tau * _scale(normalize, entropy, t + s_w - delta, delta)",
                         "tau * _scale(normalize, entropy, t, s_w - delta)"),
    "td_noise_entropy_start": ("tau * _scale(normalize, entropy, t + s_w - delta, delta)",
                               "tau * _scale(normalize, entropy, t, delta)"),
    "td_noise_raw": ("I_d < tau * _scale(normalize, entropy, t + s_w - delta, delta)", "I_d < tau"),
    "bu_noise_union": ("thr = tau * _scale(normalize, entropy, s, ext)", "thr = tau * _scale(normalize, entropy, s, e - s)"),
    "bu_noise_base": ("thr = tau * _scale(normalize, entropy, s, ext)", "thr = tau * _scale(normalize, entropy, ws, we - ws)"),
    "bu_noise_raw": ("thr = tau * _scale(normalize, entropy, s, ext)", "thr = tau"),
    "bu_report_raw": ("thr_w = sigma * _scale(normalize, entropy, ws, we - ws)", "thr_w = sigma"),
}


@pytest.mark.parametrize("name", sorted(SEARCH_MUTANTS))
def test_search_mutant_is_caught(name):
    import types
    old, new = SEARCH_MUTANTS[name]
    text = open(search.__file__).read()
    assert text.count(old) >= 1, name
    mod = types.ModuleType("search_mutant_" + name)
    exec(compile(text.replace(old, new), search.__file__ + ":" + name, "exec"), mod.__dict__)
    with pytest.raises(AssertionError):
        normalized_pin_suite(mod)
