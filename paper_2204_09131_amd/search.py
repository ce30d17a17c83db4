"""Host-side helpers around the search drivers of the library."""
from __future__ import annotations


def overlap_accuracy(reference, candidate) -> float:
    """Share of the reference windows that overlap some candidate window.
    Two windows count as the same finding when their index ranges overlap,
    the similarity used to grade noise pruning against the search without it
    (Section 8, accuracy of noise pruning).  Windows are (start, length)
    pairs; the candidate windows must not overlap each other."""
    if len(reference) == 0:
        return 1.0
    c = sorted((int(s), int(s) + int(m)) for s, m in candidate)
    hits = 0
    j = 0
    for s, m in sorted((int(s), int(m)) for s, m in reference):
        e = s + m
        while j < len(c) and c[j][1] <= s:
            j += 1
        k = j
        while k < len(c) and c[k][0] < e:
            if c[k][1] > s:
                hits += 1
                break
            k += 1
    return hits / len(reference)


def efficiency_scores(t_td: float, t_bu: float, n_large_td: int, n_small_bu: int, alpha: float):
    """Normalised efficiency scores of the top-down and bottom-up searches
    (Section 5.3): runtimes and window counts are each normalised by their
    sum, then nscore = alpha / t~ + (1 - alpha) n~, with the count of large
    windows for top-down and of small windows for bottom-up.  When neither
    search found a window of its kind both counts are taken as 0."""
    t_sum = t_td + t_bu
    tt, tb = t_td / t_sum, t_bu / t_sum
    n_sum = n_large_td + n_small_bu
    nl = n_large_td / n_sum if n_sum else 0.0
    ns = n_small_bu / n_sum if n_sum else 0.0
    return alpha / tt + (1.0 - alpha) * nl, alpha / tb + (1.0 - alpha) * ns


def count_windows(windows, rho: float, s_max: int):
    """(small, large) windows: a window is small when |w| <= rho * s_max."""
    small = sum(1 for w in windows if int(w["len"]) <= rho * s_max)
    return small, len(windows) - small


def isycos(store, a: int, b: int, begin: int, end: int, td: dict, bu: dict, M: int = 64, m: int = 6,
           alpha: float = 0.5, rho: float = 0.5, seed: int = 0):
    """Integrated search (Algorithm 3): cut [begin, end) into M partitions of
    floor(N / M) points, draw m of them at random, run both searches on each
    and time them, score both with efficiency_scores, and run the selected
    search on the whole range.  td and bu are the keyword arguments of
    Store.td_search and Store.bu_search (without the range)."""
    import time

    import numpy as np
    n = end - begin
    L = n // M
    pick = np.sort(np.random.Generator(np.random.PCG64(seed)).choice(M, size=min(m, M), replace=False))
    t_td = t_bu = 0.0
    w_td, w_bu = [], []
    for i in pick:
        s0 = begin + int(i) * L
        t0 = time.perf_counter()
        got, _ = store.td_search(a, b, s0, s0 + L, **td)
        t_td += time.perf_counter() - t0
        w_td.extend(got)
        t0 = time.perf_counter()
        got, _ = store.bu_search(a, b, s0, s0 + L, **bu)
        t_bu += time.perf_counter() - t0
        w_bu.extend(got)
    t_td /= len(pick)
    t_bu /= len(pick)
    s_max = td["s_max"]
    _, n_large_td = count_windows(w_td, rho, s_max)
    n_small_bu, _ = count_windows(w_bu, rho, s_max)
    score_td, score_bu = efficiency_scores(t_td, t_bu, n_large_td, n_small_bu, alpha)
    selected = "top-down" if score_td > score_bu else "bottom-up"
    t0 = time.perf_counter()
    if selected == "top-down":
        windows, stats = store.td_search(a, b, begin, end, **td)
    else:
        windows, stats = store.bu_search(a, b, begin, end, **bu)
    return {"selected": selected, "nscore_td": score_td, "nscore_bu": score_bu, "t_td": t_td, "t_bu": t_bu,
            "n_large_td": n_large_td, "n_small_bu": n_small_bu, "partitions": [int(i) for i in pick],
            "windows": windows, "stats": stats, "search_seconds": time.perf_counter() - t0}
