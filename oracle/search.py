"""The paper's search rules written out sequentially, window by window, for
tests.  Test infrastructure like the rest of ``oracle/``: only tests, the
smoke check and the CPU baseline of the benchmark use it.

``top_down`` follows Algorithm 1 (Section 5.1) with the noise pruning of
Section 6.2, taking every decision in the order the paper describes and
computing each estimate only when the rule asks for it.  ``mi(start, length)``
is any function giving I of the window [start, start + length); tests pass
the CPU oracle's estimator on a series pair, or a constructed function.

Readings (the library's driver takes the same ones):
* windows are half-open, so a window created by shifting w by delta splits
  into its overlap with w, [t, t + s_w - delta), and its new part
  [t + s_w - delta, t + s_w);
* after a correlated window, or a cancelled shift, the next window starts
  where the current one ends;
* the layers halve the window size from s_max while it is at least s_min,
  and the sliding step of a layer is max(1, s_w // step_div);
* the uncorrelated partitions handed to lower layers are the stretches of a
  partition not covered by its correlated windows, kept if at least s_min
  long;
* with ``normalize`` the thresholds scale with the window entropy of the
  normalised MI (Section 5.4): normalize=1 takes ln m, the entropy of m
  distinct samples (I_w >= sigma ln|w|, I(w_d) < tau ln|w_d|); normalize=2
  takes ``entropy(start, length)``, any function giving H of the window
  (tests pass the oracle's empirical entropy of the window's pairs).
"""
from __future__ import annotations

import math


def _scale(normalize, entropy, start: int, length: int) -> float:
    """The factor sigma and tau are multiplied by for the window [start,
    start + length): 1, ln length, or its entropy."""
    if normalize == 2:
        return entropy(start, length)
    return math.log(length) if normalize else 1.0


def top_down(mi, begin: int, end: int, s_max: int, s_min: int, sigma: float, tau: float = 0.0,
             p: int = 0, step_div: int = 8, normalize: int = 0, trace: list | None = None, entropy=None):
    """Correlated windows as (start, length, layer, I) in ascending start
    order.  ``trace`` (a list) receives every window the rule examines, as
    (layer, start)."""
    found = []
    partitions = [(begin, end)] if end - begin >= s_min else []
    s_w, layer = s_max, 0
    while s_w >= s_min and partitions:
        delta = max(1, s_w // step_div)
        pruning = p > 0 and delta < s_w
        lower = []
        for ps, pe in partitions:
            uncovered = ps
            t = ps
            came_by_shift = False
            detections = 0
            while t + s_w <= pe:
                if trace is not None:
                    trace.append((layer, t))
                I = mi(t, s_w)
                if I >= sigma * _scale(normalize, entropy, t, s_w):   # correlated: report, move past it
                    found.append((t, s_w, layer, I))
                    if t - uncovered >= s_min:
                        lower.append((uncovered, t))
                    uncovered = t + s_w
                    t += s_w
                    came_by_shift = False
                    detections = 0
                    continue
                noise = False
                if pruning and came_by_shift:          # Definition 6.2 on (overlap, new part)
                    I_o = mi(t, s_w - delta)
                    I_d = mi(t + s_w - delta, delta)
                    noise = I_o > 0 and I_d < tau * _scale(normalize, entropy, t + s_w - delta, delta) and I < I_o
                detections = detections + 1 if noise else 0
                if pruning and detections >= p:        # p detections in a row: no more shifting
                    t += s_w
                    came_by_shift = False
                    detections = 0
                else:
                    t += delta
                    came_by_shift = True
            if pe - uncovered >= s_min:
                lower.append((uncovered, pe))
        partitions = lower
        s_w //= 2
        layer += 1
    found.sort()
    return found


MASK64 = (1 << 64) - 1
GOLDEN64 = 0x9E3779B97F4A7C15


def splitmix64(z: int) -> int:
    """Output function of Steele, Lea and Flood's SplitMix64 generator."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def bottom_up(mi, begin: int, end: int, s_min: int, s_max: int, delta: int, sigma: float,
              max_idle: int = 2, history: int = 4, tau: float = 0.0, p: int = 0, normalize: int = 0,
              chunk: int = 0, seed: int = 0, trace: list | None = None, entropy=None):
    """Algorithm 2 (Section 5.2) with the directional pruning of Section 6.3,
    chunk by chunk, one climb after another.  Readings (the library's driver
    takes the same ones):
    * the first window of a climb is the s_min first points of the unexplored
      rest of the chunk; the next climb starts where the last one's window ends;
    * the neighbourhood examined when idle = i is the ring of windows whose
      start and end each move by at most r = i + 1 steps, one of them by
      exactly r (the 8 and 16 windows of the paper's figure for r = 1, 2),
      inside the rest, of s_min to s_max points, examined in order of start
      offset then end offset; the first largest estimate is the best;
    * the history entry compared and updated in an iteration is one pick,
      splitmix64(seed + (chunk * 2^32 + i) * golden) mod h for the walker's
      i-th pick (i = 1, 2, ...), the same entry for both uses;
    * pruning: the ring's pure left and pure right extensions are noise
      triples over w; a direction closes for the rest of the climb after p
      consecutive examined extensions of it were noise (Definition 6.2);
    * a window is reported when I >= sigma (normalize 1: sigma ln|w|;
      2: sigma H(w)); a noise test compares with tau, tau ln|w_d| or
      tau H(w_d) likewise.
    ``trace`` receives every examined window as (start, end)."""
    found = []
    size = chunk if chunk else max(end - begin, 1)
    c = 0
    for c0 in range(begin, end, size):
        c1 = min(end, c0 + size)
        n_picks = 0
        rest = c0
        while c1 - rest >= s_min:
            ws, we = rest, rest + s_min
            if trace is not None:
                trace.append((ws, we))
            Iw = mi(ws, s_min)
            hist = [Iw] * history
            idle = 0
            runs = {"left": 0, "right": 0}
            closed = {"left": False, "right": False}
            while idle <= max_idle:
                r = idle + 1
                best = None
                seen = {}
                for ds in range(-r, r + 1):
                    for de in range(-r, r + 1):
                        if max(abs(ds), abs(de)) != r:
                            continue
                        s, e = ws + ds * delta, we + de * delta
                        if s < rest or e > c1 or not (s_min <= e - s <= s_max):
                            continue
                        if (closed["left"] and ds < 0) or (closed["right"] and de > 0):
                            continue
                        if trace is not None:
                            trace.append((s, e))
                        I = mi(s, e - s)
                        if p and de == 0 and ds == -r:      # w extended on the left
                            ext = ws - s
                            thr = tau * _scale(normalize, entropy, s, ext)
                            seen["left"] = Iw > 0 and mi(s, ext) < thr and I < Iw
                        if p and ds == 0 and de == r:       # w extended on the right
                            ext = e - we
                            thr = tau * _scale(normalize, entropy, we, ext)
                            seen["right"] = Iw > 0 and mi(we, ext) < thr and I < Iw
                        if not math.isnan(I) and (best is None or I > best[2]):
                            best = (s, e, I)
                for side, noise in seen.items():
                    runs[side] = runs[side] + 1 if noise else 0
                n_picks += 1
                j = splitmix64(seed + ((c << 32) + n_picks) * GOLDEN64) % history
                if best is not None and (best[2] > hist[j] or best[2] > Iw):
                    ws, we, Iw = best
                    idle = 0
                else:
                    idle += 1
                if Iw > hist[j]:
                    hist[j] = Iw
                for side in ("left", "right"):
                    if p and runs[side] >= p:
                        closed[side] = True
            thr_w = sigma * _scale(normalize, entropy, ws, we - ws)
            if Iw >= thr_w:
                found.append((ws, we - ws, 0, Iw))
            rest = we
        c += 1
    found.sort()
    return found
