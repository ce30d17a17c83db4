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
* with ``normalize`` the thresholds scale with the entropy ln m of m distinct
  samples: I_w >= sigma ln|w| and I(w_d) < tau ln|w_d|.
"""
from __future__ import annotations

import math


def top_down(mi, begin: int, end: int, s_max: int, s_min: int, sigma: float, tau: float = 0.0,
             p: int = 0, step_div: int = 8, normalize: bool = False, trace: list | None = None):
    """Correlated windows as (start, length, layer, I) in ascending start
    order.  ``trace`` (a list) receives every window the rule examines, as
    (layer, start)."""
    found = []
    partitions = [(begin, end)] if end - begin >= s_min else []
    s_w, layer = s_max, 0
    while s_w >= s_min and partitions:
        delta = max(1, s_w // step_div)
        corr_thr = sigma * math.log(s_w) if normalize else sigma
        noise_thr = tau * math.log(delta) if normalize else tau
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
                if I >= corr_thr:                      # correlated: report, move past it
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
                    noise = I_o > 0 and I_d < noise_thr and I < I_o
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
