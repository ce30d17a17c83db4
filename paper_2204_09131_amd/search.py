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
