// wmi_ranges.h -- expansion of one query of a run (RangeDesc) into its window
// descriptors, query descriptor and work items.  Plain C++ usable on the host
// and the device: the expansion kernel runs it once per query, and the CPU
// plan checker runs the same code to verify the queue it writes.
#pragma once
#include "wmi_internal.h"

#ifdef __HIPCC__
#define WMI_HD __host__ __device__
#else
#define WMI_HD
#endif

namespace wmi {

// Sweep items of a run of n windows, C per item (n >= 2): k = (n - 2) / C full
// items when n > C + 1, then a tail of 2 .. C + 1 windows, cut in two halves
// when it is C + 1 >= 4 (never one window alone).  The item of window i and
// that item's first window and length.
WMI_HD inline void sweep_chunk(uint32_t n, uint32_t C, uint32_t i, uint32_t *item, uint32_t *first, uint32_t *len)
{
    const uint32_t k = n > C + 1u ? (n - 2u) / C : 0u;
    const uint32_t tail = n - k * C;
    if (i < k * C) {
        *item = i / C;
        *first = *item * C;
        *len = C;
        return;
    }
    const uint32_t j = i - k * C;
    if (tail == C + 1u && tail >= 4u) {
        const uint32_t h = tail / 2u;
        *item = k + (j < h ? 0u : 1u);
        *first = k * C + (j < h ? 0u : h);
        *len = j < h ? h : tail - h;
        return;
    }
    *item = k;
    *first = k * C;
    *len = tail;
}

WMI_HD inline uint32_t sweep_items(uint32_t n, uint32_t C)
{
    const uint32_t k = n > C + 1u ? (n - 2u) / C : 0u;
    const uint32_t tail = n - k * C;
    return k + ((tail == C + 1u && tail >= 4u) ? 2u : 1u);
}

// Windows of query i of R (a triple: base, extension, union).
WMI_HD inline void range_windows(const RangeDesc &R, uint32_t i, uint64_t st[3], uint32_t m[3])
{
    const uint64_t s = R.start + (uint64_t)i * R.stride;
    st[0] = s;
    m[0] = R.m;
    st[1] = R.side > 0 ? s + R.m : s - R.e;
    m[1] = R.e;
    st[2] = R.side > 0 ? s : s - R.e;
    m[2] = R.m + R.e;
}

// Descriptors and queue entries of query i of R.  Each item is written by
// the query of its first window, so every queue entry is written once.
WMI_HD inline void expand_query(const RangeDesc &R, uint32_t i, WinDesc *win, QDesc *qd, Item *queue)
{
    uint64_t st[3];
    uint32_t m[3];
    range_windows(R, i, st, m);
    const uint32_t q = R.q0 + i;
    const uint32_t nw = R.side == 0 ? 1u : 3u;
    const uint32_t w0 = R.win0 + nw * i;
    QDesc d;
    d.win0 = w0;
    d.nwin = nw;
    d.tau_eff = R.tau_eff;
    qd[q] = d;
    for (uint32_t r = 0; r < nw; ++r) {
        WinDesc w;
        w.x = R.x + st[r];
        w.y = R.y + st[r];
        w.m = m[r];
        w.query = q;
        w.sorted_off = 0u;
        w.n_items = 1u;
        win[w0 + r] = w;
    }
    switch (R.kind) {
    case kRangeLocal:
        if (i % R.per_item == 0u) {
            const uint32_t n = R.count - i < R.per_item ? R.count - i : R.per_item;
            queue[R.item0 + i / R.per_item] = Item{w0, kItemLocal | n};
        }
        break;
    case kRangeTriple:
        if (i % R.per_item == 0u) {
            const uint32_t n = R.count - i < R.per_item ? R.count - i : R.per_item;
            queue[R.item0 + i / R.per_item] = Item{w0, kItemTriple | n};
        }
        break;
    case kRangeSweep: {
        uint32_t it, first, len;
        sweep_chunk(R.count, R.per_item, i, &it, &first, &len);
        if (first == i)
            queue[R.item0 + it] = Item{w0, kItemSweep | len};
        break;
    }
    case kRangeSplit: {
        const uint32_t ns = (R.m + (uint32_t)kSplitPoints - 1u) / (uint32_t)kSplitPoints;
        win[w0].sorted_off = R.sorted0 + i * R.m;
        win[w0].n_items = ns;
        queue[R.prep0 + i] = Item{w0, kItemPrep};
        for (uint32_t t = 0; t < ns; ++t)
            queue[R.item0 + i * ns + t] = Item{w0, t * (uint32_t)kSplitPoints};
        break;
    }
    default: {  // kRangeTripleWide: per query L local windows, P split windows of SP points and S items
        uint32_t L = 0, P = 0, SP = 0, S = 0;
        for (uint32_t r = 0; r < 3u; ++r) {
            if (m[r] > (uint32_t)kLocalSlots) {
                P++;
                SP += m[r];
                S += (m[r] + (uint32_t)kSplitPoints - 1u) / (uint32_t)kSplitPoints;
            } else {
                L++;
            }
        }
        uint32_t l = 0, p = 0, sp = 0, sn = 0;
        for (uint32_t r = 0; r < 3u; ++r) {
            const uint32_t w = w0 + r;
            if (m[r] > (uint32_t)kLocalSlots) {
                const uint32_t ns = (m[r] + (uint32_t)kSplitPoints - 1u) / (uint32_t)kSplitPoints;
                win[w].sorted_off = R.sorted0 + i * SP + sp;
                win[w].n_items = ns;
                queue[R.prep0 + i * P + p] = Item{w, kItemPrep};
                for (uint32_t t = 0; t < ns; ++t)
                    queue[R.item1 + i * S + sn + t] = Item{w, t * (uint32_t)kSplitPoints};
                sp += m[r];
                sn += ns;
                p++;
            } else {
                queue[R.item0 + i * L + l] = Item{w, kItemLocal | 1u};
                l++;
            }
        }
        break;
    }
    }
}

}  // namespace wmi
