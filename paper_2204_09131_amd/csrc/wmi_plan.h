// wmi_plan.h -- host-side work list of a batch (no HIP dependency).
//
// Windows above kLocalSlots points are split into blocks of kSplitPoints
// query points; their marginals are sorted by the prep kernel (prep_list).
// The other windows are packed, in window order, into local items of at most
// kLocalWindows consecutive windows, kLocalSlots points (each window padded
// to an even count) and kLocalSort sort entries (windows x the power of two
// at or above the largest m).  A query whose windows are all local and fit one
// item is never cut across items; otherwise its windows may land in several
// items and the kernel completes it with atomics.  In the plain form every
// window is alone.  Items carry a cost (work estimate) for largest-first
// ordering.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

#include "wmi_internal.h"
#include "wmi_ranges.h"

namespace wmi {

struct Plan {
    std::vector<Item> items;
    std::vector<uint64_t> cost;
    std::vector<uint32_t> prep_list;   // split windows
    std::vector<uint32_t> wsorted;     // per window: offset of its sorted marginals (split windows)
    std::vector<uint32_t> wnitems;     // per window: split items (1 for local windows)
    std::vector<uint32_t> first_item;  // plain form: first item of each window, plus the end
    std::vector<int32_t> wprep;        // plain form: prep-list entry of each window, or -1
    uint64_t split_pts = 0;
};

// The power of two at or above v (1 for v <= 1).
inline uint32_t plan_pow2(uint32_t v)
{
    return v <= 1u ? 1u : 1u << (32 - __builtin_clz(v - 1u));
}

// wm[w]: points of window w; wquery[w]: its query (non-decreasing, every query
// in [0, count) present).  A query of three windows is a noise triple (base,
// extension, union); with fuse_triples (batched form only) triples whose
// union has at most kLocalSlots points go to triple items: consecutive
// triples, up to kTripleMax of them, kLocalSlots union points (each padded
// to even) and kLocalSort sort entries (triples x the power of two at or
// above the largest union).  With wx, wy (the address of each window's
// first x and y value) runs of one-window queries of the same m whose
// windows advance by a constant stride s in both series (kSweepMinM <= m,
// m + s <= kSweepRing, kSweepStrideDiv s <= m) go to sweep items of
// kSweepWindows windows (the last one or two items of a run share its
// remainder, never leaving one window alone).  Reuse (triple and sweep items)
// is off with fuse_triples false.  tune (null: defaults) caps windows per
// local item, triples per triple item and windows per sweep item by window
// size.
inline void plan_items(const std::vector<uint32_t> &wm, const std::vector<uint32_t> &wquery, uint64_t count,
                       bool plain, Plan &out, bool fuse_triples = true, const std::vector<uint64_t> *wx = nullptr,
                       const std::vector<uint64_t> *wy = nullptr, const Tuning *tune = nullptr)
{
    const Tuning T = tune ? *tune : default_tuning();
    const uint64_t n_win = wm.size();
    out = Plan();
    out.wsorted.assign(n_win, 0);
    out.wnitems.assign(n_win, 1);
    if (plain) {
        out.first_item.reserve(n_win + 1);
        out.wprep.assign(n_win, -1);
    }
    struct Cur {
        uint32_t start = 0, n = 0, slots = 0, maxm = 0;
        uint64_t cost = 0;
    } cur;
    auto fits = [&T](const Cur &c, uint32_t m) {
        uint32_t maxm = std::max(std::max(c.maxm, m), 2u);
        const uint32_t cap = std::min<uint32_t>(std::max(T.local_windows[local_bucket(maxm)], 1u), kLocalWindows);
        return c.n + 1 <= cap && c.slots + ((m + 1u) & ~1u) <= (uint32_t)kLocalSlots &&
               (c.n + 1) * plan_pow2(maxm) <= (uint32_t)kLocalSort;
    };
    auto add = [](Cur &c, uint32_t w, uint32_t m) {
        if (c.n == 0)
            c.start = w;
        c.n++;
        c.slots += (m + 1u) & ~1u;
        c.maxm = std::max(c.maxm, m);
        c.cost += (uint64_t)m * m + 4096u;  // fixed per-window share of the item's overhead
    };
    auto close = [&]() {
        if (cur.n) {
            out.items.push_back(Item{cur.start, kItemLocal | cur.n});
            out.cost.push_back(cur.cost);
        }
        cur = Cur();
    };
    Cur tri;  // the open triple item: n triples from window start
    auto fits_tri = [&T](const Cur &c, uint32_t mu) {
        uint32_t maxm = std::max(std::max(c.maxm, mu), 2u);
        const uint32_t cap = std::min<uint32_t>(std::max(T.triples[local_bucket(maxm)], 1u), kTripleMax);
        return c.n + 1 <= cap && c.slots + ((mu + 1u) & ~1u) <= (uint32_t)kLocalSlots &&
               (c.n + 1) * plan_pow2(maxm) <= (uint32_t)kLocalSort;
    };
    auto close_tri = [&]() {
        if (tri.n) {
            out.items.push_back(Item{tri.start, kItemTriple | tri.n});
            out.cost.push_back(tri.cost);
        }
        tri = Cur();
    };
    // the window is its query's only one
    auto single = [&](uint64_t v) {
        return (v == 0 || wquery[v - 1] != wquery[v]) && (v + 1 >= n_win || wquery[v + 1] != wquery[v]);
    };
    const bool sweeps = !plain && fuse_triples && wx && wy && wx->size() == n_win && wy->size() == n_win;
    uint32_t w = 0;
    for (uint64_t t = 0; t < count; ++t) {
        const uint32_t w0 = w;
        uint32_t nw = 0;
        while (w0 + nw < n_win && wquery[w0 + nw] == (uint32_t)t)
            ++nw;
        if (sweeps && nw == 1 && w0 + 1 < n_win && single(w0 + 1) && wm[w0 + 1] == wm[w0]) {
            // a run of equally spaced one-window queries
            const uint32_t m = wm[w0];
            const int64_t dx = (int64_t)((*wx)[w0 + 1] - (*wx)[w0]), dy = (int64_t)((*wy)[w0 + 1] - (*wy)[w0]);
            const int64_t s = dx / (int64_t)sizeof(float);
            if (dx == dy && dx > 0 && dx % (int64_t)sizeof(float) == 0 && m >= (uint32_t)kSweepMinM &&
                (int64_t)m + s <= kSweepRing && kSweepStrideDiv * s <= (int64_t)m &&
                T.sweep_windows[sweep_bucket(m)] >= 2) {
                uint64_t e = w0 + 1;
                while (e + 1 < n_win && single(e + 1) && wm[e + 1] == m && (*wx)[e + 1] - (*wx)[e] == (uint64_t)dx &&
                       (*wy)[e + 1] - (*wy)[e] == (uint64_t)dy)
                    ++e;
                close();
                close_tri();
                uint64_t rest = e + 1 - w0;
                // windows per item: the tuned count, within 255 and a span
                // of kSweepSpan points
                const uint64_t C = std::min<uint64_t>(std::min<uint64_t>(T.sweep_windows[sweep_bucket(m)], 255),
                                                      (uint64_t)(kSweepSpan - (int64_t)m) / (uint64_t)s + 1);
                while (rest > 0) {
                    // never leave one window alone: C + 1 windows split in
                    // two halves (three go together)
                    const uint64_t c = rest <= C ? rest : (rest == C + 1 ? (rest >= 4 ? rest / 2 : rest) : C);
                    out.items.push_back(Item{w, kItemSweep | (uint32_t)c});
                    out.cost.push_back((uint64_t)m * m + c * (uint64_t)m * (uint64_t)(16 + 2 * s));
                    w += (uint32_t)c;
                    rest -= c;
                }
                t = wquery[w - 1];  // the loop moves on to the query after the run
                continue;
            }
        }
        if (!plain && fuse_triples && nw == 3 && wm[w0 + 2] <= (uint32_t)kLocalSlots) {
            close();  // a local item holds consecutive windows only
            const uint32_t mu = wm[w0 + 2];
            if (!fits_tri(tri, mu))
                close_tri();
            if (tri.n == 0)
                tri.start = w0;
            tri.n++;
            tri.slots += (mu + 1u) & ~1u;
            tri.maxm = std::max(tri.maxm, mu);
            tri.cost += (uint64_t)mu * mu + 4096u;
            w += 3;
            continue;
        }
        close_tri();
        if (!plain && nw > 1) {
            // start a fresh item rather than cut a query that fits in one
            bool all_local = true, whole = true;
            Cur sim;
            for (uint32_t r = 0; r < nw; ++r) {
                all_local = all_local && wm[w0 + r] <= (uint32_t)kLocalSlots;
                if (fits(sim, wm[w0 + r]))
                    add(sim, w0 + r, wm[w0 + r]);
                else
                    whole = false;
            }
            if (all_local && whole) {
                Cur c2 = cur;
                bool ok = true;
                for (uint32_t r = 0; r < nw && ok; ++r) {
                    ok = fits(c2, wm[w0 + r]);
                    if (ok)
                        add(c2, w0 + r, wm[w0 + r]);
                }
                if (!ok)
                    close();
            }
        }
        for (uint32_t r = 0; r < nw; ++r, ++w) {
            const uint32_t m = wm[w];
            if (plain)
                out.first_item.push_back((uint32_t)out.items.size());
            if (m > (uint32_t)kLocalSlots) {
                close();
                const uint32_t ni = (m + kSplitPoints - 1) / kSplitPoints;
                out.wnitems[w] = ni;
                out.wsorted[w] = (uint32_t)out.split_pts;
                out.split_pts += m;
                if (plain)
                    out.wprep[w] = (int32_t)out.prep_list.size();
                out.prep_list.push_back(w);
                for (uint32_t it = 0; it < ni; ++it) {
                    out.items.push_back(Item{w, it * (uint32_t)kSplitPoints});
                    out.cost.push_back((uint64_t)std::min<uint32_t>(kSplitPoints, m - it * kSplitPoints) * m);
                }
            } else {
                if (plain || !fits(cur, m))
                    close();
                add(cur, w, m);
                if (plain)
                    close();
            }
        }
    }
    close();
    close_tri();
    if (plain)
        out.first_item.push_back((uint32_t)out.items.size());
}

// Batched form: the queue the persistent kernel takes items from.  Prep
// items (one per split window, largest first) come first, then the local
// items, then the split items, then the local items cheaper than kTailCost,
// each class largest cost first (a stable bucket order by log2(cost) is
// enough for the greedy schedule).  A split item scans its window in x order,
// which its prep item writes: the local items in between keep the device busy
// while those sorts finish, and the cheap ones at the end shorten the tail
// that the last, long split items would leave.  kTailCost (in the cost units
// of plan_items: m^2 + 4096 per window) puts the items of windows up to 128
// points there.
constexpr uint64_t kTailCost = 100000;

inline void plan_queue(const Plan &P, const std::vector<uint32_t> &wm, std::vector<Item> &queue)
{
    queue.clear();
    queue.reserve(P.items.size() + P.prep_list.size());
    std::vector<uint32_t> prep(P.prep_list);
    std::stable_sort(prep.begin(), prep.end(), [&](uint32_t a, uint32_t b) { return wm[a] > wm[b]; });
    for (uint32_t w : prep)
        queue.push_back(Item{w, kItemPrep});
    auto bucket = [](uint64_t c) { return 63 - (63 - __builtin_clzll(c | 1ull)); };
    // phase 0: local items; 1: split items; 2: the cheapest local items,
    // which end the queue and fill the device while the last split items run
    for (int phase = 0; phase < 3; ++phase) {
        std::vector<uint32_t> cnt(66, 0);
        std::vector<size_t> idx;
        for (size_t i = 0; i < P.items.size(); ++i) {
            const bool local = (P.items[i].info & (kItemLocal | kItemTriple | kItemSweep)) != 0;
            const int ph = local ? (P.cost[i] < kTailCost ? 2 : 0) : 1;
            if (ph == phase) {
                cnt[bucket(P.cost[i]) + 1]++;
                idx.push_back(i);
            }
        }
        for (int i = 1; i <= 65; ++i)
            cnt[i] += cnt[i - 1];
        const size_t base = queue.size();
        queue.resize(base + idx.size());
        for (size_t i : idx)
            queue[base + cnt[bucket(P.cost[i])]++] = P.items[i];
    }
}

// Serving: local windows per item for a run of windows of m points (the
// local-item limits above, every window of the run the same size).
inline uint32_t plan_local_per_item(uint32_t m, const Tuning *tune = nullptr)
{
    const Tuning T = tune ? *tune : default_tuning();
    const uint32_t even = (m + 1u) & ~1u;
    const uint32_t cap = std::min<uint32_t>(std::max(T.local_windows[local_bucket(std::max(m, 2u))], 1u), kLocalWindows);
    const uint32_t n = std::min<uint32_t>(cap, (uint32_t)kLocalSlots / even);
    return std::max(1u, std::min(n, (uint32_t)kLocalSort / plan_pow2(std::max(m, 2u))));
}

// Serving: queue layout of a launch made of parts (m and count set, in launch
// window order).  Sets win0, and per part its prep items, sorted-data offset
// and items: all prep items first, then local items, then split items,
// larger windows first within each.  Returns the queue length; *split
// receives the sorted-marginal points (sum of m over split windows).
inline uint32_t plan_parts(PartDesc *pd, uint32_t n, uint64_t *split, const Tuning *tune = nullptr)
{
    std::vector<uint32_t> order(n);
    uint32_t win0 = 0;
    for (uint32_t i = 0; i < n; ++i) {
        order[i] = i;
        pd[i].win0 = win0;
        win0 += pd[i].count;
        pd[i].prep0 = pd[i].sorted0 = pd[i].item0 = 0;
        pd[i].per_item = 1;
    }
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return pd[a].m > pd[b].m; });
    uint32_t q = 0;
    uint64_t sorted = 0;
    for (uint32_t i : order)
        if (pd[i].m > (uint32_t)kLocalSlots) {
            pd[i].prep0 = q;
            pd[i].sorted0 = (uint32_t)sorted;
            q += pd[i].count;
            sorted += (uint64_t)pd[i].count * pd[i].m;
        }
    for (uint32_t i : order)
        if (pd[i].m <= (uint32_t)kLocalSlots) {
            pd[i].item0 = q;
            pd[i].per_item = plan_local_per_item(pd[i].m, tune);
            q += (pd[i].count + pd[i].per_item - 1) / pd[i].per_item;
        }
    for (uint32_t i : order)
        if (pd[i].m > (uint32_t)kLocalSlots) {
            pd[i].item0 = q;
            q += pd[i].count * ((pd[i].m + kSplitPoints - 1) / kSplitPoints);
        }
    *split = sorted;
    return q;
}

// Runs of equally spaced queries (wmi_submit_ranges): the kind, the windows
// or triples per item and the queue offsets of each run, for the device-side
// expansion (expand_query in wmi_ranges.h).  rd[0..n) come with x, y, start,
// stride, count (> 0), m, e, side and tau_eff set.  The queue has the layout
// of plan_queue: prep items (larger windows first), local items (triple and
// sweep items included) costing at least kTailCost, split items (larger
// windows first), then the cheaper local items; runs keep their items
// together.  fuse allows triple and sweep items (off: every window evaluated
// on its own).  Returns the queue length; *n_win and *split_pts receive the
// window count and the points of split windows.
inline uint64_t plan_ranges(RangeDesc *rd, uint32_t n, bool fuse, const Tuning *tune, uint64_t *n_win,
                            uint64_t *split_pts)
{
    const Tuning T = tune ? *tune : default_tuning();
    std::vector<uint64_t> cost(n, 0), nloc(n, 0), nsplit(n, 0), nprep(n, 0), msplit(n, 0);
    uint64_t q = 0, w = 0, sp = 0;
    for (uint32_t r = 0; r < n; ++r) {
        RangeDesc &R = rd[r];
        R.q0 = (uint32_t)q;
        R.win0 = (uint32_t)w;
        R.item0 = R.item1 = R.prep0 = R.sorted0 = 0u;
        R.per_item = 1u;
        R.pad = 0u;
        q += R.count;
        w += (uint64_t)R.count * (R.side ? 3u : 1u);
        const uint64_t cnt = R.count;
        if (R.side == 0) {
            const uint32_t m = R.m, st = R.stride;
            if (m > (uint32_t)kLocalSlots) {
                R.kind = kRangeSplit;
                const uint64_t ns = (m + kSplitPoints - 1) / kSplitPoints;
                nprep[r] = cnt;
                nsplit[r] = cnt * ns;
                msplit[r] = m;
                R.sorted0 = (uint32_t)sp;
                sp += cnt * m;
            } else if (fuse && cnt >= 2 && st >= 1 && m >= (uint32_t)kSweepMinM && m + st <= (uint32_t)kSweepRing &&
                       (uint64_t)kSweepStrideDiv * st <= m && T.sweep_windows[sweep_bucket(m)] >= 2) {
                R.kind = kRangeSweep;
                const uint32_t C = std::min<uint32_t>(std::min<uint32_t>(T.sweep_windows[sweep_bucket(m)], 255u),
                                                      ((uint32_t)kSweepSpan - m) / st + 1u);
                R.per_item = C;
                nloc[r] = sweep_items(R.count, C);
                cost[r] = (uint64_t)m * m + (uint64_t)C * m * (16u + 2u * st);
            } else {
                R.kind = kRangeLocal;
                R.per_item = plan_local_per_item(m, &T);
                nloc[r] = (cnt + R.per_item - 1) / R.per_item;
                cost[r] = (uint64_t)R.per_item * ((uint64_t)m * m + 4096u);
            }
        } else {
            const uint32_t u = R.m + R.e;
            if (fuse && u <= (uint32_t)kLocalSlots) {
                R.kind = kRangeTriple;
                const uint32_t um = std::max(u, 2u);
                uint32_t per = std::min<uint32_t>(std::max(T.triples[local_bucket(um)], 1u), kTripleMax);
                per = std::min(per, (uint32_t)kLocalSlots / ((u + 1u) & ~1u));
                per = std::max(1u, std::min(per, (uint32_t)kLocalSort / plan_pow2(um)));
                R.per_item = per;
                nloc[r] = (cnt + per - 1) / per;
                cost[r] = (uint64_t)per * ((uint64_t)u * u + 4096u);
            } else {
                R.kind = kRangeTripleWide;
                const uint32_t m3[3] = {R.m, R.e, u};
                uint64_t L = 0, P = 0, SP = 0, S = 0, mx = 0;
                for (uint32_t m : m3) {
                    if (m > (uint32_t)kLocalSlots) {
                        P++;
                        SP += m;
                        S += (m + kSplitPoints - 1) / kSplitPoints;
                        mx = std::max<uint64_t>(mx, m);
                    } else {
                        L++;
                    }
                }
                nloc[r] = cnt * L;
                nprep[r] = cnt * P;
                nsplit[r] = cnt * S;
                msplit[r] = mx;
                R.sorted0 = (uint32_t)sp;
                sp += cnt * SP;
                cost[r] = ~0ull;  // its single-window local items go with the costly ones
            }
        }
    }
    *n_win = w;
    *split_pts = sp;
    auto by = [&](std::vector<uint64_t> key, auto pick) {
        std::vector<uint32_t> idx;
        for (uint32_t r = 0; r < n; ++r)
            if (pick(r))
                idx.push_back(r);
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return key[a] > key[b]; });
        return idx;
    };
    uint64_t at = 0;
    for (uint32_t r : by(msplit, [&](uint32_t r) { return nprep[r] > 0; })) {
        rd[r].prep0 = (uint32_t)at;
        at += nprep[r];
    }
    for (uint32_t r : by(cost, [&](uint32_t r) { return nloc[r] > 0 && cost[r] >= kTailCost; })) {
        rd[r].item0 = (uint32_t)at;
        at += nloc[r];
    }
    for (uint32_t r : by(msplit, [&](uint32_t r) { return nsplit[r] > 0; })) {
        (rd[r].kind == kRangeTripleWide ? rd[r].item1 : rd[r].item0) = (uint32_t)at;
        at += nsplit[r];
    }
    for (uint32_t r : by(cost, [&](uint32_t r) { return nloc[r] > 0 && cost[r] < kTailCost; })) {
        rd[r].item0 = (uint32_t)at;
        at += nloc[r];
    }
    return at;
}

}  // namespace wmi
