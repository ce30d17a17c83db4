// Host-side check of the work lists (csrc/wmi_plan.h): the batch plan on
// random query mixes (every window covered exactly once, every item within
// the limits the main kernel's LDS layout assumes) and the queue layout of
// serving launches.  Prints OK or the first violation.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "wmi_plan.h"

using namespace wmi;

static int fail(const char *what, long a, long b)
{
    std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
    return 1;
}

// One queue item against the limits of the main kernel's LDS layout; marks
// the windows it covers (local_item) or the split block it scans (split_q0).
static int check_item(size_t it, const Item &I, const std::vector<uint32_t> &wm, const std::vector<uint32_t> &wq,
                      const std::vector<uint64_t> &wx, const std::vector<uint64_t> &wy, const Tuning &T, bool plain,
                      bool fuse, std::vector<int> &local_item, std::vector<std::vector<uint32_t>> &split_q0)
{
    const size_t n = wm.size();
    auto single = [&](size_t v) {
        return (v == 0 || wq[v - 1] != wq[v]) && (v + 1 >= n || wq[v + 1] != wq[v]);
    };
    if (I.info & kItemSweep) {
        // equally spaced one-window queries of one m, within the ring
        const uint32_t nw = I.info & 0xFFu;
        if (plain || !fuse)
            return fail("sweep item without reuse", (long)it, (long)nw);
        if (nw < 2 || (I.info & 0x0FFFFF00u) || I.win + nw > n || T.sweep_windows[sweep_bucket(wm[I.win])] < 2 ||
            nw > std::max<uint32_t>(T.sweep_windows[sweep_bucket(wm[I.win])], 3u))
            return fail("sweep window count", (long)it, (long)nw);
        const uint32_t m = wm[I.win];
        const int64_t dx = (int64_t)(wx[I.win + 1] - wx[I.win]), dy = (int64_t)(wy[I.win + 1] - wy[I.win]);
        const int64_t s = dx / 4;
        if (dx != dy || dx <= 0 || dx % 4 || m < (uint32_t)kSweepMinM || (int64_t)m + s > kSweepRing ||
            kSweepStrideDiv * s > (int64_t)m || (int64_t)(nw - 1) * s + m > kSweepSpan)
            return fail("sweep shape", (long)it, (long)s);
        for (uint32_t r = 0; r < nw; ++r) {
            const uint32_t v = I.win + r;
            if (!single(v) || wm[v] != m)
                return fail("sweep window", (long)it, (long)v);
            if (r && (wx[v] - wx[v - 1] != (uint64_t)dx || wy[v] - wy[v - 1] != (uint64_t)dy))
                return fail("sweep stride", (long)it, (long)v);
            if (local_item[v] >= 0)
                return fail("window in two items", (long)v, (long)it);
            local_item[v] = (int)it;
        }
    } else if (I.info & kItemTriple) {
        // whole noise triples (base, extension, union of one query), the
        // union within the limits of the kernel's LDS layout
        const uint32_t nt = I.info & 0xFFu;
        uint32_t slots = 0, maxm = 2;
        if (plain || !fuse)
            return fail("triple item without fusing", (long)it, (long)nt);
        if (nt < 1 || nt > (uint32_t)kTripleMax || (I.info & 0x1FFFFF00u))
            return fail("triple count", (long)it, (long)nt);
        uint32_t umax = 2;
        for (uint32_t r = 0; r < nt && I.win + 3 * r + 2 < n; ++r)
            umax = std::max(umax, wm[I.win + 3 * r + 2]);
        if (nt > T.triples[local_bucket(umax)])
            return fail("triples above the tuned cap", (long)it, (long)nt);
        for (uint32_t r = 0; r < nt; ++r) {
            const uint32_t wb = I.win + 3 * r;
            if (wb + 2 >= n)
                return fail("triple window out of range", (long)it, (long)wb);
            const uint32_t q = wq[wb];
            if (wq[wb + 1] != q || wq[wb + 2] != q || (wb > 0 && wq[wb - 1] == q) ||
                (wb + 3 < n && wq[wb + 3] == q))
                return fail("triple item window not a whole triple", (long)it, (long)wb);
            if (wm[wb + 2] != wm[wb] + wm[wb + 1] || wm[wb + 2] > (uint32_t)kLocalSlots)
                return fail("triple union", (long)wb, (long)wm[wb + 2]);
            for (uint32_t e = 0; e < 3; ++e) {
                if (local_item[wb + e] >= 0)
                    return fail("window in two items", (long)(wb + e), (long)it);
                local_item[wb + e] = (int)it;
            }
            slots += (wm[wb + 2] + 1u) & ~1u;
            maxm = std::max(maxm, wm[wb + 2]);
        }
        if (slots > (uint32_t)kLocalSlots)
            return fail("triple slots", (long)it, (long)slots);
        if (nt * plan_pow2(maxm) > (uint32_t)kLocalSort)
            return fail("triple sort entries", (long)it, (long)(nt * plan_pow2(maxm)));
    } else if (I.info & kItemLocal) {
        uint32_t nw = I.info & 0xFFu, slots = 0, maxm = 2;
        if (nw < 1 || nw > (uint32_t)kLocalWindows || (I.info & 0x7FFFFF00u))
            return fail("local window count", (long)it, (long)nw);
        if (plain && nw != 1)
            return fail("plain local item with several windows", (long)it, (long)nw);
        for (uint32_t r = 0; r < nw; ++r) {
            uint32_t w = I.win + r;
            if (w >= n)
                return fail("local window out of range", (long)it, (long)w);
            if (wm[w] > (uint32_t)kLocalSlots)
                return fail("large window in a local item", (long)w, (long)wm[w]);
            if (local_item[w] >= 0)
                return fail("window in two local items", (long)w, (long)it);
            local_item[w] = (int)it;
            slots += (wm[w] + 1u) & ~1u;
            maxm = std::max(maxm, wm[w]);
        }
        if (slots > (uint32_t)kLocalSlots)
            return fail("local slots", (long)it, (long)slots);
        if (!plain && nw > T.local_windows[local_bucket(maxm)])
            return fail("local windows above the tuned cap", (long)it, (long)nw);
        if (nw * plan_pow2(maxm) > (uint32_t)kLocalSort)
            return fail("local sort entries", (long)it, (long)(nw * plan_pow2(maxm)));
    } else {
        if (I.win >= n || wm[I.win] <= (uint32_t)kLocalSlots)
            return fail("split item of a small window", (long)it, (long)I.win);
        if (I.info % kSplitPoints || I.info >= wm[I.win])
            return fail("split first point", (long)it, (long)I.info);
        split_q0[I.win].push_back(I.info);
    }
    return 0;
}

static int check(const std::vector<uint32_t> &wm, const std::vector<uint32_t> &wq, uint64_t count, bool plain,
                 bool fuse, const std::vector<uint64_t> &wx, const std::vector<uint64_t> &wy, const Tuning &T)
{
    Plan P;
    plan_items(wm, wq, count, plain, P, fuse, &wx, &wy, &T);
    const size_t n = wm.size();
    if (P.items.size() != P.cost.size())
        return fail("cost size", (long)P.items.size(), (long)P.cost.size());
    std::vector<int> local_item(n, -1);
    std::vector<std::vector<uint32_t>> split_q0(n);
    for (size_t it = 0; it < P.items.size(); ++it)
        if (int rc = check_item(it, P.items[it], wm, wq, wx, wy, T, plain, fuse, local_item, split_q0))
            return rc;
    uint64_t pts = 0;
    size_t pi = 0;
    for (size_t w = 0; w < n; ++w) {
        if (wm[w] > (uint32_t)kLocalSlots) {
            uint32_t ni = (wm[w] + kSplitPoints - 1) / kSplitPoints;
            if (split_q0[w].size() != ni || P.wnitems[w] != ni)
                return fail("split coverage", (long)w, (long)split_q0[w].size());
            std::vector<bool> seen(ni, false);
            for (uint32_t q0 : split_q0[w]) {
                if (seen[q0 / kSplitPoints])
                    return fail("split block twice", (long)w, (long)q0);
                seen[q0 / kSplitPoints] = true;
            }
            if (pi >= P.prep_list.size() || P.prep_list[pi] != w)
                return fail("prep list", (long)w, (long)pi);
            if (P.wsorted[w] != pts)
                return fail("sorted offset", (long)w, (long)P.wsorted[w]);
            if (plain && P.wprep[w] != (int32_t)pi)
                return fail("plain prep index", (long)w, (long)P.wprep[w]);
            pts += wm[w];
            ++pi;
        } else if (local_item[w] < 0) {
            return fail("window not covered", (long)w, (long)wm[w]);
        }
    }
    if (pi != P.prep_list.size() || pts != P.split_pts)
        return fail("prep totals", (long)pi, (long)pts);
    if (!plain) {
        // the queue: every item once, one prep item per split window, and
        // every prep item ahead of every split item (the split items' wait
        // for their window's sorted marginals relies on this order)
        std::vector<Item> queue;
        plan_queue(P, wm, queue);
        if (queue.size() != P.items.size() + P.prep_list.size())
            return fail("queue size", (long)queue.size(), (long)P.items.size());
        size_t first_other = queue.size(), last_prep = 0, nprep = 0;
        std::vector<int> prep_seen(n, 0);
        for (size_t i = 0; i < queue.size(); ++i) {
            if (queue[i].info == kItemPrep) {
                if (queue[i].win >= n || wm[queue[i].win] <= (uint32_t)kLocalSlots)
                    return fail("prep item of a small window", (long)i, (long)queue[i].win);
                prep_seen[queue[i].win]++;
                last_prep = i;
                ++nprep;
            } else if (first_other == queue.size()) {
                first_other = i;
            }
        }
        if (nprep && last_prep > first_other)
            return fail("prep item after another item", (long)last_prep, (long)first_other);
        for (size_t w = 0; w < n; ++w)
            if ((wm[w] > (uint32_t)kLocalSlots) != (prep_seen[w] == 1))
                return fail("prep items per window", (long)w, (long)prep_seen[w]);
        std::vector<uint64_t> a, b;
        for (const Item &I : P.items)
            a.push_back(((uint64_t)I.win << 32) | I.info);
        for (size_t i = nprep; i < queue.size(); ++i)
            b.push_back(((uint64_t)queue[i].win << 32) | queue[i].info);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a != b)
            return fail("queue is not a permutation of the items", (long)a.size(), (long)b.size());
        // a query whose windows are all local and fit one item is not cut
        size_t w = 0;
        for (uint64_t t = 0; t < count; ++t) {
            size_t w0 = w;
            while (w < n && wq[w] == t)
                ++w;
            // it fits when its windows, added one by one to an empty item,
            // stay within every limit (the cap on windows depends on the
            // item's largest window so far)
            uint32_t slots = 0, maxm = 2, nw = 0;
            bool fits = true;
            for (size_t r = w0; r < w && fits; ++r) {
                fits = wm[r] <= (uint32_t)kLocalSlots;
                slots += (wm[r] + 1u) & ~1u;
                maxm = std::max(maxm, wm[r]);
                ++nw;
                fits = fits && nw <= std::min<uint32_t>(T.local_windows[local_bucket(maxm)], kLocalWindows) &&
                       slots <= (uint32_t)kLocalSlots && nw * plan_pow2(maxm) <= (uint32_t)kLocalSort;
            }
            if (fits)
                for (size_t r = w0 + 1; r < w; ++r)
                    if (local_item[r] != local_item[w0])
                        return fail("query cut across items", (long)t, (long)r);
        }
    } else {
        if (P.first_item.size() != n + 1)
            return fail("plain first_item size", (long)P.first_item.size(), (long)n);
        for (size_t w = 0; w < n; ++w)
            for (uint32_t it = P.first_item[w]; it < P.first_item[w + 1]; ++it)
                if (P.items[it].win != w)
                    return fail("plain items of another window", (long)w, (long)it);
    }
    return 0;
}

// Serving launches: expand the parts as the expand kernel does (one window
// descriptor per window, prep / split / local items at the offsets the plan
// gives) and check every queue entry is written once, every window covered,
// sorted-marginal ranges disjoint and inside the total, and local items
// within the kernel's limits.
static int check_parts(std::vector<PartDesc> pd)
{
    uint64_t split = 0;
    const uint32_t n_items = plan_parts(pd.data(), (uint32_t)pd.size(), &split);
    uint64_t n_win = 0;
    for (const PartDesc &p : pd) {
        if (p.win0 != n_win)
            return fail("part win0", (long)p.win0, (long)n_win);
        n_win += p.count;
    }
    std::vector<int> queue(n_items, 0);  // 1 prep, 2 split, 3 local
    std::vector<int> covered(n_win, 0), prepped(n_win, 0);
    std::vector<char> sorted_used(split, 0);
    uint32_t last_prep = 0, first_split = n_items, last_local = 0;
    bool any_prep = false, any_local = false;
    for (const PartDesc &p : pd) {
        const bool big = p.m > (uint32_t)kLocalSlots;
        const uint32_t nsplit = (p.m + kSplitPoints - 1) / kSplitPoints;
        for (uint32_t i = 0; i < p.count; ++i) {
            const uint32_t w = p.win0 + i;
            if (big) {
                const uint64_t off = (uint64_t)p.sorted0 + (uint64_t)i * p.m;
                if (off + p.m > split)
                    return fail("sorted range beyond total", (long)off, (long)split);
                for (uint32_t j = 0; j < p.m; ++j)
                    if (sorted_used[off + j]++)
                        return fail("sorted ranges overlap", (long)w, (long)(off + j));
                const uint32_t qp = p.prep0 + i;
                if (qp >= n_items || queue[qp]++)
                    return fail("prep entry", (long)qp, (long)n_items);
                prepped[w]++;
                last_prep = std::max(last_prep, qp);
                any_prep = true;
                for (uint32_t t = 0; t < nsplit; ++t) {
                    const uint32_t qs = p.item0 + i * nsplit + t;
                    if (qs >= n_items || queue[qs]++)
                        return fail("split entry", (long)qs, (long)n_items);
                    first_split = std::min(first_split, qs);
                }
                covered[w]++;
            } else if (i % p.per_item == 0) {
                const uint32_t nw = std::min(p.per_item, p.count - i);
                const uint32_t ql = p.item0 + i / p.per_item;
                if (ql >= n_items || queue[ql]++)
                    return fail("local entry", (long)ql, (long)n_items);
                last_local = std::max(last_local, ql);
                any_local = true;
                if (nw > (uint32_t)kLocalWindows || nw * ((p.m + 1u) & ~1u) > (uint32_t)kLocalSlots ||
                    nw * plan_pow2(std::max(p.m, 2u)) > (uint32_t)kLocalSort)
                    return fail("local item limits", (long)p.m, (long)nw);
                for (uint32_t r = 0; r < nw; ++r)
                    covered[w + r]++;
            }
        }
    }
    for (uint32_t q = 0; q < n_items; ++q)
        if (queue[q] != 1)
            return fail("queue entry not written once", (long)q, (long)queue[q]);
    for (uint64_t w = 0; w < n_win; ++w)
        if (covered[w] != 1)
            return fail("window not covered once", (long)w, (long)covered[w]);
    for (size_t j = 0; j < split; ++j)
        if (sorted_used[j] != 1)
            return fail("sorted point unused", (long)j, 0);
    if ((any_prep && last_prep >= first_split) || (any_local && last_local >= first_split))
        return fail("queue order: prep and local items before split items", (long)last_prep, (long)first_split);
    if (any_prep && any_local) {
        // every prep item precedes every local item
        for (const PartDesc &p : pd)
            if (p.m <= (uint32_t)kLocalSlots && p.count && p.item0 <= last_prep)
                return fail("local item before a prep item", (long)p.item0, (long)last_prep);
    }
    return 0;
}

// Runs of queries: plan them (plan_ranges), expand every query with the code
// the device runs (expand_query), and check the result against the query
// list the runs stand for: descriptors, every queue entry written, every
// item within the kernel's limits, every window covered once, one prep item
// per split window ahead of every split item, disjoint sorted ranges.
static int check_ranges(std::vector<RangeDesc> rd, bool fuse, const Tuning &T)
{
    uint64_t n_win = 0, split = 0;
    const uint64_t n_items = plan_ranges(rd.data(), (uint32_t)rd.size(), fuse, &T, &n_win, &split);
    uint64_t nq = 0;
    for (const RangeDesc &R : rd)
        nq += R.count;
    std::vector<WinDesc> win(n_win);
    std::vector<QDesc> qd(nq);
    std::vector<Item> queue(n_items, Item{0xFFFFFFFFu, 0xFFFFFFFFu});
    for (const RangeDesc &R : rd)
        for (uint32_t i = 0; i < R.count; ++i)
            expand_query(R, i, win.data(), qd.data(), queue.data());
    // the query list the runs stand for, window by window
    std::vector<uint32_t> wm, wq;
    std::vector<uint64_t> wx, wy;
    uint64_t t = 0;
    for (const RangeDesc &R : rd)
        for (uint32_t i = 0; i < R.count; ++i, ++t) {
            const uint64_t s = R.start + (uint64_t)i * R.stride;
            const uint64_t st[3] = {s, R.side > 0 ? s + R.m : s - R.e, R.side > 0 ? s : s - R.e};
            const uint32_t m[3] = {R.m, R.e, R.m + R.e};
            if (qd[t].nwin != (R.side ? 3u : 1u) || qd[t].win0 != wm.size() || qd[t].tau_eff != R.tau_eff)
                return fail("query descriptor", (long)t, (long)qd[t].win0);
            for (uint32_t r = 0; r < (R.side ? 3u : 1u); ++r) {
                const WinDesc &d = win[wm.size()];
                if (d.x != R.x + st[r] || d.y != R.y + st[r] || d.m != m[r] || d.query != t)
                    return fail("window descriptor", (long)t, (long)r);
                wm.push_back(m[r]);
                wq.push_back((uint32_t)t);
                wx.push_back((uint64_t)(uintptr_t)(R.x + st[r]));
                wy.push_back((uint64_t)(uintptr_t)(R.y + st[r]));
            }
        }
    const size_t n = wm.size();
    std::vector<int> local_item(n, -1), prep_seen(n, 0);
    std::vector<std::vector<uint32_t>> split_q0(n);
    size_t last_prep = 0, first_split = queue.size();
    bool any_prep = false;
    for (size_t it = 0; it < queue.size(); ++it) {
        const Item &I = queue[it];
        if (I.win == 0xFFFFFFFFu)
            return fail("queue entry not written", (long)it, 0);
        if (I.info == kItemPrep) {
            if (I.win >= n || wm[I.win] <= (uint32_t)kLocalSlots)
                return fail("prep item of a small window", (long)it, (long)I.win);
            prep_seen[I.win]++;
            last_prep = it;
            any_prep = true;
            continue;
        }
        if (!(I.info & (kItemLocal | kItemTriple | kItemSweep)))
            first_split = std::min(first_split, it);
        if (int rc = check_item(it, I, wm, wq, wx, wy, T, false, fuse, local_item, split_q0))
            return rc;
    }
    if (any_prep && first_split < queue.size() && last_prep > first_split)
        return fail("prep item after a split item", (long)last_prep, (long)first_split);
    std::vector<char> used(split, 0);
    for (size_t w = 0; w < n; ++w) {
        if (wm[w] > (uint32_t)kLocalSlots) {
            const uint32_t ni = (wm[w] + kSplitPoints - 1) / kSplitPoints;
            if (prep_seen[w] != 1 || split_q0[w].size() != ni || win[w].n_items != ni)
                return fail("split window coverage", (long)w, (long)split_q0[w].size());
            std::vector<bool> seen(ni, false);
            for (uint32_t q0 : split_q0[w]) {
                if (seen[q0 / kSplitPoints])
                    return fail("split block twice", (long)w, (long)q0);
                seen[q0 / kSplitPoints] = true;
            }
            const uint64_t off = win[w].sorted_off;
            if (off + wm[w] > split)
                return fail("sorted range beyond total", (long)w, (long)off);
            for (uint32_t j = 0; j < wm[w]; ++j)
                if (used[off + j]++)
                    return fail("sorted ranges overlap", (long)w, (long)(off + j));
        } else if (local_item[w] < 0 || prep_seen[w]) {
            return fail("window not covered", (long)w, (long)wm[w]);
        }
    }
    for (size_t j = 0; j < split; ++j)
        if (!used[j])
            return fail("sorted point unused", (long)j, 0);
    return 0;
}

int main(int argc, char **argv)
{
    int cases = argc > 1 ? std::atoi(argv[1]) : 300;
    std::mt19937_64 rng(12345);
    for (int c = 0; c < cases; ++c) {
        std::vector<uint32_t> wm, wq;
        std::vector<uint64_t> wx, wy;
        uint64_t count = 1 + rng() % 400;
        int style = (int)(rng() % 5);
        for (uint64_t t = 0; t < count; ++t) {
            auto draw = [&]() -> uint32_t {
                switch (style) {
                case 0: return (uint32_t)(1 + rng() % 4096);
                case 1: return (uint32_t)(1u << (5 + rng() % 8));   // 32..4096
                case 2: return (uint32_t)(1 + rng() % 600);
                default: return (uint32_t)(1 + rng() % 64);
                }
            };
            if (style == 4 && rng() % 2 == 0) {  // a run of equally spaced windows
                const uint32_t m = (uint32_t)(kSweepMinM - 2 + rng() % 480), s = 1 + (uint32_t)(rng() % (m / 12 + 1));
                const uint64_t L = 1 + rng() % 30, bx = (rng() % 1000000) * 4, by = (rng() % 1000000) * 4;
                for (uint64_t i = 0; i < L && t < count; ++i, ++t) {
                    wm.push_back(m);
                    wq.push_back((uint32_t)t);
                    wx.push_back(bx + 4 * i * s);
                    wy.push_back(by + 4 * i * s);
                }
                --t;
            } else if (rng() % 3 == 0) {  // a noise triple: base, extension, union
                uint32_t base = draw(), ext = 1 + (uint32_t)(rng() % 300);
                if (base + ext > 4096)
                    base = 4096 - ext;
                wm.push_back(base);
                wm.push_back(ext);
                wm.push_back(base + ext);
                for (int r = 0; r < 3; ++r) {
                    wq.push_back((uint32_t)t);
                    wx.push_back(rng() & ~3ull);
                    wy.push_back(rng() & ~3ull);
                }
            } else {
                wm.push_back(draw());
                wq.push_back((uint32_t)t);
                wx.push_back(rng() & ~3ull);
                wy.push_back(rng() & ~3ull);
            }
        }
        Tuning T = default_tuning();
        if (c % 2) {  // other work-list choices
            for (int b = 0; b < 5; ++b) {
                T.local_windows[b] = 1 + (uint32_t)(rng() % kLocalWindows);
                T.triples[b] = 1 + (uint32_t)(rng() % kTripleMax);
            }
            for (int b = 0; b < 3; ++b)
                T.sweep_windows[b] = 1 + (uint32_t)(rng() % 40);
        }
        for (int plain = 0; plain < 2; ++plain)
            for (int fuse = 0; fuse < 2; ++fuse)
                if (check(wm, wq, count, plain != 0, fuse != 0, wx, wy, T)) {
                    std::printf("case %d style %d plain %d fuse %d\n", c, style, plain, fuse);
                    return 1;
                }
    }
    for (int c = 0; c < cases; ++c) {
        std::vector<PartDesc> pd(1 + rng() % 40);
        for (PartDesc &p : pd) {
            p = PartDesc{};
            p.m = (rng() % 3 == 0) ? 1u << (5 + rng() % 8) : (uint32_t)(1 + rng() % 4096);
            p.count = (uint32_t)(1 + rng() % 300);
        }
        if (check_parts(pd)) {
            std::printf("parts case %d\n", c);
            return 1;
        }
    }
    for (int c = 0; c < cases; ++c) {
        std::vector<RangeDesc> rd(1 + rng() % 12);
        static float X[1], Y[1];  // only addresses are formed, never read
        for (RangeDesc &R : rd) {
            R = RangeDesc{};
            R.x = X;
            R.y = Y;
            R.count = (uint32_t)(1 + rng() % (rng() % 4 == 0 ? 2000 : 40));
            R.tau_eff = (double)(rng() % 100) / 100.0;
            switch (rng() % 4) {
            case 0:  // plain windows of any size
                R.m = (uint32_t)(1 + rng() % 4096);
                R.stride = (uint32_t)(1 + rng() % 600);
                break;
            case 1:  // sweeps: small strides
                R.m = (uint32_t)(kSweepMinM + rng() % 240);
                R.stride = (uint32_t)(1 + rng() % (R.m / 16 + 1));
                break;
            default: {  // triples, small and large
                R.e = (uint32_t)(1 + rng() % (rng() % 2 ? 64 : 1500));
                R.m = (uint32_t)(1 + rng() % (rng() % 2 ? 400 : 4096 - R.e));
                R.side = rng() % 2 ? 1 : -1;
                R.stride = (uint32_t)(1 + rng() % 64);
                R.start = R.e;
                break;
            }
            }
        }
        Tuning T = default_tuning();
        if (c % 2) {
            for (int b = 0; b < 5; ++b) {
                T.local_windows[b] = 1 + (uint32_t)(rng() % kLocalWindows);
                T.triples[b] = 1 + (uint32_t)(rng() % kTripleMax);
            }
            for (int b = 0; b < 3; ++b)
                T.sweep_windows[b] = 1 + (uint32_t)(rng() % 40);
        }
        for (int fuse = 0; fuse < 2; ++fuse)
            if (check_ranges(rd, fuse != 0, T)) {
                std::printf("ranges case %d fuse %d\n", c, fuse);
                return 1;
            }
    }
    std::printf("OK %d\n", cases);
    return 0;
}
