// wmi_search.cpp -- search drivers over the batch path (include/wmi.h).
//
// Top-down search (Algorithm 1, Section 5.1) with noise pruning (Section
// 6.2).  The rule is sequential inside a partition: whether the next window
// is shifted by the step or starts after the current one depends on the
// current window's estimate.  Every window the rule can reach still lies on
// the partition's grid of starts ps, ps + delta, ... whenever delta divides
// the window size (a jump of s_w is a whole number of steps), so a layer is
// evaluated speculatively: all grid windows of all partitions in a few large
// batches (as noise triples when pruning is on), then the rule walks each
// partition on the host over those estimates.  When delta does not divide
// s_w the walk meets windows off the grid; those are evaluated in follow-up
// batches and the walk resumes.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "wmi.h"
#include "wmi_store.h"

using namespace wmi;

namespace {

constexpr uint64_t kChunkQueries = 1ull << 18;
constexpr uint64_t kChunkPoints = 1ull << 26;

// Distances the path computes for a window of m points, or for a noise triple
// (base m, extension e): a triple whose union fits a triple item costs its
// union's only (its parts' lists come from the union's scan).
uint64_t window_pairs(uint64_t m) { return m * (m - 1); }
uint64_t triple_pairs(uint64_t m, uint64_t e)
{
    const uint64_t u = m + e;
    return u <= (uint64_t)kLocalSlots ? window_pairs(u) : window_pairs(m) + window_pairs(e) + window_pairs(u);
}

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

struct Eval {
    double mi = 0.0;   // I(w)
    double h = 0.0;    // H(w) when the batch computed entropies
    bool noise = false;
};

// Evaluate windows of s_w points at the given starts (as noise triples with a
// delta-point right extension when triple is set) in chunked batches.  The
// starts of a partition's grid advance by delta: each such stretch goes to
// the device as one run (wmi_submit_ranges), whose descriptors the device
// writes.
int evaluate(wmi_store *st, uint32_t a, uint32_t b, const std::vector<uint64_t> &starts, uint32_t s_w,
             uint32_t delta, bool triple, const wmi_params &prm, std::vector<Eval> &out, wmi_search_stats &stats)
{
    out.assign(starts.size(), Eval());
    const uint64_t per_q = triple ? 2ull * s_w : s_w;
    const uint64_t chunk = std::max<uint64_t>(1, std::min(kChunkQueries, kChunkPoints / per_q));
    std::vector<wmi_range> q;
    std::vector<wmi_result> r;
    std::vector<double> h;
    const bool ent = (prm.flags & WMI_SUBMIT_ENTROPY) != 0;
    for (uint64_t i0 = 0; i0 < starts.size(); i0 += chunk) {
        const uint64_t n = std::min<uint64_t>(chunk, starts.size() - i0);
        q.clear();
        for (uint64_t i = 0; i < n;) {
            uint64_t j = i + 1;
            while (j < n && starts[i0 + j] == starts[i0 + j - 1] + delta)
                ++j;
            wmi_range x{};
            x.a = a;
            x.b = b;
            x.start = starts[i0 + i];
            x.count = (uint32_t)(j - i);
            x.stride = delta;
            x.len = triple ? s_w - delta : s_w;
            x.ext_len = triple ? delta : 0;
            x.ext_side = triple ? 1 : 0;
            q.push_back(x);
            i = j;
        }
        wmi_batch *bt = nullptr;
        auto t0 = Clock::now();
        if (int rc = wmi_submit_ranges(st, q.data(), q.size(), &prm, nullptr, &bt))
            return rc;
        stats.submit_ms += ms_since(t0);
        t0 = Clock::now();
        r.assign(n, wmi_result());
        int rc = wmi_read(bt, r.data());
        if (rc == WMI_OK && ent) {
            h.assign(3 * n, 0.0);
            rc = wmi_read_entropy(bt, h.data());
        }
        (void)wmi_batch_destroy(bt);
        stats.wait_ms += ms_since(t0);
        if (rc)
            return rc;
        for (uint64_t i = 0; i < n; ++i) {
            out[i0 + i].mi = triple ? r[i].mi_union : r[i].mi_base;
            out[i0 + i].h = ent ? h[3 * i + (triple ? 2 : 0)] : 0.0;
            out[i0 + i].noise = (r[i].flags & WMI_F_NOISE) != 0;
        }
        stats.batches++;
        stats.windows_evaluated += triple ? 3 * n : n;
        stats.ordered_pairs += n * (triple ? triple_pairs(s_w - delta, delta) : window_pairs(s_w));
    }
    return WMI_OK;
}

struct Walk {
    uint64_t ps, pe;     // partition [ps, pe)
    uint64_t w;          // next window start
    uint32_t run = 0;    // consecutive noise detections
    bool shifted = false;
    bool done = false;
    std::vector<std::pair<uint64_t, uint64_t>> corr;  // correlated windows found
};

}  // namespace

extern "C" int wmi_td_search(wmi_store *st, uint32_t a, uint32_t b, uint64_t begin, uint64_t end,
                             const wmi_td_params *p, wmi_window *host_out, uint64_t capacity, uint64_t *n_out,
                             wmi_search_stats *stats_out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!st || !p || !n_out)
        return fail(WMI_EINVAL, "wmi_td_search: null argument");
    *n_out = 0;
    if (p->s_min < 2 || p->s_min > p->s_max || p->s_max > (uint32_t)WMI_MAX_WINDOW || p->flags)
        return fail(WMI_EINVAL, "wmi_td_search: need 2 <= s_min <= s_max <= %d and flags 0", WMI_MAX_WINDOW);
    if (p->k < 1 || p->k > WMI_MAX_K || p->estimator > 1 || p->normalize > 2)
        return fail(WMI_EINVAL, "wmi_td_search: bad k, estimator or normalize");
    uint64_t na = 0, nb = 0;
    if (int rc = wmi_series_length(st, a, &na))
        return rc;
    if (int rc = wmi_series_length(st, b, &nb))
        return rc;
    if (begin > end || end > std::min(na, nb))
        return fail(WMI_EINVAL, "wmi_td_search: range [%llu, %llu) outside the series", (unsigned long long)begin,
                    (unsigned long long)end);
    const uint32_t div = p->step_div ? p->step_div : 8u;
    wmi_params prm{};
    prm.k = p->k;
    prm.estimator = p->estimator;
    prm.tau = p->tau;
    prm.tau_normalize = p->normalize;
    prm.flags = p->normalize == 2 ? WMI_SUBMIT_ENTROPY : 0u;  // sigma * H(w) needs every window's H

    wmi_search_stats stats{};
    std::vector<wmi_window> found;
    std::vector<std::pair<uint64_t, uint64_t>> parts;
    if (end - begin >= p->s_min)
        parts.push_back({begin, end});
    uint32_t layer = 0;
    for (uint32_t s_w = p->s_max; s_w >= p->s_min; s_w /= 2, ++layer) {
        if (parts.empty())
            break;
        stats.layers++;
        const uint32_t delta = std::max(1u, s_w / div);
        const bool triple = p->p > 0 && delta < s_w;
        const double thr = p->normalize == 1 ? p->sigma * std::log((double)s_w) : p->sigma;
        // speculative pass: every grid window of every partition
        std::vector<Walk> walks;
        std::vector<uint64_t> starts;
        std::vector<uint64_t> grid0;  // first grid index of each partition
        for (const auto &pr : parts) {
            Walk wk;
            wk.ps = pr.first;
            wk.pe = pr.second;
            wk.w = pr.first;
            grid0.push_back(starts.size());
            for (uint64_t s = pr.first; s + s_w <= pr.second; s += delta)
                starts.push_back(s);
            walks.push_back(std::move(wk));
        }
        std::vector<Eval> ev;
        if (int rc = evaluate(st, a, b, starts, s_w, delta, triple, prm, ev, stats))
            return rc;
        std::map<uint64_t, Eval> extra;  // off-grid windows evaluated on demand
        bool pending = true;
        while (pending) {
            pending = false;
            std::vector<uint64_t> need;
            for (size_t pi = 0; pi < walks.size(); ++pi) {
                Walk &wk = walks[pi];
                while (!wk.done) {
                    if (wk.w + s_w > wk.pe) {
                        wk.done = true;
                        break;
                    }
                    const Eval *e = nullptr;
                    const uint64_t off = wk.w - wk.ps;
                    if (off % delta == 0) {
                        e = &ev[grid0[pi] + off / delta];
                    } else {
                        auto it = extra.find(wk.w);
                        if (it == extra.end()) {
                            need.push_back(wk.w);
                            break;
                        }
                        e = &it->second;
                    }
                    stats.windows_visited++;
                    if (e->mi >= (p->normalize == 2 ? p->sigma * e->h : thr)) {
                        found.push_back(wmi_window{wk.w, s_w, layer, e->mi});
                        wk.corr.push_back({wk.w, wk.w + s_w});
                        wk.w += s_w;
                        wk.run = 0;
                        wk.shifted = false;
                        continue;
                    }
                    if (triple && wk.shifted && e->noise) {
                        stats.noise_detections++;
                        wk.run++;
                    } else {
                        wk.run = 0;
                    }
                    if (triple && wk.run >= p->p) {
                        stats.noise_skips++;
                        wk.w += s_w;
                        wk.run = 0;
                        wk.shifted = false;
                    } else {
                        wk.w += delta;
                        wk.shifted = true;
                    }
                }
            }
            if (!need.empty()) {
                std::sort(need.begin(), need.end());
                need.erase(std::unique(need.begin(), need.end()), need.end());
                std::vector<Eval> ex;
                if (int rc = evaluate(st, a, b, need, s_w, delta, triple, prm, ex, stats))
                    return rc;
                for (size_t i = 0; i < need.size(); ++i)
                    extra[need[i]] = ex[i];
                pending = true;
            }
        }
        // uncorrelated partitions for the lower layers: each partition minus
        // its correlated windows (stretches shorter than s_min can hold no
        // window of any layer)
        std::vector<std::pair<uint64_t, uint64_t>> np;
        for (const Walk &wk : walks) {
            uint64_t at = wk.ps;
            for (const auto &c : wk.corr) {
                if (c.first - at >= p->s_min)
                    np.push_back({at, c.first});
                at = c.second;
            }
            if (wk.pe - at >= p->s_min)
                np.push_back({at, wk.pe});
        }
        parts.swap(np);
        if (s_w == 1)
            break;
    }
    std::sort(found.begin(), found.end(),
              [](const wmi_window &x, const wmi_window &y) { return x.start < y.start; });
    *n_out = found.size();
    if (found.size() > capacity)
        return fail(WMI_EINVAL, "wmi_td_search: %llu windows found, room for %llu", (unsigned long long)found.size(),
                    (unsigned long long)capacity);
    if (!found.empty() && !host_out)
        return fail(WMI_EINVAL, "wmi_td_search: null output");
    if (!found.empty())
        std::memcpy(host_out, found.data(), found.size() * sizeof(wmi_window));
    stats.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats_out)
        *stats_out = stats;
    return WMI_OK;
}

// --------------------------------------------------------------------------
// bottom-up search (Algorithm 2) with directional noise pruning
// --------------------------------------------------------------------------
namespace {

// SplitMix64 output function (Steele, Lea and Flood), used counter-based:
// pick i of walker c draws mix(seed + (c * 2^32 + i + 1) * golden).
uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t bu_pick(uint64_t seed, uint64_t chunk, uint64_t i)
{
    return splitmix64_mix(seed + ((chunk << 32) + i + 1) * 0x9E3779B97F4A7C15ull);
}

// Evaluate a query list in batches of at most kChunkQueries queries and
// kChunkPoints points.  The host planning of a batch costs about as much as
// its kernels, so a step's queries go out in up to kPlanThreads batches from
// as many host threads (the store is thread-safe): their planning overlaps
// each other's and the earlier batches' GPU time.  Results do not depend on
// the batching.  stats.submit_ms and wait_ms are summed over the threads.
constexpr unsigned kPlanThreads = 8;
constexpr uint64_t kMinThreadQueries = 8192;  // smaller batches cost more than they overlap

int run_queries(wmi_store *st, const std::vector<wmi_query> &q, const wmi_params &prm, std::vector<wmi_result> &r,
                std::vector<double> &h, wmi_search_stats &stats)
{
    r.assign(q.size(), wmi_result());
    const bool ent = (prm.flags & WMI_SUBMIT_ENTROPY) != 0;
    h.assign(ent ? 3 * q.size() : 0, 0.0);
    if (q.empty())
        return WMI_OK;
    // batch boundaries: the size caps, and at most kPlanThreads batches of at
    // least kMinThreadQueries queries each where the caps leave fewer
    const uint64_t per_thread = std::max<uint64_t>(
        kMinThreadQueries, (q.size() + kPlanThreads - 1) / kPlanThreads);
    std::vector<std::pair<size_t, size_t>> parts;
    for (size_t i0 = 0; i0 < q.size();) {
        size_t i1 = i0;
        uint64_t pts = 0;
        while (i1 < q.size() && i1 - i0 < std::min(kChunkQueries, per_thread) && (i1 == i0 || pts < kChunkPoints)) {
            pts += 2ull * q[i1].len + 2ull * q[i1].ext_len;
            ++i1;
        }
        parts.emplace_back(i0, i1);
        i0 = i1;
    }
    struct Tally {
        double submit_ms = 0.0, wait_ms = 0.0;
        uint64_t batches = 0;
        int rc = WMI_OK;
        std::string msg;
    };
    const unsigned nt = (unsigned)std::min<size_t>(kPlanThreads, parts.size());
    std::vector<Tally> tally(nt);
    std::atomic<size_t> next{0};
    std::atomic<bool> failed{false};
    auto work = [&](unsigned t) {
        Tally &y = tally[t];
        for (;;) {
            const size_t c = next.fetch_add(1);
            if (c >= parts.size() || failed.load())
                return;
            const size_t i0 = parts[c].first, i1 = parts[c].second;
            wmi_batch *bt = nullptr;
            auto t0 = Clock::now();
            int rc = wmi_submit(st, q.data() + i0, i1 - i0, &prm, nullptr, &bt);
            y.submit_ms += ms_since(t0);
            if (rc == WMI_OK) {
                t0 = Clock::now();
                rc = wmi_read(bt, r.data() + i0);
                if (rc == WMI_OK && ent)
                    rc = wmi_read_entropy(bt, h.data() + 3 * i0);
                (void)wmi_batch_destroy(bt);
                y.wait_ms += ms_since(t0);
            }
            if (rc != WMI_OK) {
                y.rc = rc;
                y.msg = wmi_last_error();  // this thread's message
                failed.store(true);
                return;
            }
            y.batches++;
        }
    };
    if (nt == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; ++t)
            pool.emplace_back(work, t);
        work(0);
        for (auto &th : pool)
            th.join();
    }
    for (const Tally &y : tally) {
        stats.submit_ms += y.submit_ms;
        stats.wait_ms += y.wait_ms;
        stats.batches += y.batches;
    }
    for (const Tally &y : tally)
        if (y.rc != WMI_OK)
            return fail(y.rc, "%s", y.msg.c_str());  // on the calling thread
    for (size_t i = 0; i < q.size(); ++i) {
        const uint64_t m = q[i].len, e = q[i].ext_len;
        if (q[i].ext_side) {
            stats.windows_evaluated += 3;
            stats.ordered_pairs += triple_pairs(m, e);
        } else {
            stats.windows_evaluated += 1;
            stats.ordered_pairs += window_pairs(m);
        }
    }
    return WMI_OK;
}

struct Walker {
    uint32_t span = 0, a = 0, b = 0;  // the span and series pair it searches
    uint64_t chunk_id = 0;
    uint64_t cursor = 0, cend = 0;  // unexplored rest of the chunk
    uint64_t picks = 0;
    bool climbing = false, done = false;
    uint64_t ws = 0, we = 0;        // current window [ws, we)
    double iw = 0.0;
    double hw = 0.0;                // H(w) when the thresholds take entropies
    std::vector<double> hist;
    uint32_t idle = 0, lrun = 0, rrun = 0;
    bool loff = false, roff = false;
    // requests of this step
    int pend = 0;                   // 0 none, 1 first window, 2 ring
    std::vector<std::pair<uint64_t, uint64_t>> ring;
    int left = -1, right = -1;      // ring entries evaluated as noise triples
    size_t req0 = 0;
};

wmi_query window_query(uint32_t a, uint32_t b, uint64_t s, uint64_t e)
{
    wmi_query q{};
    q.a = a;
    q.b = b;
    q.start = s;
    q.len = (uint32_t)(e - s);
    return q;
}

}  // namespace

namespace {

// The walkers of every span, advanced together (one batch per step).
int bu_search(wmi_store *st, const wmi_span *spans, uint64_t n_spans, const wmi_bu_params *p, wmi_window *host_out,
              uint32_t *host_span, uint64_t capacity, uint64_t *n_out, wmi_search_stats *stats_out, const char *who)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!st || !p || !n_out || (n_spans && !spans))
        return fail(WMI_EINVAL, "%s: null argument", who);
    *n_out = 0;
    if (p->s_min < 2 || p->s_min > p->s_max || p->s_max > (uint32_t)WMI_MAX_WINDOW || p->delta < 1 ||
        p->history < 1 || p->flags || p->reserved)
        return fail(WMI_EINVAL, "%s: need 2 <= s_min <= s_max <= %d, delta >= 1, history >= 1", who,
                    WMI_MAX_WINDOW);
    if (p->k < 1 || p->k > WMI_MAX_K || p->estimator > 1 || p->normalize > 2)
        return fail(WMI_EINVAL, "%s: bad k, estimator or normalize", who);
    std::vector<Walker> walkers;
    for (uint64_t si = 0; si < n_spans; ++si) {
        const wmi_span &sp = spans[si];
        uint64_t na = 0, nb = 0;
        if (int rc = wmi_series_length(st, sp.a, &na))
            return rc;
        if (int rc = wmi_series_length(st, sp.b, &nb))
            return rc;
        if (sp.begin > sp.end || sp.end > std::min(na, nb))
            return fail(WMI_EINVAL, "%s: span %llu outside the series", who, (unsigned long long)si);
        const uint64_t chunk = p->chunk ? p->chunk : std::max<uint64_t>(sp.end - sp.begin, 1);
        for (uint64_t c0 = sp.begin, id = 0; c0 < sp.end; c0 += chunk, ++id) {
            Walker w;
            w.span = (uint32_t)si;
            w.a = sp.a;
            w.b = sp.b;
            w.chunk_id = id;
            w.cursor = c0;
            w.cend = std::min(sp.end, c0 + chunk);
            walkers.push_back(w);
        }
    }
    wmi_params prm{};
    prm.k = p->k;
    prm.estimator = p->estimator;
    prm.tau = p->tau;
    prm.tau_normalize = p->normalize;
    prm.flags = p->normalize == 2 ? WMI_SUBMIT_ENTROPY : 0u;
    const bool prune = p->p > 0;
    const uint64_t d = p->delta;

    wmi_search_stats stats{};
    std::vector<wmi_window> found;
    std::vector<uint32_t> found_span;
    std::vector<wmi_query> q;
    std::vector<wmi_result> res;
    std::vector<double> hres;
    // report threshold of a walker's window: sigma, sigma ln|w| or sigma H(w)
    auto threshold = [&](const Walker &w) {
        if (p->normalize == 2)
            return p->sigma * w.hw;
        return p->normalize ? p->sigma * std::log((double)(w.we - w.ws)) : p->sigma;
    };

    for (;;) {
        q.clear();
        bool any = false;
        for (Walker &w : walkers) {
            w.pend = 0;
            while (!w.done && w.pend == 0) {
                if (!w.climbing) {
                    if (w.cend - w.cursor < p->s_min) {
                        w.done = true;
                        break;
                    }
                    w.ws = w.cursor;
                    w.we = w.cursor + p->s_min;
                    w.pend = 1;
                    w.req0 = q.size();
                    q.push_back(window_query(w.a, w.b, w.ws, w.we));
                    stats.windows_visited++;
                    break;
                }
                // the ring of radius r = idle + 1 around w
                const uint64_t r = w.idle + 1ull, rd = r * d;
                w.ring.clear();
                w.left = w.right = -1;
                for (int64_t ds = -(int64_t)r; ds <= (int64_t)r; ++ds)
                    for (int64_t de = -(int64_t)r; de <= (int64_t)r; ++de) {
                        if (std::max(std::llabs(ds), std::llabs(de)) != (int64_t)r)
                            continue;
                        const int64_t s = (int64_t)w.ws + ds * (int64_t)d, e = (int64_t)w.we + de * (int64_t)d;
                        if (s < (int64_t)w.cursor || e > (int64_t)w.cend || e - s < (int64_t)p->s_min ||
                            e - s > (int64_t)p->s_max)
                            continue;
                        if ((w.loff && ds < 0) || (w.roff && de > 0))
                            continue;
                        if (prune && ds == -(int64_t)r && de == 0)
                            w.left = (int)w.ring.size();
                        if (prune && ds == 0 && de == (int64_t)r)
                            w.right = (int)w.ring.size();
                        w.ring.push_back({(uint64_t)s, (uint64_t)e});
                    }
                if (w.ring.empty()) {
                    // nothing to examine: an iteration without improvement
                    const uint64_t j = bu_pick(p->seed, w.chunk_id, w.picks++) % p->history;
                    w.idle++;
                    if (w.iw > w.hist[j])
                        w.hist[j] = w.iw;
                    if (w.idle > p->max_idle) {
                        if (w.iw >= threshold(w)) {
                            found.push_back(wmi_window{w.ws, (uint32_t)(w.we - w.ws), 0, w.iw});
                            found_span.push_back(w.span);
                        }
                        w.cursor = w.we;
                        w.climbing = false;
                    }
                    continue;
                }
                w.pend = 2;
                w.req0 = q.size();
                for (size_t i = 0; i < w.ring.size(); ++i) {
                    wmi_query x = window_query(w.a, w.b, w.ring[i].first, w.ring[i].second);
                    if ((int)i == w.left) {  // base w, extension on the left
                        x = window_query(w.a, w.b, w.ws, w.we);
                        x.ext_len = (uint32_t)rd;
                        x.ext_side = -1;
                    } else if ((int)i == w.right) {
                        x = window_query(w.a, w.b, w.ws, w.we);
                        x.ext_len = (uint32_t)rd;
                        x.ext_side = 1;
                    }
                    q.push_back(x);
                }
                stats.windows_visited += w.ring.size();
            }
            any = any || !w.done;
        }
        if (!any)
            break;
        if (q.empty())
            continue;
        if (int rc = run_queries(st, q, prm, res, hres, stats))
            return rc;
        for (Walker &w : walkers) {
            if (w.pend == 1) {
                w.iw = res[w.req0].mi_base;
                w.hw = hres.empty() ? 0.0 : hres[3 * w.req0];
                w.hist.assign(p->history, w.iw);
                w.idle = 0;
                w.lrun = w.rrun = 0;
                w.loff = w.roff = false;
                w.climbing = true;
            } else if (w.pend == 2) {
                int best = -1;
                double ib = 0.0;
                for (size_t i = 0; i < w.ring.size(); ++i) {
                    const wmi_result &x = res[w.req0 + i];
                    const double v = ((int)i == w.left || (int)i == w.right) ? x.mi_union : x.mi_base;
                    if (!std::isnan(v) && (best < 0 || v > ib)) {
                        best = (int)i;
                        ib = v;
                    }
                }
                if (w.left >= 0) {
                    const bool nz = (res[w.req0 + w.left].flags & WMI_F_NOISE) != 0;
                    stats.noise_detections += nz;
                    w.lrun = nz ? w.lrun + 1 : 0;
                }
                if (w.right >= 0) {
                    const bool nz = (res[w.req0 + w.right].flags & WMI_F_NOISE) != 0;
                    stats.noise_detections += nz;
                    w.rrun = nz ? w.rrun + 1 : 0;
                }
                const uint64_t j = bu_pick(p->seed, w.chunk_id, w.picks++) % p->history;
                if (best >= 0 && (ib > w.hist[j] || ib > w.iw)) {
                    w.ws = w.ring[best].first;
                    w.we = w.ring[best].second;
                    w.iw = ib;
                    if (!hres.empty())  // a triple's window is its union
                        w.hw = hres[3 * (w.req0 + best) + ((best == w.left || best == w.right) ? 2 : 0)];
                    w.idle = 0;
                } else {
                    w.idle++;
                }
                if (w.iw > w.hist[j])
                    w.hist[j] = w.iw;
                if (prune && !w.loff && w.lrun >= p->p) {
                    w.loff = true;
                    stats.noise_skips++;
                }
                if (prune && !w.roff && w.rrun >= p->p) {
                    w.roff = true;
                    stats.noise_skips++;
                }
                if (w.idle > p->max_idle) {
                    if (w.iw >= threshold(w)) {
                        found.push_back(wmi_window{w.ws, (uint32_t)(w.we - w.ws), 0, w.iw});
                        found_span.push_back(w.span);
                    }
                    w.cursor = w.we;
                    w.climbing = false;
                }
            }
        }
    }
    // by span, then start
    std::vector<size_t> order(found.size());
    for (size_t i = 0; i < order.size(); ++i)
        order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return found_span[x] != found_span[y] ? found_span[x] < found_span[y] : found[x].start < found[y].start;
    });
    *n_out = found.size();
    if (found.size() > capacity)
        return fail(WMI_EINVAL, "%s: %llu windows found, room for %llu", who, (unsigned long long)found.size(),
                    (unsigned long long)capacity);
    if (!found.empty() && !host_out)
        return fail(WMI_EINVAL, "%s: null output", who);
    for (size_t i = 0; i < order.size(); ++i) {
        host_out[i] = found[order[i]];
        if (host_span)
            host_span[i] = found_span[order[i]];
    }
    stats.layers = 1;
    stats.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats_out)
        *stats_out = stats;
    return WMI_OK;
}

}  // namespace

extern "C" int wmi_bu_search(wmi_store *st, uint32_t a, uint32_t b, uint64_t begin, uint64_t end,
                             const wmi_bu_params *p, wmi_window *host_out, uint64_t capacity, uint64_t *n_out,
                             wmi_search_stats *stats_out)
{
    const wmi_span sp{a, b, begin, end};
    return bu_search(st, &sp, 1, p, host_out, nullptr, capacity, n_out, stats_out, "wmi_bu_search");
}

extern "C" int wmi_bu_search_many(wmi_store *st, const wmi_span *spans, uint64_t n_spans, const wmi_bu_params *p,
                                  wmi_window *host_out, uint32_t *host_span, uint64_t capacity, uint64_t *n_out,
                                  wmi_search_stats *stats_out)
{
    return bu_search(st, spans, n_spans, p, host_out, host_span, capacity, n_out, stats_out, "wmi_bu_search_many");
}
