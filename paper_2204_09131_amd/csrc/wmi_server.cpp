// wmi_server.cpp -- continuous batching of range requests (include/wmi.h).
//
// A scheduler thread owns every request after submission:
//   queued    waiting, in arrival order, for its result slice of the arena
//   admitted  holds a slice; its windows are taken into launches in order
//   copying   all windows done; its slice is being downloaded
//   done      results in host memory until read
// Each pass of the loop admits what fits, retires finished launches and
// downloads, and fills any idle launch slot with the next windows of the
// admitted requests (oldest first, cut at the slot's capacity).  A launch is a
// short list of parts -- runs of equally spaced windows of one request -- that
// the expand kernel turns into window descriptors and queue items on the
// device, so the host does work per part, not per window.  Two slots on two
// streams let one launch be built while the other runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wmi.h"
#include "wmi_internal.h"
#include "wmi_plan.h"
#include "wmi_store.h"

using namespace wmi;

static_assert(sizeof(wmi_request) == 32, "wmi_request layout");
static_assert(sizeof(wmi_window_result) == 16 && sizeof(CompactResult) == 16, "window result layout");
static_assert(sizeof(PartDesc) == 64, "part layout");

namespace {

constexpr uint64_t kDefaultArena = 256ull << 20;
constexpr uint32_t kDefaultLaunchWindows = 65536;
constexpr uint32_t kMaxParts = 2048;
constexpr uint64_t kLaunchSplitPoints = 16ull << 20;  // points of windows above kLocalSlots per launch
constexpr uint64_t kArenaUnit = 256;

// First-fit allocator over [0, size) in kArenaUnit units.
struct ArenaAlloc {
    uint64_t size = 0, used = 0, peak = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    void init(uint64_t n)
    {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    static uint64_t round(uint64_t n) { return (n + kArenaUnit - 1) / kArenaUnit * kArenaUnit; }
    bool alloc(uint64_t n, uint64_t &off)
    {
        n = round(std::max<uint64_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n)
                continue;
            off = it->first;
            const uint64_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest)
                free_[at] = rest;
            used += n;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = round(std::max<uint64_t>(n, 1));
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Req {
    uint64_t ticket = 0;
    wmi_request r{};
    uint64_t nwin = 0, next = 0, done = 0, pairs = 0;
    uint64_t arena_off = 0;
    bool has_arena = false;
    bool pinned = false;  // holds a reader count on series a and b (store mutex)
    int32_t state = 0;  // 0 queued, 1 admitted, 3 copying, 2 done, < 0 error
    double t_arrival = 0, t_admit = 0, t_first = 0, t_complete = 0;
    uint32_t launches = 0, inflight = 0;
    hipEvent_t ev_copy = nullptr;
    std::vector<wmi_window_result> host;
};

struct Part {
    Req *r;
    uint64_t first;
    uint32_t count;
};

struct Slot {
    char *dev = nullptr;
    char *host = nullptr;  // pinned: parts, then the error word
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool busy = false;
    std::vector<Part> parts;
    size_t o_parts = 0, o_win = 0, o_qd = 0, o_queue = 0, o_cdst = 0, o_sorted = 0, o_acc = 0, o_wdone = 0,
           o_qdone = 0, o_counter = 0, o_wmi = 0, o_wflags = 0, o_ready = 0, o_err = 0, bytes = 0;
    size_t h_err = 0, host_bytes = 0;
};

}  // namespace

struct wmi_server {
    wmi_store *st = nullptr;
    uint32_t k = 4, est = 0, cap_windows = kDefaultLaunchWindows, cap_items = 0;
    uint64_t cap_split = kLaunchSplitPoints;
    CompactResult *arena_dev = nullptr;
    char *arena_host = nullptr;  // pinned mirror of the arena
    ArenaAlloc arena;
    Slot slots[2];
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_origin = nullptr;  // device-time origin of the launch intervals
    std::vector<std::pair<float, float>> intervals;  // launch [start, end) in ms after ev_origin
    int occupancy = 1;
    Tuning tune;  // the store's work-list choices when the server was created
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;       // request state changes
    std::condition_variable cv_work;  // new submissions / stop
    std::deque<Req *> incoming;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool failed = false;
    std::chrono::steady_clock::time_point t0;
    wmi_server_stats stats{};

    double now() const
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void layout_slot(Slot &s, uint32_t cap_windows, uint32_t cap_items, uint64_t cap_split)
{
    const size_t A = 256;
    s.o_parts = 0;
    s.o_win = align_up(s.o_parts + kMaxParts * sizeof(PartDesc), A);
    s.o_qd = align_up(s.o_win + (size_t)cap_windows * sizeof(WinDesc), A);
    s.o_queue = align_up(s.o_qd + (size_t)cap_windows * sizeof(QDesc), A);
    s.o_cdst = align_up(s.o_queue + (size_t)cap_items * sizeof(Item), A);
    s.o_sorted = align_up(s.o_cdst + (size_t)cap_windows * sizeof(uint64_t), A);
    s.o_acc = align_up(s.o_sorted + (size_t)kSortedWords * cap_split * sizeof(int32_t), A);
    s.o_wdone = align_up(s.o_acc + (size_t)cap_windows * sizeof(unsigned long long), A);
    s.o_qdone = align_up(s.o_wdone + (size_t)cap_windows * sizeof(uint32_t), A);
    s.o_counter = align_up(s.o_qdone + (size_t)cap_windows * sizeof(uint32_t), A);
    s.o_wmi = align_up(s.o_counter + sizeof(uint32_t), A);
    s.o_wflags = align_up(s.o_wmi + (size_t)cap_windows * sizeof(double), A);
    s.o_ready = align_up(s.o_wflags + (size_t)cap_windows * sizeof(uint32_t), A);
    s.o_err = align_up(s.o_ready + (size_t)cap_windows * sizeof(uint32_t), A);
    s.bytes = align_up(s.o_err + sizeof(uint32_t), A);
    s.h_err = align_up(kMaxParts * sizeof(PartDesc), A);
    s.host_bytes = s.h_err + A;
}

void fail_all(wmi_server *S, int code)
{
    std::lock_guard<std::mutex> lk(S->mu);
    S->failed = true;
    for (auto &kv : S->reqs)
        if (kv.second->state != 2)
            kv.second->state = code;
    S->cv.notify_all();
}

// Give back the request's reader counts on its series, once: a request that
// failed after its download may reach here again from destroy.
void unpin(wmi_server *S, Req *r)
{
    std::lock_guard<std::mutex> lk(S->st->mu);
    if (!r->pinned)
        return;
    r->pinned = false;
    for (uint32_t id : {r->r.a, r->r.b})
        if (id < S->st->series.size() && S->st->series[id].busy)
            S->st->series[id].busy--;
    S->st->cv.notify_all();
}

// Fill an idle slot with the next windows of the admitted requests and
// enqueue it (*launched false if there was nothing to launch).
int launch(wmi_server *S, Slot &slot, std::deque<Req *> &active, bool &launched)
{
    launched = false;
    wmi_store *st = S->st;
    slot.parts.clear();
    uint64_t nwin = 0, nsplit_pts = 0;
    std::vector<Series> ser;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        ser = st->series;
    }
    while (!active.empty() && slot.parts.size() < kMaxParts && nwin < S->cap_windows) {
        Req *r = active.front();
        const uint32_t m = r->r.w;
        uint64_t take = std::min<uint64_t>(r->nwin - r->next, S->cap_windows - nwin);
        if (m > (uint32_t)kLocalSlots)
            take = std::min<uint64_t>(take, (S->cap_split - nsplit_pts) / m);
        if (take == 0)
            break;
        slot.parts.push_back(Part{r, r->next, (uint32_t)take});
        nwin += take;
        if (m > (uint32_t)kLocalSlots)
            nsplit_pts += take * m;
        if (r->launches == 0)
            r->t_first = S->now();
        r->launches++;
        r->inflight++;
        r->next += take;
        if (r->next == r->nwin)
            active.pop_front();
    }
    if (slot.parts.empty())
        return WMI_OK;

    PartDesc *pd = reinterpret_cast<PartDesc *>(slot.host);
    for (uint32_t i = 0; i < slot.parts.size(); ++i) {
        const Part &p = slot.parts[i];
        PartDesc &d = pd[i];
        d.x = ser[p.r->r.a].d;
        d.y = ser[p.r->r.b].d;
        d.start = p.r->r.start + p.first * p.r->r.stride;
        d.dst = p.r->arena_off / sizeof(CompactResult) + p.first;
        d.stride = p.r->r.stride;
        d.count = p.count;
        d.m = p.r->r.w;
    }
    uint64_t split_pts = 0;
    const uint32_t n_items = plan_parts(pd, (uint32_t)slot.parts.size(), &split_pts, &S->tune);
    if (n_items > S->cap_items || split_pts > S->cap_split)
        return fail(WMI_EINVAL, "server launch exceeds its slot (%u items, %llu points)", n_items,
                    (unsigned long long)split_pts);

    LaunchArgs a{};
    char *D = slot.dev;
    a.win = reinterpret_cast<const WinDesc *>(D + slot.o_win);
    a.item = reinterpret_cast<const Item *>(D + slot.o_queue);
    a.qd = reinterpret_cast<const QDesc *>(D + slot.o_qd);
    a.sorted = reinterpret_cast<int32_t *>(D + slot.o_sorted);
    a.acc = reinterpret_cast<unsigned long long *>(D + slot.o_acc);
    a.wdone = reinterpret_cast<uint32_t *>(D + slot.o_wdone);
    a.qdone = reinterpret_cast<uint32_t *>(D + slot.o_qdone);
    a.counter = reinterpret_cast<uint32_t *>(D + slot.o_counter);
    a.wmi = reinterpret_cast<double *>(D + slot.o_wmi);
    a.wflags = reinterpret_cast<uint32_t *>(D + slot.o_wflags);
    a.ready = reinterpret_cast<uint32_t *>(D + slot.o_ready);
    a.err = reinterpret_cast<uint32_t *>(D + slot.o_err);
    a.res = nullptr;
    a.cdst = reinterpret_cast<const uint64_t *>(D + slot.o_cdst);
    a.arena = S->arena_dev;
    a.psi_d = st->psi_d;
    a.psi_fix = st->psi_fix;
    a.n_win = (uint32_t)nwin;
    a.n_items = n_items;
    a.n_query = (uint32_t)nwin;
    a.k = S->k;
    a.estimator = S->est;
    a.persistent = 1;
    for (int i = 0; i < 3; ++i)
        a.strag[i] = S->tune.stragglers[i];
    const uint32_t grid = (uint32_t)std::min<uint64_t>(n_items, (uint64_t)st->cu_count * S->occupancy);
    hipStream_t s = slot.stream;
    HIPCHK(st, hipEventRecord(slot.ev0, s));
    HIPCHK(st, hipMemcpyAsync(D + slot.o_parts, slot.host, slot.parts.size() * sizeof(PartDesc),
                              hipMemcpyHostToDevice, s));
    HIPCHK(st, launch_expand(a, reinterpret_cast<const PartDesc *>(D + slot.o_parts), (uint32_t)slot.parts.size(),
                             reinterpret_cast<Item *>(D + slot.o_queue), reinterpret_cast<WinDesc *>(D + slot.o_win),
                             reinterpret_cast<QDesc *>(D + slot.o_qd), reinterpret_cast<uint64_t *>(D + slot.o_cdst),
                             s));
    HIPCHK(st, launch_clear(a, s));
    HIPCHK(st, launch_main(a, grid, s));
    HIPCHK(st, hipMemcpyAsync(slot.host + slot.h_err, D + slot.o_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(st, hipEventRecord(slot.ev1, s));
    slot.busy = true;
    launched = true;
    return WMI_OK;
}

void scheduler(wmi_server *S)
{
    wmi_store *st = S->st;
    DeviceGuard g(st->device);
    std::deque<Req *> queued, active;
    std::vector<Req *> copying;
    for (;;) {
        bool progress = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            while (!S->incoming.empty()) {
                queued.push_back(S->incoming.front());
                S->incoming.pop_front();
            }
            const bool idle = queued.empty() && active.empty() && copying.empty() && !S->slots[0].busy &&
                              !S->slots[1].busy;
            if (idle && (S->stop || S->failed))
                break;
            if (idle) {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            // admission, in arrival order: a slice of the arena for the results
            while (!queued.empty() && !S->failed) {
                Req *r = queued.front();
                if (r->nwin == 0) {
                    r->state = 2;
                    r->t_admit = r->t_first = r->t_complete = S->now();
                    queued.pop_front();
                    S->stats.requests_done++;
                    S->cv.notify_all();
                    continue;
                }
                uint64_t off = 0;
                if (!S->arena.alloc(r->nwin * sizeof(CompactResult), off))
                    break;
                r->arena_off = off;
                r->has_arena = true;
                r->state = 1;
                r->t_admit = S->now();
                active.push_back(r);
                queued.pop_front();
                progress = true;
            }
            S->stats.queued_peak = std::max<uint64_t>(S->stats.queued_peak, queued.size());
            S->stats.arena_peak_bytes = S->arena.peak;
        }
        if (S->failed)
            break;
        // finished launches
        for (Slot &slot : S->slots) {
            if (!slot.busy)
                continue;
            hipError_t e = hipEventQuery(slot.ev1);
            if (e == hipErrorNotReady)
                continue;
            if (e != hipSuccess) {
                poison(st, e, "server launch");
                fail_all(S, WMI_EHIP);
                break;
            }
            float ms = 0.f, t_start = 0.f, t_end = 0.f;
            (void)hipEventElapsedTime(&ms, slot.ev0, slot.ev1);
            const bool have_iv = hipEventElapsedTime(&t_start, S->ev_origin, slot.ev0) == hipSuccess &&
                                 hipEventElapsedTime(&t_end, S->ev_origin, slot.ev1) == hipSuccess;
            uint32_t err = 0;
            std::memcpy(&err, slot.host + slot.h_err, sizeof err);
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.busy_us += 1e3 * ms;
            if (have_iv)
                S->intervals.emplace_back(t_start, t_end);
            S->stats.launches++;
            for (const Part &p : slot.parts) {
                Req *r = p.r;
                r->done += p.count;
                r->inflight--;
                if (err)
                    r->state = WMI_EHIP;
                if (r->done == r->nwin) {
                    const size_t bytes = r->nwin * sizeof(CompactResult);
                    hipError_t e2 = hipMemcpyAsync(S->arena_host + r->arena_off,
                                                   reinterpret_cast<char *>(S->arena_dev) + r->arena_off, bytes,
                                                   hipMemcpyDeviceToHost, S->copy_stream);
                    if (e2 == hipSuccess)
                        e2 = hipEventRecord(r->ev_copy, S->copy_stream);
                    if (e2 != hipSuccess) {
                        S->failed = true;
                        r->state = WMI_EHIP;
                    } else if (r->state >= 0) {
                        r->state = 3;
                    }
                    copying.push_back(r);
                }
            }
            slot.busy = false;
            progress = true;
        }
        // finished downloads
        for (size_t i = 0; i < copying.size();) {
            Req *r = copying[i];
            hipError_t e = hipEventQuery(r->ev_copy);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            r->host.resize(r->nwin);
            std::memcpy(r->host.data(), S->arena_host + r->arena_off, r->nwin * sizeof(CompactResult));
            unpin(S, r);
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.release(r->arena_off, r->nwin * sizeof(CompactResult));
            r->has_arena = false;
            if (e != hipSuccess)
                r->state = WMI_EHIP;
            if (r->state >= 0) {
                r->state = 2;
                S->stats.requests_done++;
                S->stats.windows_done += r->nwin;
                S->stats.ordered_pairs_done += r->pairs;
            }
            r->t_complete = S->now();
            S->cv.notify_all();
            copying[i] = copying.back();
            copying.pop_back();
            progress = true;
        }
        // idle slots take the next windows
        for (Slot &slot : S->slots) {
            if (slot.busy || active.empty())
                continue;
            bool launched = false;
            int rc;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                rc = launch(S, slot, active, launched);
            }
            if (rc != WMI_OK) {
                fail_all(S, rc);
                break;
            }
            progress = progress || launched;
        }
        if (!progress)
            std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
}

}  // namespace

extern "C" {

int wmi_server_create(wmi_store *st, const wmi_server_desc *desc, wmi_server **out)
{
    if (!st || !desc || !out)
        return fail(WMI_EINVAL, "wmi_server_create: null argument");
    *out = nullptr;
    if (desc->k < 1 || desc->k > WMI_MAX_K || desc->estimator > 1 || desc->flags)
        return fail(WMI_EINVAL, "wmi_server_create: bad k, estimator or flags");
    if (int rc = check_poison(st))
        return rc;
    DeviceGuard g(st->device);
    wmi_server *S = new wmi_server();
    S->st = st;
    S->k = desc->k;
    S->est = desc->estimator;
    S->cap_windows = desc->max_launch_windows ? desc->max_launch_windows : kDefaultLaunchWindows;
    S->cap_items = S->cap_windows * 10u;  // local: <= 1 per window; split: prep + up to 8 per window
    const uint64_t arena_bytes = ArenaAlloc::round(desc->hbm_budget_bytes ? desc->hbm_budget_bytes : kDefaultArena);
    S->arena.init(arena_bytes);
    S->stats.arena_bytes = arena_bytes;
    S->occupancy = main_occupancy(S->k);
    {
        std::lock_guard<std::mutex> lk(st->mu);
        S->tune = st->tune;
    }
    S->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipMalloc(&S->arena_dev, arena_bytes);
    if (e == hipSuccess)
        e = hipHostMalloc(&S->arena_host, arena_bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking);
    for (Slot &slot : S->slots) {
        layout_slot(slot, S->cap_windows, S->cap_items, S->cap_split);
        if (e == hipSuccess)
            e = hipMalloc(&slot.dev, slot.bytes);
        if (e == hipSuccess)
            e = hipHostMalloc(&slot.host, slot.host_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreate(&slot.ev0);
        if (e == hipSuccess)
            e = hipEventCreate(&slot.ev1);
    }
    if (e == hipSuccess)
        e = hipEventCreate(&S->ev_origin);
    if (e == hipSuccess)
        e = hipEventRecord(S->ev_origin, S->slots[0].stream);
    if (e == hipSuccess)
        e = hipEventSynchronize(S->ev_origin);
    if (e != hipSuccess) {
        int rc = fail(WMI_EHIP, "wmi_server_create: %s", hipGetErrorString(e));
        for (Slot &slot : S->slots) {
            if (slot.dev) (void)hipFree(slot.dev);
            if (slot.host) (void)hipHostFree(slot.host);
            if (slot.stream) (void)hipStreamDestroy(slot.stream);
            if (slot.ev0) (void)hipEventDestroy(slot.ev0);
            if (slot.ev1) (void)hipEventDestroy(slot.ev1);
        }
        if (S->arena_dev) (void)hipFree(S->arena_dev);
        if (S->arena_host) (void)hipHostFree(S->arena_host);
        if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
        if (S->ev_origin) (void)hipEventDestroy(S->ev_origin);
        delete S;
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(st->mu);
        st->servers.insert(S);
    }
    S->th = std::thread(scheduler, S);
    *out = S;
    return WMI_OK;
}

int wmi_server_submit(wmi_server *S, const wmi_request *req, uint64_t *ticket)
{
    if (!S || !req || !ticket)
        return fail(WMI_EINVAL, "wmi_server_submit: null argument");
    const wmi_request r = *req;
    if (r.w < 1 || r.w > (uint32_t)WMI_MAX_WINDOW)
        return fail(WMI_EINVAL, "wmi_server_submit: window of %u points outside 1..%d", r.w, WMI_MAX_WINDOW);
    if (r.stride < 1)
        return fail(WMI_EINVAL, "wmi_server_submit: stride must be >= 1");
    if (r.end < r.start)
        return fail(WMI_EINVAL, "wmi_server_submit: end before start");
    wmi_store *st = S->st;
    Req *q = new Req();
    {
        std::lock_guard<std::mutex> lk(st->mu);
        if (r.a >= st->series.size() || !st->series[r.a].live || r.b >= st->series.size() || !st->series[r.b].live) {
            delete q;
            return fail(WMI_EINVAL, "wmi_server_submit: unknown series id (%u, %u)", r.a, r.b);
        }
        const uint64_t n = std::min(st->series[r.a].n, st->series[r.b].n);
        if (r.end > n) {
            delete q;
            return fail(WMI_EINVAL, "wmi_server_submit: range end %llu beyond series of %llu points",
                        (unsigned long long)r.end, (unsigned long long)n);
        }
        q->nwin = (r.end - r.start >= r.w) ? (r.end - r.start - r.w) / r.stride + 1 : 0;
        if (q->nwin * sizeof(CompactResult) > S->arena.size) {
            delete q;
            return fail(WMI_ENOMEM, "wmi_server_submit: %llu windows need more than the %llu-byte arena",
                        (unsigned long long)q->nwin, (unsigned long long)S->arena.size);
        }
        if (q->nwin > 0xFFFFFFF0ull) {
            delete q;
            return fail(WMI_EINVAL, "wmi_server_submit: too many windows in one request");
        }
        st->series[r.a].busy++;
        st->series[r.b].busy++;
        q->pinned = true;
    }
    q->r = r;
    q->pairs = q->nwin * (uint64_t)r.w * (r.w - 1);
    {
        DeviceGuard g(st->device);
        if (hipEventCreateWithFlags(&q->ev_copy, hipEventDisableTiming) != hipSuccess) {
            unpin(S, q);
            delete q;
            return fail(WMI_EHIP, "wmi_server_submit: hipEventCreate failed");
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop || S->failed) {
        unpin(S, q);
        (void)hipEventDestroy(q->ev_copy);
        delete q;
        return fail(WMI_ESTATE, "wmi_server_submit: server stopping or failed");
    }
    q->ticket = S->next_ticket++;
    q->t_arrival = S->now();
    S->reqs[q->ticket] = q;
    S->incoming.push_back(q);
    S->cv_work.notify_one();
    *ticket = q->ticket;
    return WMI_OK;
}

static void fill_info(const Req *r, wmi_request_info *info)
{
    info->windows = r->nwin;
    info->t_arrival_us = r->t_arrival;
    info->t_admit_us = r->t_admit;
    info->t_first_launch_us = r->t_first;
    info->t_complete_us = r->t_complete;
    info->state = r->state == 3 ? 1 : r->state;
    info->launches = r->launches;
}

int wmi_server_wait(wmi_server *S, uint64_t ticket, int64_t timeout_us)
{
    if (!S)
        return fail(WMI_EINVAL, "wmi_server_wait: null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return fail(WMI_EINVAL, "wmi_server_wait: unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second;
    auto pred = [&] { return r->state == 2 || r->state < 0; };
    if (timeout_us < 0)
        S->cv.wait(lk, pred);
    else if (!S->cv.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
        return fail(WMI_ETIMEDOUT, "wmi_server_wait: request %llu not done after %lld us", (unsigned long long)ticket,
                    (long long)timeout_us);
    if (r->state < 0)
        return fail(r->state, "wmi_server_wait: request %llu failed", (unsigned long long)ticket);
    return WMI_OK;
}

int wmi_server_info(wmi_server *S, uint64_t ticket, wmi_request_info *info)
{
    if (!S || !info)
        return fail(WMI_EINVAL, "wmi_server_info: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return fail(WMI_EINVAL, "wmi_server_info: unknown ticket %llu", (unsigned long long)ticket);
    fill_info(it->second, info);
    return WMI_OK;
}

int wmi_server_read(wmi_server *S, uint64_t ticket, wmi_window_result *out, uint64_t capacity,
                    wmi_request_info *info)
{
    if (!S)
        return fail(WMI_EINVAL, "wmi_server_read: null server");
    Req *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end())
            return fail(WMI_EINVAL, "wmi_server_read: unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        if (r->state < 0)
            return fail(r->state, "wmi_server_read: request %llu failed", (unsigned long long)ticket);
        if (r->state != 2)
            return fail(WMI_ESTATE, "wmi_server_read: request %llu not complete", (unsigned long long)ticket);
        if (capacity < r->nwin || (r->nwin && !out))
            return fail(WMI_EINVAL, "wmi_server_read: room for %llu results, request has %llu",
                        (unsigned long long)capacity, (unsigned long long)r->nwin);
        if (r->nwin)
            std::memcpy(out, r->host.data(), r->nwin * sizeof(wmi_window_result));
        if (info)
            fill_info(r, info);
        S->reqs.erase(it);
    }
    DeviceGuard g(S->st->device);
    (void)hipEventDestroy(r->ev_copy);
    delete r;
    return WMI_OK;
}

int wmi_server_stats_get(wmi_server *S, wmi_server_stats *out)
{
    if (!S || !out)
        return fail(WMI_EINVAL, "wmi_server_stats_get: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    // union of the launch intervals: device time with at least one launch
    // of the server in flight (the two slots overlap)
    std::vector<std::pair<float, float>> iv = S->intervals;
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, cur_s = 0.0, cur_e = -1.0;
    for (const auto &p : iv) {
        if (p.first > cur_e) {
            if (cur_e > cur_s)
                busy += cur_e - cur_s;
            cur_s = p.first;
            cur_e = p.second;
        } else if (p.second > cur_e) {
            cur_e = p.second;
        }
    }
    if (cur_e > cur_s)
        busy += cur_e - cur_s;
    out->busy_union_us = 1e3 * busy;
    return WMI_OK;
}

double wmi_server_clock_us(wmi_server *S) { return S ? S->now() : 0.0; }

int wmi_server_destroy(wmi_server *S)
{
    if (!S)
        return WMI_OK;
    wmi_store *st = S->st;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->th.joinable())
        S->th.join();
    DeviceGuard g(st->device);
    for (Slot &slot : S->slots)
        if (slot.stream)
            (void)hipStreamSynchronize(slot.stream);
    (void)hipStreamSynchronize(S->copy_stream);
    for (auto &kv : S->reqs) {
        Req *r = kv.second;
        unpin(S, r);
        (void)hipEventDestroy(r->ev_copy);
        delete r;
    }
    for (Slot &slot : S->slots) {
        (void)hipFree(slot.dev);
        (void)hipHostFree(slot.host);
        (void)hipStreamDestroy(slot.stream);
        (void)hipEventDestroy(slot.ev0);
        (void)hipEventDestroy(slot.ev1);
    }
    (void)hipFree(S->arena_dev);
    (void)hipHostFree(S->arena_host);
    (void)hipStreamDestroy(S->copy_stream);
    (void)hipEventDestroy(S->ev_origin);
    {
        std::lock_guard<std::mutex> lk(st->mu);
        st->servers.erase(S);
    }
    delete S;
    return WMI_OK;
}

}  // extern "C"
