// wmi_runtime.cpp -- host runtime behind the C-ABI of include/wmi.h.
//
// A store holds resident series on one device, the digamma tables and a
// memory budget.  A submit validates queries, expands noise triples into
// their three windows (Definition 6.2 as applied in Section 6.2: overlap,
// newly added part, union), builds the window and work-item descriptors in
// pinned host memory, and enqueues on one stream:
//   descriptor upload -> clear -> prep (sort) -> persistent main -> result download
// Work items are (window, block of 512 query points); the persistent kernel
// takes them largest-first from an atomic counter.  A batch can be replayed as
// a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "wmi.h"
#include "wmi_internal.h"
#include "wmi_plan.h"
#include "wmi_store.h"


using namespace wmi;

static_assert(sizeof(wmi_query) == 32, "wmi_query layout");
static_assert(sizeof(wmi_result) == 32 && sizeof(Result) == 32, "result layout");
static_assert(sizeof(WinDesc) == 32 && sizeof(Item) == 8 && sizeof(QDesc) == 16, "descriptors");
static_assert(sizeof(wmi_tuning) == sizeof(Tuning), "tuning layout");

namespace wmi {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char *last_error() { return g_err.c_str(); }

int poison(wmi_store *st, hipError_t e, const char *what)
{
    std::lock_guard<std::mutex> lk(st->mu);
    st->poisoned = true;
    st->poison_msg = std::string(what) + ": " + hipGetErrorString(e);
    return fail(WMI_EHIP, "%s", st->poison_msg.c_str());
}

int check_poison(wmi_store *st)
{
    std::lock_guard<std::mutex> lk(st->mu);
    if (st->poisoned)
        return fail(WMI_EHIP, "store poisoned by an earlier HIP error: %s", st->poison_msg.c_str());
    return WMI_OK;
}

}  // namespace wmi

// Events of one run: start, prep start, main start, main end, end.
struct RunEvents {
    hipEvent_t s0 = nullptr, p0 = nullptr, m0 = nullptr, m1 = nullptr, s1 = nullptr;
    int mode = 0;  // 0 direct (per-kernel events valid), 1 graph, 2 plain
};
constexpr int kSlots = 16;  // runs whose timings are kept

struct wmi_batch {
    wmi_store *st = nullptr;
    size_t dev_cap = 0, host_cap = 0;  // allocated sizes of dev and host
    uint64_t count = 0;
    hipStream_t stream = nullptr;
    wmi_params params{};
    // device buffer and its layout
    char *dev = nullptr;
    size_t dev_bytes = 0;
    // pinned host buffer: descriptors followed by results
    char *host = nullptr;
    size_t host_bytes = 0;
    size_t desc_bytes = 0;  // uploaded prefix
    LaunchArgs args{};
    EntropyArgs eargs{};   // the entropy pass, when eargs.n_query > 0
    // runs of queries (wmi_submit_ranges): expanded into descriptors on the
    // device at every run
    const RangeDesc *d_rd = nullptr;
    uint32_t n_rd = 0;
    WinDesc *d_win = nullptr;
    QDesc *d_qd = nullptr;
    Item *d_queue = nullptr;
    size_t res_bytes = 0;  // results, error word, entropies (in the pinned host buffer)
    uint32_t grid = 0;
    std::vector<uint32_t> win_first_item;  // plain form: first item of each window
    std::vector<int32_t> win_prep;         // plain form: prep-list entry of a split window, or -1
    Result *h_res = nullptr;  // written by the kernels straight into pinned host memory
    const double *h_hres = nullptr;  // entropies in the host buffer, or null
    RunEvents slot[kSlots];
    hipEvent_t ev_end = nullptr;  // recorded after the completion callback of the latest run
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint32_t> series_used;
    wmi_batch_stats stats{};
    // run bookkeeping, guarded by the store mutex: runs may be pipelined on a
    // stream; budget and series pins are held while any run is pending
    uint64_t runs_enq = 0;
    uint64_t runs_done = 0;
    bool held = false;
    bool enqueue_failed = false;
};

namespace {

constexpr size_t kSpareBytes = size_t(256) << 20;  // parked buffers kept per kind
constexpr size_t kSpareCount = 8;

// A parked buffer of at least `bytes` (the smallest that fits, if it is not
// more than four times too large), else a new allocation.
hipError_t take_buffer(wmi_store *st, bool device, size_t bytes, char **out, size_t *cap)
{
    {
        std::lock_guard<std::mutex> lk(st->mu);
        auto &v = device ? st->spare_dev : st->spare_host;
        size_t best = v.size();
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].bytes >= bytes && v[i].bytes <= 4 * bytes + 4096 && (best == v.size() || v[i].bytes < v[best].bytes))
                best = i;
        if (best < v.size()) {
            *out = v[best].p;
            *cap = v[best].bytes;
            (device ? st->spare_dev_bytes : st->spare_host_bytes) -= v[best].bytes;
            v.erase(v.begin() + (long)best);
            return hipSuccess;
        }
    }
    *cap = bytes;
    void *p = nullptr;
    hipError_t e = device ? hipMalloc(&p, bytes) : hipHostMalloc(&p, bytes, hipHostMallocDefault);
    *out = static_cast<char *>(p);
    return e;
}

// Keep a buffer for reuse while the parked total stays small, else free it.
void park_buffer(wmi_store *st, bool device, char *p, size_t cap)
{
    if (!p)
        return;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        auto &v = device ? st->spare_dev : st->spare_host;
        size_t &tot = device ? st->spare_dev_bytes : st->spare_host_bytes;
        if (v.size() < kSpareCount && tot + cap <= kSpareBytes) {
            v.push_back(wmi_store::Spare{p, cap});
            tot += cap;
            return;
        }
    }
    if (device)
        (void)hipFree(p);
    else
        (void)hipHostFree(p);
}

bool value_on_grid(float v)
{
    double s = (double)v * 4096.0;
    return std::isfinite(s) && s == std::nearbyint(s) && std::fabs(s) <= 8388607.0;
}

// Take the budget and series pins for a pending run (store mutex held).
void hold_locked(wmi_batch *b)
{
    wmi_store *st = b->st;
    if (b->held)
        return;
    for (uint32_t id : b->series_used)
        st->series[id].busy++;
    st->inflight += b->dev_bytes;
    b->held = true;
}

// Give them back once no run is pending (store mutex held).
void release_locked(wmi_batch *b)
{
    wmi_store *st = b->st;
    if (!b->held)
        return;
    for (uint32_t id : b->series_used)
        if (id < st->series.size() && st->series[id].busy)
            st->series[id].busy--;
    st->inflight -= b->dev_bytes;
    b->held = false;
    st->cv.notify_all();
}

int enqueue_work(wmi_batch *b, hipStream_t s, const RunEvents *ev)
{
    wmi_store *st = b->st;
    const LaunchArgs &a = b->args;
    if (b->desc_bytes)
        HIPCHK(st, hipMemcpyAsync(b->dev, b->host, b->desc_bytes, hipMemcpyHostToDevice, s));
    if (b->n_rd)
        HIPCHK(st, launch_expand_ranges(b->d_rd, b->n_rd, (uint32_t)b->count, b->d_win, b->d_qd, b->d_queue, s));
    HIPCHK(st, launch_clear(a, s));
    if (ev)
        HIPCHK(st, hipEventRecord(ev->p0, s));
    // window entropies first: the noise thresholds of tau_normalize 2 need them
    HIPCHK(st, launch_entropy(b->eargs, s));
    if (b->params.flags & WMI_SUBMIT_PLAIN) {
        // baseline form: every window is its own prep launch and main launch
        for (uint32_t w = 0; w < a.n_win; ++w) {
            LaunchArgs aw = a;
            if (b->win_prep[w] >= 0) {
                aw.win_begin = (uint32_t)b->win_prep[w];
                HIPCHK(st, launch_prep(aw, 1, s));
            }
            aw.item_begin = b->win_first_item[w];
            aw.n_items = b->win_first_item[w + 1] - b->win_first_item[w];
            aw.persistent = 0;
            HIPCHK(st, launch_main(aw, aw.n_items, s));
        }
        if (ev) {
            HIPCHK(st, hipEventRecord(ev->m0, s));
            HIPCHK(st, hipEventRecord(ev->m1, s));
        }
    } else {
        // prep items run inside the main kernel, at the head of its queue
        if (ev)
            HIPCHK(st, hipEventRecord(ev->m0, s));
        HIPCHK(st, launch_main(a, b->grid, s));
        if (ev)
            HIPCHK(st, hipEventRecord(ev->m1, s));
    }
    // the results are already in host memory: the kernels wrote them there
    return WMI_OK;
}

// Runs on a HIP runtime thread once everything enqueued before it on the
// stream has finished; the last pending run releases budget and pins.
void on_run_complete(void *user)
{
    wmi_batch *b = static_cast<wmi_batch *>(user);
    std::lock_guard<std::mutex> lk(b->st->mu);
    b->runs_done++;
    if (b->runs_done == b->runs_enq)
        release_locked(b);
}

int create_slot(wmi_store *st, RunEvents &e)
{
    if (e.s0)
        return WMI_OK;
    for (hipEvent_t *p : {&e.s0, &e.p0, &e.m0, &e.m1, &e.s1})
        HIPCHK(st, hipEventCreate(p));
    return WMI_OK;
}

// Enqueue one run.  mode: 0 direct with per-kernel events, 1 graph launch.
int run_batch(wmi_batch *b, hipStream_t s, int mode)
{
    wmi_store *st = b->st;
    uint64_t run;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        for (uint32_t id : b->series_used)
            if (id >= st->series.size() || !st->series[id].live)
                return fail(WMI_ESTATE, "series %u of the batch was removed", id);
        hold_locked(b);
        run = b->runs_enq++;
    }
    RunEvents &ev = b->slot[run % kSlots];
    int rc = create_slot(st, ev);
    if (rc == WMI_OK) {
        ev.mode = (b->params.flags & WMI_SUBMIT_PLAIN) ? 2 : mode;
        hipError_t e = hipEventRecord(ev.s0, s);
        if (e != hipSuccess)
            rc = poison(st, e, "hipEventRecord");
        else if (mode == 1)
            rc = (e = hipGraphLaunch(b->graph_exec, s)) == hipSuccess ? WMI_OK : poison(st, e, "hipGraphLaunch");
        else
            rc = enqueue_work(b, s, &ev);
        if (rc == WMI_OK && (e = hipEventRecord(ev.s1, s)) != hipSuccess)
            rc = poison(st, e, "hipEventRecord");
        if (rc == WMI_OK && (e = hipLaunchHostFunc(s, on_run_complete, b)) != hipSuccess)
            rc = poison(st, e, "hipLaunchHostFunc");
        if (rc == WMI_OK && (e = hipEventRecord(b->ev_end, s)) != hipSuccess)
            rc = poison(st, e, "hipEventRecord");
    }
    if (rc != WMI_OK) {
        // the completion callback of this run is not enqueued: undo its count
        std::lock_guard<std::mutex> lk(st->mu);
        b->runs_enq--;
        b->enqueue_failed = true;
        if (b->runs_done == b->runs_enq)
            release_locked(b);
        return rc;
    }
    b->stats.launches = ((b->params.flags & WMI_SUBMIT_PLAIN) ? 1 + 2ull * b->args.n_win : 3) +
                        (b->eargs.n_query ? 1 : 0) + (b->n_rd ? 1 : 0);
    return WMI_OK;
}

bool runs_pending(wmi_batch *b)
{
    std::lock_guard<std::mutex> lk(b->st->mu);
    return b->runs_done != b->runs_enq;
}

// Wait (or poll) until every enqueued run of the batch has completed.
int finish_if_done(wmi_batch *b, bool block, int64_t timeout_us)
{
    wmi_store *st = b->st;
    auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        if (!runs_pending(b))
            break;
        hipError_t e = hipEventQuery(b->ev_end);
        if (e != hipSuccess && e != hipErrorNotReady)
            return poison(st, e, "hipEventQuery");
        {
            std::lock_guard<std::mutex> lk(st->mu);
            if (st->poisoned)
                return fail(WMI_EHIP, "store poisoned: %s", st->poison_msg.c_str());
        }
        if (!block)
            return WMI_ETIMEDOUT;
        if (timeout_us >= 0) {
            auto el = std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0);
            if (el.count() >= timeout_us)
                return fail(WMI_ETIMEDOUT, "batch not finished after %lld us", (long long)timeout_us);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (b->runs_enq) {
        const RunEvents &ev = b->slot[(b->runs_enq - 1) % kSlots];
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.s0, ev.s1) == hipSuccess)
            b->stats.device_ms = ms;
        uint32_t err = 0;
        std::memcpy(&err, reinterpret_cast<const char *>(b->h_res) + b->count * sizeof(Result), sizeof err);
        if (err)
            return fail(WMI_EHIP, "device reported internal error 0x%x (1: a dependency wait gave up; 2: an item the kernel variant does not run)", err);
    }
    return WMI_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

int wmi_version(void) { return (WMI_VERSION_MAJOR << 16) | WMI_VERSION_MINOR; }

const char *wmi_last_error(void) { return g_err.c_str(); }

int wmi_psi_table(uint32_t n, double *host_out)
{
    if (!host_out || n < 1 || n > (uint32_t)kPsiMax)
        return fail(WMI_EINVAL, "wmi_psi_table: n must be in 1..%d", kPsiMax);
    std::vector<double> d;
    std::vector<long long> f;
    build_psi_tables(kPsiMax, d, f);
    for (uint32_t i = 0; i < n; ++i)
        host_out[i] = d[i + 1];
    return WMI_OK;
}

int wmi_store_create(const wmi_store_desc *desc, wmi_store **out)
{
    if (!desc || !out)
        return fail(WMI_EINVAL, "wmi_store_create: null argument");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(WMI_EHIP, "wmi_store_create: no HIP device available");
    if (desc->device < 0 || desc->device >= ndev)
        return fail(WMI_EINVAL, "wmi_store_create: device %d out of range (%d devices)", desc->device, ndev);
    if (desc->flags & ~WMI_STORE_STRICT_GRID)
        return fail(WMI_EINVAL, "wmi_store_create: unknown flags 0x%x", desc->flags);
    DeviceGuard g(desc->device);
    if (!g.ok)
        return fail(WMI_EHIP, "wmi_store_create: hipSetDevice(%d) failed", desc->device);
    wmi_store *st = new wmi_store();
    st->device = desc->device;
    st->flags = desc->flags;
    st->budget = desc->hbm_budget_bytes ? desc->hbm_budget_bytes : kDefaultBudget;
    hipError_t e = hipStreamCreateWithFlags(&st->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&st->capture_stream, hipStreamNonBlocking);
    hipDeviceProp_t prop;
    if (e == hipSuccess)
        e = hipGetDeviceProperties(&prop, st->device);
    if (e == hipSuccess)
        st->cu_count = prop.multiProcessorCount;
    std::vector<double> pd;
    std::vector<long long> pf;
    build_psi_tables(kPsiMax, pd, pf);
    if (e == hipSuccess)
        e = hipMalloc(&st->psi_d, pd.size() * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(&st->psi_fix, pf.size() * sizeof(long long));
    if (e == hipSuccess)
        e = hipMemcpy(st->psi_d, pd.data(), pd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(st->psi_fix, pf.data(), pf.size() * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = noalloc_scratch(st->device, &st->scratch);
    if (e != hipSuccess) {
        int rc = fail(WMI_EHIP, "wmi_store_create: %s", hipGetErrorString(e));
        if (st->psi_d) (void)hipFree(st->psi_d);
        if (st->psi_fix) (void)hipFree(st->psi_fix);
        if (st->stream) (void)hipStreamDestroy(st->stream);
        if (st->capture_stream) (void)hipStreamDestroy(st->capture_stream);
        delete st;
        return rc;
    }
    *out = st;
    return WMI_OK;
}

int wmi_batch_destroy(wmi_batch *b);

int wmi_store_set_tuning(wmi_store *st, const wmi_tuning *t)
{
    if (!st)
        return fail(WMI_EINVAL, "wmi_store_set_tuning: null store");
    Tuning v = default_tuning();
    if (t) {
        std::memcpy(&v, t, sizeof v);
        for (int b = 0; b < 5; ++b) {
            if (v.local_windows[b] < 1 || v.local_windows[b] > (uint32_t)kLocalWindows)
                return fail(WMI_EINVAL, "wmi_store_set_tuning: local_windows[%d] = %u outside 1..%d", b,
                            v.local_windows[b], kLocalWindows);
            if (v.triples[b] < 1 || v.triples[b] > (uint32_t)kTripleMax)
                return fail(WMI_EINVAL, "wmi_store_set_tuning: triples[%d] = %u outside 1..%d", b, v.triples[b],
                            kTripleMax);
        }
        for (int b = 0; b < 3; ++b) {
            if (v.sweep_windows[b] < 1 || v.sweep_windows[b] > 255)
                return fail(WMI_EINVAL, "wmi_store_set_tuning: sweep_windows[%d] = %u outside 1..255", b,
                            v.sweep_windows[b]);
            if (v.stragglers[b] > 128)
                return fail(WMI_EINVAL, "wmi_store_set_tuning: stragglers[%d] = %u above 128", b, v.stragglers[b]);
        }
    }
    std::lock_guard<std::mutex> lk(st->mu);
    st->tune = v;
    return WMI_OK;
}

int wmi_store_get_tuning(wmi_store *st, wmi_tuning *out)
{
    if (!st || !out)
        return fail(WMI_EINVAL, "wmi_store_get_tuning: null argument");
    std::lock_guard<std::mutex> lk(st->mu);
    std::memcpy(out, &st->tune, sizeof *out);
    return WMI_OK;
}

int wmi_store_destroy(wmi_store *st)
{
    if (!st)
        return fail(WMI_EINVAL, "wmi_store_destroy: null store");
    DeviceGuard g(st->device);
    std::vector<wmi_batch *> bs;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        bs.assign(st->batches.begin(), st->batches.end());
    }
    for (wmi_batch *b : bs)
        wmi_batch_destroy(b);
    std::vector<wmi_server *> ss;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        ss.assign(st->servers.begin(), st->servers.end());
    }
    for (wmi_server *sv : ss)
        wmi_server_destroy(sv);
    (void)hipStreamSynchronize(st->stream);
    for (Series &s : st->series)
        if (s.live && s.owned)
            (void)hipFree((void *)s.d);
    for (const wmi_store::Spare &sp : st->spare_dev)
        (void)hipFree(sp.p);
    for (const wmi_store::Spare &sp : st->spare_host)
        (void)hipHostFree(sp.p);
    (void)hipFree(st->psi_d);
    (void)hipFree(st->psi_fix);
    (void)hipStreamDestroy(st->stream);
    (void)hipStreamDestroy(st->capture_stream);
    delete st;
    return WMI_OK;
}

static int add_series_entry(wmi_store *st, const float *d, uint64_t n, bool owned, bool offgrid, uint32_t *id)
{
    std::lock_guard<std::mutex> lk(st->mu);
    Series s;
    s.d = d;
    s.n = n;
    s.owned = owned;
    s.live = true;
    s.offgrid = offgrid;
    st->series.push_back(s);
    *id = (uint32_t)(st->series.size() - 1);
    return WMI_OK;
}

int wmi_series_add(wmi_store *st, const float *host_values, uint64_t n, uint32_t *id)
{
    if (!st || !host_values || !id)
        return fail(WMI_EINVAL, "wmi_series_add: null argument");
    if (n == 0)
        return fail(WMI_EINVAL, "wmi_series_add: empty series");
    if (int rc = check_poison(st))
        return rc;
    bool off = false;
    for (uint64_t i = 0; i < n; ++i) {
        float v = host_values[i];
        if (!std::isfinite(v))
            return fail(WMI_EINVAL, "wmi_series_add: value %llu is not finite", (unsigned long long)i);
        if (!off && !value_on_grid(v))
            off = true;
    }
    if (off && (st->flags & WMI_STORE_STRICT_GRID))
        return fail(WMI_EINVAL, "wmi_series_add: values off the 2^-12 grid (strict store)");
    DeviceGuard g(st->device);
    float *d = nullptr;
    HIPCHK(st, hipMalloc(&d, n * sizeof(float)));
    hipError_t e = hipMemcpy(d, host_values, n * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return poison(st, e, "hipMemcpy(series)");
    }
    return add_series_entry(st, d, n, true, off, id);
}

int wmi_series_add_device(wmi_store *st, const float *d_values, uint64_t n, void *stream, uint32_t *id)
{
    if (!st || !d_values || !id)
        return fail(WMI_EINVAL, "wmi_series_add_device: null argument");
    if (n == 0)
        return fail(WMI_EINVAL, "wmi_series_add_device: empty series");
    if (int rc = check_poison(st))
        return rc;
    DeviceGuard g(st->device);
    hipStream_t s = stream ? (hipStream_t)stream : st->stream;
    unsigned long long *bad = nullptr;
    HIPCHK(st, hipMalloc(&bad, 2 * sizeof(unsigned long long)));
    unsigned long long hbad[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(bad, hbad, sizeof hbad, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_validate(d_values, n, bad, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(bad);
    if (e != hipSuccess)
        return poison(st, e, "validate series");
    if (hbad[0])
        return fail(WMI_EINVAL, "wmi_series_add_device: %llu values are not finite", hbad[0]);
    if (hbad[1] && (st->flags & WMI_STORE_STRICT_GRID))
        return fail(WMI_EINVAL, "wmi_series_add_device: %llu values off the 2^-12 grid (strict store)", hbad[1]);
    return add_series_entry(st, d_values, n, false, hbad[1] != 0, id);
}

int wmi_series_remove(wmi_store *st, uint32_t id)
{
    if (!st)
        return fail(WMI_EINVAL, "wmi_series_remove: null store");
    const float *to_free = nullptr;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        if (id >= st->series.size() || !st->series[id].live)
            return fail(WMI_EINVAL, "wmi_series_remove: unknown series %u", id);
        if (st->series[id].busy)
            return fail(WMI_EBUSY, "wmi_series_remove: series %u is read by %u unfinished batches", id,
                        st->series[id].busy);
        if (st->series[id].owned)
            to_free = st->series[id].d;
        st->series[id].live = false;
        st->series[id].d = nullptr;
    }
    if (to_free) {
        DeviceGuard g(st->device);
        HIPCHK(st, hipFree((void *)to_free));
    }
    return WMI_OK;
}

int wmi_series_length(wmi_store *st, uint32_t id, uint64_t *n)
{
    if (!st || !n)
        return fail(WMI_EINVAL, "wmi_series_length: null argument");
    std::lock_guard<std::mutex> lk(st->mu);
    if (id >= st->series.size() || !st->series[id].live)
        return fail(WMI_EINVAL, "wmi_series_length: unknown series %u", id);
    *n = st->series[id].n;
    return WMI_OK;
}

static int validate_params(const wmi_params *p)
{
    if (p->k < 1 || p->k > WMI_MAX_K)
        return fail(WMI_EINVAL, "k = %u outside 1..%d", p->k, WMI_MAX_K);
    if (p->estimator > 1)
        return fail(WMI_EINVAL, "estimator %u unknown (0 or 1)", p->estimator);
    if (p->tau_normalize > 2)
        return fail(WMI_EINVAL, "tau_normalize must be 0, 1 or 2");
    if (p->flags & ~(WMI_SUBMIT_NONBLOCKING | WMI_SUBMIT_PLAIN | WMI_SUBMIT_NO_REUSE | WMI_SUBMIT_ENTROPY))
        return fail(WMI_EINVAL, "unknown submit flags 0x%x", p->flags);
    if (!std::isfinite(p->tau))
        return fail(WMI_EINVAL, "tau must be finite");
    return WMI_OK;
}

// window list of one query: (start, m) for base, extension, union
static int query_windows(const wmi_query &q, const std::vector<Series> &ser, uint64_t idx, uint64_t st[3],
                         uint32_t m[3], uint32_t *nwin)
{
    if (q.reserved)
        return fail(WMI_EINVAL, "query %llu: reserved field must be 0", (unsigned long long)idx);
    if (q.a >= ser.size() || !ser[q.a].live || q.b >= ser.size() || !ser[q.b].live)
        return fail(WMI_EINVAL, "query %llu: unknown series id (%u, %u)", (unsigned long long)idx, q.a, q.b);
    const uint64_t n = std::min(ser[q.a].n, ser[q.b].n);
    if (q.len == 0)
        return fail(WMI_EINVAL, "query %llu: empty window", (unsigned long long)idx);
    if (q.ext_side == 0) {
        if (q.len > (uint32_t)WMI_MAX_WINDOW)
            return fail(WMI_EINVAL, "query %llu: window of %u points exceeds %d", (unsigned long long)idx, q.len,
                        WMI_MAX_WINDOW);
        if (q.start > n || q.len > n - q.start)
            return fail(WMI_EINVAL, "query %llu: window [%llu, +%u) outside series of %llu points",
                        (unsigned long long)idx, (unsigned long long)q.start, q.len, (unsigned long long)n);
        st[0] = q.start;
        m[0] = q.len;
        *nwin = 1;
        return WMI_OK;
    }
    if (q.ext_side != 1 && q.ext_side != -1)
        return fail(WMI_EINVAL, "query %llu: ext_side must be -1, 0 or +1", (unsigned long long)idx);
    if (q.ext_len == 0)
        return fail(WMI_EINVAL, "query %llu: empty extension", (unsigned long long)idx);
    if ((uint64_t)q.len + q.ext_len > (uint64_t)WMI_MAX_WINDOW)
        return fail(WMI_EINVAL, "query %llu: union of %llu points exceeds %d", (unsigned long long)idx,
                    (unsigned long long)q.len + q.ext_len, WMI_MAX_WINDOW);
    uint64_t lo = q.ext_side > 0 ? q.start : q.start - q.ext_len;
    if (q.ext_side < 0 && q.start < q.ext_len)
        return fail(WMI_EINVAL, "query %llu: left extension before the series start", (unsigned long long)idx);
    uint64_t total = (uint64_t)q.len + q.ext_len;
    if (lo > n || total > n - lo)
        return fail(WMI_EINVAL, "query %llu: triple outside series of %llu points", (unsigned long long)idx,
                    (unsigned long long)n);
    st[0] = q.start;
    m[0] = q.len;
    st[1] = q.ext_side > 0 ? q.start + q.len : q.start - q.ext_len;
    m[1] = q.ext_len;
    st[2] = lo;
    m[2] = (uint32_t)total;
    *nwin = 3;
    return WMI_OK;
}

}  // extern "C"

namespace {

// A batch's validated queries, their windows, its work list and the layout
// of its device buffer (offsets in bytes, 256-byte aligned).
struct BatchBuild {
    std::vector<Series> ser;
    std::vector<uint64_t> wstart;  // windows in query order (a triple: base, extension, union)
    std::vector<uint32_t> wm, wquery, used;
    std::vector<uint64_t> wx, wy;  // address of each window's first x and y value
    std::vector<RangeDesc> rd;     // runs of queries (wmi_submit_ranges): the descriptor prefix
    bool ranged = false;
    bool local_only = false;       // local and triple items only: the lighter kernel variant
    Tuning tune;
    uint64_t pairs = 0, n_win = 0, n_items = 0, n_prep = 0;
    bool plain = false;
    Plan plan;
    std::vector<Item> queue;
    size_t o_win = 0, o_item = 0, o_qd = 0, o_prep = 0, desc_bytes = 0, o_sorted = 0, o_acc = 0, o_wdone = 0,
           o_qdone = 0, o_counter = 0, o_wmi = 0, o_wflags = 0, o_ready = 0, o_res = 0, o_hres = 0,
           res_bytes = 0, dev_bytes = 0;
};

void layout_batch(BatchBuild &B, uint64_t count, const wmi_params *p);

int build_batch(wmi_store *st, const wmi_query *qs, uint64_t count, const wmi_params *p, BatchBuild &B)
{
    {
        std::lock_guard<std::mutex> lk(st->mu);
        B.ser = st->series;
        B.tune = st->tune;
    }
    uint64_t nw_all = 0;
    for (uint64_t t = 0; t < count; ++t)
        nw_all += qs[t].ext_side ? 3u : 1u;
    B.wstart.reserve(nw_all);
    B.wm.reserve(nw_all);
    B.wquery.reserve(nw_all);
    B.wx.reserve(nw_all);
    B.wy.reserve(nw_all);
    B.used.reserve(2 * count);
    for (uint64_t t = 0; t < count; ++t) {
        uint64_t s3[3];
        uint32_t m3[3], nw = 0;
        if (int rc = query_windows(qs[t], B.ser, t, s3, m3, &nw))
            return rc;
        for (uint32_t r = 0; r < nw; ++r) {
            B.wstart.push_back(s3[r]);
            B.wx.push_back((uint64_t)(uintptr_t)(B.ser[qs[t].a].d + s3[r]));
            B.wy.push_back((uint64_t)(uintptr_t)(B.ser[qs[t].b].d + s3[r]));
            B.wm.push_back(m3[r]);
            B.wquery.push_back((uint32_t)t);
            B.pairs += (uint64_t)m3[r] * (m3[r] - 1);
        }
        B.used.push_back(qs[t].a);
        B.used.push_back(qs[t].b);
    }
    B.n_win = B.wm.size();
    if (B.n_win > 0x7FFFFFF0ull)
        return fail(WMI_ENOMEM, "wmi_submit: batch too large for one launch (%llu windows)",
                    (unsigned long long)B.n_win);
    std::sort(B.used.begin(), B.used.end());
    B.used.erase(std::unique(B.used.begin(), B.used.end()), B.used.end());

    // ---- work items ---------------------------------------------------------
    B.plain = (p->flags & WMI_SUBMIT_PLAIN) != 0;
    plan_items(B.wm, B.wquery, count, B.plain, B.plan, !(p->flags & WMI_SUBMIT_NO_REUSE), &B.wx, &B.wy, &B.tune);
    if (!B.plain) {
        plan_queue(B.plan, B.wm, B.queue);
        // the lighter variant gains occupancy for k <= 5 only
        B.local_only = p->k <= 5 && std::all_of(B.queue.begin(), B.queue.end(), [](const Item &it) {
            const uint32_t top = it.info & 0xF0000000u;
            return top == kItemLocal || top == kItemTriple;
        });
    }
    B.n_items = B.plain ? B.plan.items.size() : B.queue.size();
    B.n_prep = B.plan.prep_list.size();
    if (B.plan.split_pts > 0xFFFFFFF0ull)
        return fail(WMI_ENOMEM, "wmi_submit: batch too large for one launch (%llu points in large windows)",
                    (unsigned long long)B.plan.split_pts);

    layout_batch(B, count, p);
    return WMI_OK;
}

// Offsets of the batch's device buffer.  The uploaded prefix [0, desc_bytes)
// holds the window, item, query and prep-list descriptors, or for runs of
// queries only the runs (their descriptors are written on the device, right
// after them).
void layout_batch(BatchBuild &B, uint64_t count, const wmi_params *p)
{
    const size_t A = 256;
    B.o_win = B.ranged ? align_up(B.rd.size() * sizeof(RangeDesc), A) : 0;
    B.o_item = align_up(B.o_win + B.n_win * sizeof(WinDesc), A);
    B.o_qd = align_up(B.o_item + B.n_items * sizeof(Item), A);
    B.o_prep = align_up(B.o_qd + count * sizeof(QDesc), A);
    const size_t desc_end = align_up(B.o_prep + B.n_prep * sizeof(uint32_t), A);
    B.desc_bytes = B.ranged ? B.o_win : desc_end;
    B.o_sorted = desc_end;
    B.o_acc = align_up(B.o_sorted + (size_t)kSortedWords * B.plan.split_pts * sizeof(int32_t), A);
    B.o_wdone = align_up(B.o_acc + B.n_win * sizeof(unsigned long long), A);
    B.o_qdone = align_up(B.o_wdone + B.n_win * sizeof(uint32_t), A);
    B.o_counter = align_up(B.o_qdone + count * sizeof(uint32_t), A);
    B.o_wmi = align_up(B.o_counter + sizeof(uint32_t), A);
    B.o_wflags = align_up(B.o_wmi + B.n_win * sizeof(double), A);
    B.o_ready = align_up(B.o_wflags + B.n_win * sizeof(uint32_t), A);
    B.o_res = align_up(B.o_ready + B.n_win * sizeof(uint32_t), A);
    // results, the error word and the entropies are downloaded together
    B.res_bytes = count * sizeof(Result) + sizeof(uint32_t);
    if (p->flags & WMI_SUBMIT_ENTROPY) {
        B.o_hres = align_up(B.o_res + B.res_bytes, 8);
        B.res_bytes = B.o_hres - B.o_res + 3 * count * sizeof(double);
    }
    B.dev_bytes = align_up(B.o_res + B.res_bytes, A);
}

// Runs of queries: validated (the first and the last query of each run; the
// others lie between them), planned per run (plan_ranges) and laid out.
int build_ranges(wmi_store *st, const wmi_range *rg, uint64_t n_ranges, const wmi_params *p, BatchBuild &B,
                 uint64_t *count)
{
    {
        std::lock_guard<std::mutex> lk(st->mu);
        B.ser = st->series;
        B.tune = st->tune;
    }
    B.ranged = true;
    uint64_t total = 0;
    for (uint64_t r = 0; r < n_ranges; ++r) {
        const wmi_range &g = rg[r];
        if (g.reserved)
            return fail(WMI_EINVAL, "range %llu: reserved field must be 0", (unsigned long long)r);
        if (g.count == 0)
            continue;
        if (g.count > 1 && g.stride == 0)
            return fail(WMI_EINVAL, "range %llu: stride 0 with %u queries", (unsigned long long)r, g.count);
        const uint64_t span = (uint64_t)(g.count - 1) * g.stride;
        if (g.start > ~0ull - span)
            return fail(WMI_EINVAL, "range %llu: start overflows", (unsigned long long)r);
        wmi_query q{};
        q.a = g.a;
        q.b = g.b;
        q.len = g.len;
        q.ext_len = g.ext_len;
        q.ext_side = g.ext_side;
        const uint64_t ends[2] = {0, span};
        for (uint64_t i : ends) {
            q.start = g.start + i;
            uint64_t s3[3];
            uint32_t m3[3], nw = 0;
            if (int rc = query_windows(q, B.ser, total + (i ? g.count - 1 : 0), s3, m3, &nw))
                return rc;
        }
        RangeDesc R{};
        R.x = B.ser[g.a].d;
        R.y = B.ser[g.b].d;
        R.start = g.start;
        R.stride = g.stride;
        R.count = g.count;
        R.m = g.len;
        R.side = g.ext_side;
        R.e = g.ext_side ? g.ext_len : 0u;
        R.tau_eff = p->tau_normalize == 1 ? p->tau * std::log((double)g.ext_len) : p->tau;
        B.rd.push_back(R);
        const uint64_t u = (uint64_t)R.m + R.e;
        B.pairs += (uint64_t)g.count * (R.side ? (uint64_t)R.m * (R.m - 1) + (uint64_t)R.e * (R.e - 1) + u * (u - 1)
                                               : (uint64_t)R.m * (R.m - 1));
        B.used.push_back(g.a);
        B.used.push_back(g.b);
        total += g.count;
        if (total > 0xFFFFFFF0ull)
            return fail(WMI_EINVAL, "wmi_submit_ranges: more than 2^32 - 16 queries");
    }
    std::sort(B.used.begin(), B.used.end());
    B.used.erase(std::unique(B.used.begin(), B.used.end()), B.used.end());
    if (B.rd.size() > 0xFFFFFFF0ull)
        return fail(WMI_EINVAL, "wmi_submit_ranges: too many runs");
    const bool fuse = !(p->flags & WMI_SUBMIT_NO_REUSE);
    B.n_items = plan_ranges(B.rd.data(), (uint32_t)B.rd.size(), fuse, &B.tune, &B.n_win, &B.plan.split_pts);
    if (B.n_win > 0x7FFFFFF0ull || B.n_items > 0xFFFFFFF0ull)
        return fail(WMI_ENOMEM, "wmi_submit_ranges: batch too large for one launch (%llu windows)",
                    (unsigned long long)B.n_win);
    if (B.plan.split_pts > 0xFFFFFFF0ull)
        return fail(WMI_ENOMEM, "wmi_submit_ranges: batch too large for one launch (%llu points in large windows)",
                    (unsigned long long)B.plan.split_pts);
    B.n_prep = 0;
    B.plain = false;
    B.local_only = p->k <= 5 && std::all_of(B.rd.begin(), B.rd.end(),
                               [](const RangeDesc &R) { return R.kind == kRangeLocal || R.kind == kRangeTriple; });
    layout_batch(B, total, p);
    *count = total;
    return WMI_OK;
}

// Window, item, query and prep-list descriptors into the host image of the
// descriptor prefix [0, desc_bytes) of the device buffer.
void write_descriptors(const BatchBuild &B, const wmi_query *qs, uint64_t count, const wmi_params *p, char *host)
{
    WinDesc *hw = reinterpret_cast<WinDesc *>(host + B.o_win);
    Item *hi = reinterpret_cast<Item *>(host + B.o_item);
    QDesc *hq = reinterpret_cast<QDesc *>(host + B.o_qd);
    uint32_t *hp = reinterpret_cast<uint32_t *>(host + B.o_prep);
    for (uint64_t i = 0; i < B.n_win; ++i) {
        const uint32_t t = B.wquery[i];
        WinDesc &d = hw[i];
        d.x = B.ser[qs[t].a].d + B.wstart[i];
        d.y = B.ser[qs[t].b].d + B.wstart[i];
        d.m = B.wm[i];
        d.query = t;
        d.sorted_off = B.plan.wsorted[i];
        d.n_items = B.plan.wnitems[i];
    }
    for (uint64_t t = 0, i = 0; t < count; ++t) {
        hq[t].win0 = (uint32_t)i;
        uint32_t nw = 0;
        while (i < B.n_win && B.wquery[i] == (uint32_t)t) {
            ++nw;
            ++i;
        }
        hq[t].nwin = nw;
        // tau_normalize 2: the entropy pass writes tau * H(w_d) here
        hq[t].tau_eff = p->tau_normalize == 1 ? p->tau * std::log((double)qs[t].ext_len) : p->tau;
    }
    std::copy(B.plan.prep_list.begin(), B.plan.prep_list.end(), hp);
    if (B.plain)
        std::copy(B.plan.items.begin(), B.plan.items.end(), hi);
    else
        std::copy(B.queue.begin(), B.queue.end(), hi);
}

// Launch arguments over a device buffer laid out as B (results to res, the
// error word to err).
void set_args(const BatchBuild &B, const wmi_store *st, const wmi_params *p, uint64_t count, char *dev, Result *res,
              uint32_t *err, LaunchArgs &a)
{
    a = LaunchArgs{};
    a.win = reinterpret_cast<const WinDesc *>(dev + B.o_win);
    a.item = reinterpret_cast<const Item *>(dev + B.o_item);
    a.qd = reinterpret_cast<const QDesc *>(dev + B.o_qd);
    a.sorted = reinterpret_cast<int32_t *>(dev + B.o_sorted);
    a.acc = reinterpret_cast<unsigned long long *>(dev + B.o_acc);
    a.wdone = reinterpret_cast<uint32_t *>(dev + B.o_wdone);
    a.qdone = reinterpret_cast<uint32_t *>(dev + B.o_qdone);
    a.counter = reinterpret_cast<uint32_t *>(dev + B.o_counter);
    a.wmi = reinterpret_cast<double *>(dev + B.o_wmi);
    a.wflags = reinterpret_cast<uint32_t *>(dev + B.o_wflags);
    a.res = res;
    a.err = err;
    a.ready = reinterpret_cast<uint32_t *>(dev + B.o_ready);
    a.psi_d = st->psi_d;
    a.psi_fix = st->psi_fix;
    a.prep_list = reinterpret_cast<const uint32_t *>(dev + B.o_prep);
    a.n_prep = (uint32_t)B.n_prep;
    a.n_win = (uint32_t)B.n_win;
    a.n_items = (uint32_t)B.n_items;
    a.n_query = (uint32_t)count;
    a.item_begin = 0;
    a.k = p->k;
    a.estimator = p->estimator;
    a.persistent = 1;
    a.win_begin = 0;
    for (int i = 0; i < 3; ++i)
        a.strag[i] = B.tune.stragglers[i];
    a.local_only = B.local_only ? 1u : 0u;
}

// The entropy pass over a device buffer laid out as B: all windows' entropies
// into hres when given; the extensions' only (the thresholds) otherwise.  No
// pass (n_query 0) when neither is wanted.
void set_entropy_args(const BatchBuild &B, const wmi_params *p, uint64_t count, char *dev, double *hres,
                      EntropyArgs &e)
{
    e = EntropyArgs{};
    if (!hres && p->tau_normalize != 2)
        return;
    e.win = reinterpret_cast<const WinDesc *>(dev + B.o_win);
    e.qd = reinterpret_cast<QDesc *>(dev + B.o_qd);
    e.hres = hres;
    e.tau = p->tau;
    e.n_query = (uint32_t)count;
    e.set_tau = p->tau_normalize == 2 ? 1u : 0u;
}

}  // namespace

namespace {

// A planned batch (query list qs, or runs in B.rd): budget, buffers,
// descriptors, launch arguments and its first run.
int start_batch(wmi_store *st, BatchBuild &B, const wmi_query *qs, uint64_t count, const wmi_params *p,
                void *stream, const char *who, wmi_batch **out)
{
    const size_t dev_bytes = B.dev_bytes, desc_bytes = B.desc_bytes;
    if (dev_bytes > st->budget)
        return fail(WMI_ENOMEM, "%s: batch needs %zu bytes of device memory, budget is %llu", who, dev_bytes,
                    (unsigned long long)st->budget);
    {
        std::unique_lock<std::mutex> lk(st->mu);
        if (st->inflight + dev_bytes > st->budget) {
            if (p->flags & WMI_SUBMIT_NONBLOCKING)
                return fail(WMI_EBUSY, "%s: %zu bytes do not fit beside %llu in flight (budget %llu)",
                            who, dev_bytes, (unsigned long long)st->inflight, (unsigned long long)st->budget);
            // running batches release their budget from the stream callback
            st->cv.wait(lk, [&] { return st->inflight + dev_bytes <= st->budget; });
        }
        for (uint32_t id : B.used)
            if (id >= st->series.size() || !st->series[id].live)
                return fail(WMI_EINVAL, "%s: series %u removed during submit", who, id);
    }
    wmi_batch *b = new wmi_batch();
    b->st = st;
    b->count = count;
    b->params = *p;
    b->stream = stream ? (hipStream_t)stream : st->stream;
    b->series_used = B.used;
    b->dev_bytes = dev_bytes;
    b->desc_bytes = desc_bytes;
    b->stats.windows = B.n_win;
    b->stats.ordered_pairs = B.pairs;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        hold_locked(b);  // reserve budget and pins until the batch's runs complete
    }

    auto bail = [&](hipError_t e, const char *what) {
        int rc = poison(st, e, what);
        {
            std::lock_guard<std::mutex> lk(st->mu);
            release_locked(b);
        }
        if (b->dev) (void)hipFree(b->dev);
        if (b->host) (void)hipHostFree(b->host);
        if (b->ev_end) (void)hipEventDestroy(b->ev_end);
        delete b;
        return rc;
    };
    hipError_t e = take_buffer(st, true, dev_bytes, &b->dev, &b->dev_cap);
    if (e != hipSuccess)
        return bail(e, "hipMalloc(batch)");
    b->host_bytes = desc_bytes + align_up(B.res_bytes, 256);
    e = take_buffer(st, false, std::max<size_t>(b->host_bytes, 256), &b->host, &b->host_cap);
    if (e != hipSuccess)
        return bail(e, "hipHostMalloc(batch)");
    e = hipEventCreate(&b->ev_end);
    if (e != hipSuccess)
        return bail(e, "hipEventCreate");

    // ---- descriptors and launch arguments ------------------------------------
    if (B.ranged) {
        std::memcpy(b->host, B.rd.data(), B.rd.size() * sizeof(RangeDesc));
        b->d_rd = reinterpret_cast<const RangeDesc *>(b->dev);
        b->n_rd = (uint32_t)B.rd.size();
        b->d_win = reinterpret_cast<WinDesc *>(b->dev + B.o_win);
        b->d_qd = reinterpret_cast<QDesc *>(b->dev + B.o_qd);
        b->d_queue = reinterpret_cast<Item *>(b->dev + B.o_item);
    } else {
        write_descriptors(B, qs, count, p, b->host);
    }
    // results, the error word and the entropies go straight from the kernels
    // into the pinned host buffer (its device address), after the descriptor
    // prefix: no download after a run, so consecutive batches' kernels are
    // not kept apart by copies
    b->h_res = reinterpret_cast<Result *>(b->host + desc_bytes);
    char *host_dev = nullptr;
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&host_dev), b->host, 0);
    if (e != hipSuccess)
        return bail(e, "hipHostGetDevicePointer");
    char *res_dev = host_dev + desc_bytes;
    if (B.plain) {
        b->win_first_item = std::move(B.plan.first_item);
        b->win_prep = std::move(B.plan.wprep);
    }
    LaunchArgs &a = b->args;
    set_args(B, st, p, count, b->dev, reinterpret_cast<Result *>(res_dev),
             reinterpret_cast<uint32_t *>(res_dev + count * sizeof(Result)), a);
    b->res_bytes = B.res_bytes;
    double *d_hres = nullptr;
    if (p->flags & WMI_SUBMIT_ENTROPY) {
        d_hres = reinterpret_cast<double *>(res_dev + (B.o_hres - B.o_res));
        b->h_hres = reinterpret_cast<const double *>(b->host + desc_bytes + (B.o_hres - B.o_res));
    }
    set_entropy_args(B, p, count, b->dev, d_hres, b->eargs);
    int occ = main_occupancy(p->k, B.local_only);
    uint64_t slots = (uint64_t)st->cu_count * (uint64_t)occ;
    b->grid = (uint32_t)std::min<uint64_t>(B.n_items, slots);
    b->stats.items = (uint32_t)B.n_items;
    b->stats.grid = b->grid;
    b->stats.wg_per_cu = (uint32_t)occ;
    b->stats.cus = (uint32_t)st->cu_count;

    {
        std::lock_guard<std::mutex> lk(st->mu);
        st->batches.insert(b);
    }
    int rc = run_batch(b, b->stream, 0);
    if (rc) {
        (void)hipStreamSynchronize(b->stream);
        wmi_batch_destroy(b);
        return rc;
    }
    *out = b;
    return WMI_OK;
}


}  // namespace

extern "C" {

int wmi_submit(wmi_store *st, const wmi_query *qs, uint64_t count, const wmi_params *p, void *stream,
               wmi_batch **out)
{
    if (!st || !p || !out || (count && !qs))
        return fail(WMI_EINVAL, "wmi_submit: null argument");
    *out = nullptr;
    if (int rc = validate_params(p))
        return rc;
    if (count > 0xFFFFFFF0ull)
        return fail(WMI_EINVAL, "wmi_submit: too many queries in one batch");
    if (int rc = check_poison(st))
        return rc;
    DeviceGuard g(st->device);

    BatchBuild B;
    if (int rc = build_batch(st, qs, count, p, B))
        return rc;
    return start_batch(st, B, qs, count, p, stream, "wmi_submit", out);
}

int wmi_submit_ranges(wmi_store *st, const wmi_range *ranges, uint64_t n_ranges, const wmi_params *p, void *stream,
                      wmi_batch **out)
{
    if (!st || !p || !out || (n_ranges && !ranges))
        return fail(WMI_EINVAL, "wmi_submit_ranges: null argument");
    *out = nullptr;
    if (int rc = validate_params(p))
        return rc;
    if (p->flags & WMI_SUBMIT_PLAIN)
        return fail(WMI_EINVAL, "wmi_submit_ranges: no plain form");
    if (int rc = check_poison(st))
        return rc;
    DeviceGuard g(st->device);
    BatchBuild B;
    uint64_t count = 0;
    if (int rc = build_ranges(st, ranges, n_ranges, p, B, &count))
        return rc;
    return start_batch(st, B, nullptr, count, p, stream, "wmi_submit_ranges", out);
}

int wmi_submit_noalloc(wmi_store *st, const wmi_query *qs, uint64_t count, const wmi_params *p, void *stream,
                       wmi_result *d_results)
{
    static_assert(WMI_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "scratch size");
    if (!st || !p || (count && (!qs || !d_results)))
        return fail(WMI_EINVAL, "wmi_submit_noalloc: null argument");
    if (int rc = validate_params(p))
        return rc;
    if (p->flags)
        return fail(WMI_EINVAL, "wmi_submit_noalloc: flags must be 0");  // entropies are not returned here
    if (count > 0xFFFFFFF0ull)
        return fail(WMI_EINVAL, "wmi_submit_noalloc: too many queries in one call");
    if (int rc = check_poison(st))
        return rc;
    if (count == 0)
        return WMI_OK;
    DeviceGuard g(st->device);
    if (!st->scratch)
        return fail(WMI_EHIP, "wmi_submit_noalloc: no scratch address for device %d", st->device);
    BatchBuild B;
    if (int rc = build_batch(st, qs, count, p, B))
        return rc;
    // descriptors, sorted data, counters and estimates, then the error word
    const size_t need = B.o_res + sizeof(uint32_t);
    if (need > kNoAllocScratchBytes)
        return fail(WMI_ENOMEM,
                    "wmi_submit_noalloc: the call needs %zu bytes of scratch, the limit is %zu "
                    "(%llu windows, %llu points in windows above %d points)",
                    need, kNoAllocScratchBytes, (unsigned long long)B.n_win,
                    (unsigned long long)B.plan.split_pts, kLocalSlots);
    // one call at a time per device: every call shares the device's array
    static std::mutex dev_mu[64];
    std::lock_guard<std::mutex> call_lk(dev_mu[st->device & 63]);
    {
        std::lock_guard<std::mutex> lk(st->mu);
        for (uint32_t id : B.used)
            if (id >= st->series.size() || !st->series[id].live)
                return fail(WMI_EINVAL, "wmi_submit_noalloc: series %u removed during the call", id);
        for (uint32_t id : B.used)
            st->series[id].busy++;
    }
    auto unpin = [&]() {
        std::lock_guard<std::mutex> lk(st->mu);
        for (uint32_t id : B.used)
            if (id < st->series.size() && st->series[id].busy)
                st->series[id].busy--;
        st->cv.notify_all();
    };
    std::vector<char> host(B.desc_bytes);
    write_descriptors(B, qs, count, p, host.data());
    char *dev = static_cast<char *>(st->scratch);
    LaunchArgs a;
    set_args(B, st, p, count, dev, reinterpret_cast<Result *>(d_results), reinterpret_cast<uint32_t *>(dev + B.o_res),
             a);
    EntropyArgs ea;
    set_entropy_args(B, p, count, dev, nullptr, ea);
    const uint32_t grid =
        (uint32_t)std::min<uint64_t>(B.n_items, (uint64_t)st->cu_count * (uint64_t)main_occupancy(p->k, B.local_only));
    hipStream_t s = stream ? (hipStream_t)stream : st->stream;
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(dev, host.data(), B.desc_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_clear(a, s);  // counters, sums, flags and the error word start at zero
    if (e == hipSuccess)
        e = launch_entropy(ea, s);
    if (e == hipSuccess)
        e = launch_main(a, grid, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&err, a.err, sizeof err, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    unpin();
    if (e != hipSuccess)
        return poison(st, e, "wmi_submit_noalloc");
    if (err)
        return fail(WMI_EHIP, "device reported internal error 0x%x (1: a dependency wait gave up; 2: an item the kernel variant does not run)", err);
    return WMI_OK;
}

int wmi_wait(wmi_batch *b, int64_t timeout_us)
{
    if (!b)
        return fail(WMI_EINVAL, "wmi_wait: null batch");
    DeviceGuard g(b->st->device);
    return finish_if_done(b, true, timeout_us);
}

int wmi_done(wmi_batch *b)
{
    if (!b)
        return 0;
    DeviceGuard g(b->st->device);
    return finish_if_done(b, false, 0) == WMI_OK ? 1 : 0;
}

int wmi_read(wmi_batch *b, wmi_result *out)
{
    if (!b || (!out && b->count))
        return fail(WMI_EINVAL, "wmi_read: null argument");
    DeviceGuard g(b->st->device);
    if (int rc = finish_if_done(b, true, -1))
        return rc;
    if (b->count)
        std::memcpy(out, b->h_res, b->count * sizeof(Result));
    return WMI_OK;
}

int wmi_read_entropy(wmi_batch *b, double *host_out)
{
    if (!b || (!host_out && b->count))
        return fail(WMI_EINVAL, "wmi_read_entropy: null argument");
    if (!b->h_hres)
        return fail(WMI_ESTATE, "wmi_read_entropy: the batch was submitted without WMI_SUBMIT_ENTROPY");
    DeviceGuard g(b->st->device);
    if (int rc = finish_if_done(b, true, -1))
        return rc;
    if (b->count)
        std::memcpy(host_out, b->h_hres, b->count * 3 * sizeof(double));
    return WMI_OK;
}

int wmi_batch_replay(wmi_batch *b, void *stream, uint32_t flags)
{
    if (!b)
        return fail(WMI_EINVAL, "wmi_batch_replay: null batch");
    if (flags & ~WMI_REPLAY_DIRECT)
        return fail(WMI_EINVAL, "wmi_batch_replay: unknown flags 0x%x", flags);
    wmi_store *st = b->st;
    DeviceGuard g(st->device);
    if (int rc = check_poison(st))
        return rc;
    hipStream_t s = stream ? (hipStream_t)stream : b->stream;
    const bool graph = !(flags & WMI_REPLAY_DIRECT) && !(b->params.flags & WMI_SUBMIT_PLAIN);
    if (graph && !b->graph_exec) {
        HIPCHK(st, hipStreamBeginCapture(st->capture_stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_work(b, st->capture_stream, nullptr);
        hipGraph_t graph_h = nullptr;
        hipError_t e = hipStreamEndCapture(st->capture_stream, &graph_h);
        if (rc)
            return rc;
        if (e != hipSuccess)
            return poison(st, e, "hipStreamEndCapture");
        b->graph = graph_h;
        HIPCHK(st, hipGraphInstantiate(&b->graph_exec, graph_h, nullptr, nullptr, 0));
    }
    return run_batch(b, s, graph ? 1 : 0);
}

int wmi_batch_timing(wmi_batch *b, wmi_timing *out)
{
    if (!b || !out)
        return fail(WMI_EINVAL, "wmi_batch_timing: null argument");
    DeviceGuard g(b->st->device);
    if (int rc = finish_if_done(b, true, -1))
        return rc;
    std::memset(out, 0, sizeof *out);
    const double nan = std::nan("");
    uint64_t n = std::min<uint64_t>(b->runs_enq, kSlots);
    double tot = 0, prep = 0, mainv = 0;
    int mode = -1;
    bool mixed = false;
    for (uint64_t r = b->runs_enq - n; r < b->runs_enq; ++r) {
        const RunEvents &ev = b->slot[r % kSlots];
        float a = 0, p = 0, m = 0;
        HIPCHK(b->st, hipEventElapsedTime(&a, ev.s0, ev.s1));
        tot += a;
        if (ev.mode == 0) {
            HIPCHK(b->st, hipEventElapsedTime(&p, ev.p0, ev.m0));
            HIPCHK(b->st, hipEventElapsedTime(&m, ev.m0, ev.m1));
            prep += p;
            mainv += m;
        }
        if (mode >= 0 && mode != ev.mode)
            mixed = true;
        mode = ev.mode;
    }
    out->runs = (uint32_t)n;
    out->mode = mixed ? -1 : mode;
    out->total_ms = n ? tot / (double)n : nan;
    out->prep_ms = (n && mode == 0 && !mixed) ? prep / (double)n : nan;
    out->main_ms = (n && mode == 0 && !mixed) ? mainv / (double)n : nan;
    return WMI_OK;
}

int wmi_batch_stats_get(wmi_batch *b, wmi_batch_stats *out)
{
    if (!b || !out)
        return fail(WMI_EINVAL, "wmi_batch_stats_get: null argument");
    DeviceGuard g(b->st->device);
    if (int rc = finish_if_done(b, true, -1))
        return rc;
    *out = b->stats;
    return WMI_OK;
}

int wmi_batch_count_evals(wmi_batch *b, uint64_t *evaluated)
{
    if (!b || !evaluated)
        return fail(WMI_EINVAL, "wmi_batch_count_evals: null argument");
    if (b->params.flags & WMI_SUBMIT_PLAIN)
        return fail(WMI_EINVAL, "wmi_batch_count_evals: not available for plain batches");
    wmi_store *st = b->st;
    DeviceGuard g(st->device);
    if (int rc = finish_if_done(b, true, -1))
        return rc;
    *evaluated = 0;
    if (!b->count || !b->grid)
        return WMI_OK;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        for (uint32_t id : b->series_used)
            if (id >= st->series.size() || !st->series[id].live)
                return fail(WMI_ESTATE, "series %u of the batch was removed", id);
        hold_locked(b);
    }
    auto release = [&]() {
        std::lock_guard<std::mutex> lk(st->mu);
        release_locked(b);
    };
    unsigned long long *cnt = nullptr;
    hipError_t e = hipMalloc(&cnt, sizeof(unsigned long long) * b->grid);
    if (e != hipSuccess) {
        release();
        return fail(WMI_EHIP, "wmi_batch_count_evals: hipMalloc of %u counters failed", b->grid);
    }
    LaunchArgs a = b->args;
    a.evals = cnt;
    hipStream_t s = b->stream;
    std::vector<unsigned long long> h(b->grid);
    uint32_t err = 0;
    if ((e = hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * b->grid, s)) == hipSuccess &&
        (e = launch_clear(a, s)) == hipSuccess && (e = launch_main(a, b->grid, s)) == hipSuccess &&
        (e = hipMemcpyAsync(h.data(), cnt, sizeof(unsigned long long) * b->grid, hipMemcpyDeviceToHost, s)) ==
            hipSuccess)
        e = hipStreamSynchronize(s);
    if (e == hipSuccess)  // the error word is in the pinned host buffer
        std::memcpy(&err, reinterpret_cast<const char *>(b->h_res) + b->count * sizeof(Result), sizeof err);
    (void)hipFree(cnt);
    release();
    if (e != hipSuccess)
        return poison(st, e, "wmi_batch_count_evals");
    if (err)
        return fail(WMI_EHIP, "device reported internal error 0x%x (1: a dependency wait gave up; 2: an item the kernel variant does not run)", err);
    uint64_t total = 0;
    for (unsigned long long v : h)
        total += v;
    *evaluated = total;
    return WMI_OK;
}

int wmi_batch_destroy(wmi_batch *b)
{
    if (!b)
        return WMI_OK;
    wmi_store *st = b->st;
    DeviceGuard g(st->device);
    int rc = finish_if_done(b, true, -1);
    if (rc != WMI_OK) {
        // a HIP error left runs pending; wait for the stream before freeing
        (void)hipStreamSynchronize(b->stream);
    }
    {
        std::lock_guard<std::mutex> lk(st->mu);
        release_locked(b);
        st->batches.erase(b);
    }
    if (b->graph_exec)
        (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    for (RunEvents &ev : b->slot)
        for (hipEvent_t e : {ev.s0, ev.p0, ev.m0, ev.m1, ev.s1})
            if (e)
                (void)hipEventDestroy(e);
    if (b->ev_end)
        (void)hipEventDestroy(b->ev_end);
    park_buffer(st, true, b->dev, b->dev_cap);
    park_buffer(st, false, b->host, b->host_cap);
    delete b;
    return WMI_OK;
}

int wmi_debug_window(wmi_store *st, const wmi_query *query, const wmi_params *params, uint32_t *nx, uint32_t *ny,
                     float *ex, float *ey)
{
    if (!st || !query || !params || !nx || !ny || !ex || !ey)
        return fail(WMI_EINVAL, "wmi_debug_window: null argument");
    if (int rc = validate_params(params))
        return rc;
    wmi_query q = *query;
    q.ext_len = 0;
    q.ext_side = 0;
    q.reserved = 0;
    if (q.len <= params->k)
        return fail(WMI_EINVAL, "wmi_debug_window: window of %u points has no estimate for k = %u", q.len,
                    params->k);
    wmi_params p = *params;
    p.flags = 0;
    // run as a one-query batch with the debug pointers set
    DeviceGuard g(st->device);
    uint32_t m = q.len;
    char *dbg = nullptr;
    HIPCHK(st, hipMalloc(&dbg, 4ull * m * sizeof(uint32_t)));
    wmi_batch *b = nullptr;
    // submit normally (runs once), then rerun the main kernel with the debug
    // pointers set, on the same descriptors and sorted marginals
    if (int rc = wmi_submit(st, &q, 1, &p, nullptr, &b)) {
        (void)hipFree(dbg);
        return rc;
    }
    int rc = finish_if_done(b, true, -1);
    if (rc == WMI_OK) {
        LaunchArgs a = b->args;
        a.dbg_nx = reinterpret_cast<uint32_t *>(dbg);
        a.dbg_ny = a.dbg_nx + m;
        a.dbg_ex = reinterpret_cast<float *>(a.dbg_ny + m);
        a.dbg_ey = a.dbg_ex + m;
        hipStream_t s = b->stream;
        hipError_t e = launch_clear(a, s);
        if (e == hipSuccess)
            e = launch_main(a, b->grid, s);
        std::vector<uint32_t> h(4ull * m);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h.data(), dbg, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = poison(st, e, "wmi_debug_window");
        } else {
            std::memcpy(nx, h.data(), m * sizeof(uint32_t));
            std::memcpy(ny, h.data() + m, m * sizeof(uint32_t));
            std::memcpy(ex, h.data() + 2ull * m, m * sizeof(float));
            std::memcpy(ey, h.data() + 3ull * m, m * sizeof(float));
        }
    }
    wmi_batch_destroy(b);
    (void)hipFree(dbg);
    return rc;
}

}  // extern "C"
