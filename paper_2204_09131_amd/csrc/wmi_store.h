// wmi_store.h -- store internals shared by the batch runtime and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "wmi.h"
#include "wmi_internal.h"

namespace wmi {

constexpr uint64_t kDefaultBudget = 1ull << 30;

// Record the message of a failing call for wmi_last_error (this thread).
int fail(int code, const char *fmt, ...);
const char *last_error();

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

struct Series {
    const float *d = nullptr;
    uint64_t n = 0;
    bool owned = false;
    bool live = false;
    bool offgrid = false;
    uint32_t busy = 0;  // unfinished batches and server requests reading it
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

hipError_t launch_clear(const LaunchArgs &a, hipStream_t s);
hipError_t launch_prep(const LaunchArgs &a, uint32_t n_windows, hipStream_t s);
hipError_t launch_entropy(const EntropyArgs &a, hipStream_t s);
hipError_t launch_expand_ranges(const RangeDesc *rd, uint32_t n_rd, uint32_t n_query, WinDesc *win, QDesc *qd,
                                Item *queue, hipStream_t s);
hipError_t launch_main(const LaunchArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_validate(const float *v, uint64_t n, unsigned long long *bad, hipStream_t s);
hipError_t launch_expand(const LaunchArgs &a, const PartDesc *parts, uint32_t n_parts, Item *queue, WinDesc *win,
                         QDesc *qd, uint64_t *cdst, hipStream_t s);
int main_occupancy(uint32_t k, bool local_only = false);
// Device address of the allocation-free entry point's scratch array on
// `device` (which must be current); looked up once per device.
hipError_t noalloc_scratch(int device, void **ptr);
void build_psi_tables(int n_max, std::vector<double> &psi_d, std::vector<long long> &psi_fix);

}  // namespace wmi

struct wmi_store {
    int device = 0;
    uint32_t flags = 0;
    uint64_t budget = wmi::kDefaultBudget;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    double *psi_d = nullptr;
    long long *psi_fix = nullptr;
    int cu_count = 1;
    void *scratch = nullptr;  // device address of this device's no-alloc scratch array
    wmi::Tuning tune = wmi::default_tuning();  // work-list choices (store mutex)
    std::mutex mu;
    std::condition_variable cv;
    std::vector<wmi::Series> series;
    uint64_t inflight = 0;
    bool poisoned = false;
    std::string poison_msg;
    std::set<wmi_batch *> batches;
    std::set<wmi_server *> servers;
    // buffers of destroyed batches kept for the next submits (a driver that
    // submits thousands of small batches would otherwise allocate and free
    // device and pinned memory every time)
    struct Spare {
        char *p;
        size_t bytes;
    };
    std::vector<Spare> spare_dev, spare_host;
    size_t spare_dev_bytes = 0, spare_host_bytes = 0;
};

namespace wmi {
// Poison the store after a HIP error; returns WMI_EHIP.
int poison(wmi_store *st, hipError_t e, const char *what);
int check_poison(wmi_store *st);
}  // namespace wmi

#define HIPCHK(st, expr)                          \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess)                     \
            return wmi::poison((st), e_, #expr);  \
    } while (0)
