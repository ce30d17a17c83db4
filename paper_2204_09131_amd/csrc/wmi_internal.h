// wmi_internal.h -- device-side descriptors shared by the runtime and kernels.
//
// HBM layout of one launch (all arrays carved from one batch allocation):
//   WinDesc  win[W]      one per window (a noise triple contributes three)
//   Item     item[I]     the work queue: prep items first (sort a split
//                        window's marginals), then split items (one block of
//                        query points of a window above kLocalSlots points),
//                        local items (up to kLocalWindows consecutive
//                        windows done entirely inside one workgroup) and
//                        triple items (up to kTripleMax noise triples, each
//                        evaluated through its union), larger work first
//   u32      prep[Np]    the split windows (plain form: sorted by the prep
//                        kernel, one launch per window)
//   u32      ready[W]    per window: sorted marginals written
//   QDesc    qd[Qn]      one per query: its first window, window count, tau
//   int32    sorted[3*P] per split window (P = sum of their m): its points
//                        in x order (keys with index, and their y) and its
//                        y grid integers in ascending order
//   u64      acc[W]      fixed-point digamma sums (2^-44), integer atomics
//   u32      wdone[W], qdone[Qn], counter[1]   completion and work counters
//   double   wmi[W]; u32 wflags[W]           per-window estimate and flags
//   Result   res[Qn]     32-byte results, copied back to the host
// A serving launch has the same arrays (one window per query) and writes
// CompactResult records into request slices of the server's arena instead
// of res.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace wmi {

constexpr int kMaxWindow = 4096;
constexpr int kMaxK = 16;
constexpr int kPsiMax = 8192;         // psi tables cover 1..kPsiMax
constexpr int kBlock = 256;           // threads per workgroup
constexpr int kFixShift = 44;         // fixed-point scale of the digamma sums

constexpr uint32_t kFlagNoise = 1u, kFlagTooShort = 2u, kFlagNonPos = 4u, kFlagOffGrid = 8u;

constexpr int kSplitPoints = 2 * kBlock;  // query points per split item
constexpr int kLocalSlots = 2 * kBlock;   // points (each window padded to even) per local item
constexpr int kLocalWindows = 16;         // windows per local item
constexpr int kLocalSort = 1024;          // windows x pow2(max m) per local item
constexpr uint32_t kItemLocal = 0x80000000u;
constexpr uint32_t kItemPrep = 0x40000000u;  // sort a split window's marginals
constexpr uint32_t kItemTriple = 0x20000000u;  // noise triples evaluated through their unions
constexpr int kTripleMax = 5;                   // triples per triple item
// Sweep items: runs of equally spaced windows of one series pair, each window
// derived from the one before (points removed and added).  A run qualifies
// when kSweepMinM <= m, m + stride <= kSweepRing and kSweepStrideDiv * stride
// <= m; kSweepWindows windows per item.
constexpr uint32_t kItemSweep = 0x10000000u;
constexpr int kSweepRing = 256;  // m + stride: one window point per thread
constexpr int kSweepSpan = 512;  // points of a sweep item's run, held in LDS
constexpr int kSweepMinM = 2 * kMaxK + 2;
constexpr int kSweepStrideDiv = 16;
constexpr int kSweepWindows = 8;

// Work-list and scheduling choices (the tile shapes an autotuner picks per
// window-size bucket); every choice gives the same results.  Buckets:
//   local_windows[b]  windows per local item whose largest m is at most
//                     32, 64, 128, 256, 512 (b = 0..4): 1..kLocalWindows
//   triples[b]        triples per triple item, by the largest union in the
//                     same buckets: 1..kTripleMax
//   sweep_windows[b]  windows per sweep item of m <= 64, 128, 255: 2..255,
//                     or 1: no sweep items for that bucket
//   stragglers[b]     open query slots at which a wave of a window scanned in
//                     x order stops its shared scan (m <= 1024, 2048, 4096):
//                     0..128
struct Tuning {
    uint32_t local_windows[5];
    uint32_t triples[5];
    uint32_t sweep_windows[3];
    uint32_t stragglers[3];
};

inline Tuning default_tuning()
{
    Tuning t;
    for (int b = 0; b < 5; ++b) {
        t.local_windows[b] = (uint32_t)kLocalWindows;
        t.triples[b] = (uint32_t)kTripleMax;
    }
    for (int b = 0; b < 3; ++b) {
        t.sweep_windows[b] = (uint32_t)kSweepWindows;
        t.stragglers[b] = 16u;
    }
    return t;
}

// (constexpr: usable on the host and the device)
constexpr int local_bucket(uint32_t m) { return m <= 32 ? 0 : m <= 64 ? 1 : m <= 128 ? 2 : m <= 256 ? 3 : 4; }
constexpr int sweep_bucket(uint32_t m) { return m <= 64 ? 0 : m <= 128 ? 1 : 2; }
constexpr int split_bucket(uint32_t m) { return m <= 1024 ? 0 : m <= 2048 ? 1 : 2; }
constexpr uint32_t kWaitLimit = 1u << 22;    // polls before a dependency wait gives up
// Device scratch of the allocation-free entry point: one static array per
// device (descriptors, sorted data, counters, estimates of one call).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr uint32_t kErrWait = 1u;            // error word: a dependency wait gave up
constexpr uint32_t kErrItemKind = 2u;        // error word: an item the kernel variant does not run
// ready word of a split window, written by its prep item once the sorted data
// is in HBM: kReady, kReadyOffGrid if a value is off the grid, and the key
// index bits nb (0: 64-bit keys) from kReadyNbShift
constexpr uint32_t kReady = 1u, kReadyOffGrid = 2u;
constexpr uint32_t kReadyNbShift = 8;
// Sorted data of a split window (kSortedWords x m words from sorted_off):
//   [0, m)   32-bit keys: ((X - min_x) << nb) | i in ascending order (the
//            points in x order, each with its index); with nb == 0 (64-bit
//            keys) the grid integers X in ascending order
//   [m, 2m)  (Y - min_y) << nb of the point at each sorted-x position
//   [2m, 3m) the grid integers Y in ascending order
constexpr int kSortedWords = 3;

struct WinDesc {            // 32 bytes
    const float *x;         // series a + window start
    const float *y;         // series b + window start
    uint32_t m;             // points in the window
    uint32_t query;         // owning query (index within the launch)
    uint32_t sorted_off;    // offset of this window's sorted arrays (in points)
    uint32_t n_items;       // kNN items covering the window's points
};

struct Item {               // 8 bytes
    uint32_t win;           // split / prep: the window; local: its first window
    uint32_t info;          // split: first query point; local: kItemLocal | windows; prep: kItemPrep;
                            // triple: kItemTriple | triples (win: the first triple's base window)
};

struct QDesc {              // 16 bytes
    uint32_t win0;          // first window of the query
    uint32_t nwin;          // 1 (plain window) or 3 (base, extension, union)
    double tau_eff;         // noise threshold, already normalised if requested
};

struct WinAux {             // per split window: from its values (prep), or its ready word and sorted data
    int32_t min_x, min_y;   // window minima of the grid integers
    uint32_t nb;            // index bits in a 32-bit key; 0 selects 64-bit keys
    uint32_t flags;         // kFlagOffGrid
    uint32_t range_x, range_y;  // max - min of the grid integers
};

struct Result {             // 32 bytes, same layout as wmi_result
    double mi_base, mi_ext, mi_union;
    uint32_t flags, reserved;
};

// Serving: results of single windows, 16 bytes, written into request slices
// of an HBM arena.
struct CompactResult {
    double mi;
    uint32_t flags, reserved;
};

// Serving: a run of windows of one request inside a launch: `count` windows
// of m points starting at start, start + stride, ... on series (x, y).  The
// expand kernel turns parts into window descriptors and queue items.
struct PartDesc {           // 64 bytes
    const float *x;         // series a (window 0 starts at x + start)
    const float *y;         // series b
    uint64_t start;
    uint64_t dst;           // arena index of the part's first window result
    uint32_t stride;
    uint32_t count;
    uint32_t m;
    uint32_t win0;          // launch index of the part's first window
    uint32_t sorted0;       // sorted-marginal offset of its first window (m > kLocalSlots)
    uint32_t prep0;         // queue index of its first prep item (m > kLocalSlots)
    uint32_t item0;         // queue index of its first split / local item
    uint32_t per_item;      // local windows per item (m <= kLocalSlots)
};

struct LaunchArgs {
    const WinDesc *win;
    const Item *item;
    const QDesc *qd;
    int32_t *sorted;
    unsigned long long *acc;
    uint32_t *wdone;
    uint32_t *qdone;
    uint32_t *counter;
    double *wmi;
    uint32_t *wflags;
    Result *res;
    const double *psi_d;          // psi(n) in double, index n (0 unused)
    const long long *psi_fix;     // round(psi(n) * 2^44), index n (0 unused)
    uint32_t n_win;
    uint32_t n_items;
    uint32_t n_query;
    uint32_t item_begin;          // first item of this launch
    uint32_t k;
    uint32_t estimator;
    uint32_t persistent;          // 1: take items from *counter; 0: blockIdx.x
    uint32_t win_begin;           // prep kernel: first entry of prep_list for this launch
    const uint32_t *prep_list;    // windows the prep kernel sorts (split windows)
    uint32_t n_prep;
    uint32_t *ready;              // per window: its sorted marginals are in HBM
    uint32_t *err;                // error word (kErrWait)
    // serving: per-query arena index of the result, or null (results in res)
    const uint64_t *cdst;
    CompactResult *arena;
    // debug export (one window): per point counts and radii, or null
    uint32_t *dbg_nx, *dbg_ny;
    float *dbg_ex, *dbg_ey;
    // distance evaluations per workgroup (one counter per workgroup), or null
    unsigned long long *evals;
    uint32_t strag[3];            // straggler thresholds by split_bucket(m)
    // 1: the queue holds local and triple items only, and the launch uses the
    // main kernel compiled for those (fewer registers, more workgroups per CU)
    uint32_t local_only;
};

// A run of equally spaced queries of one series pair, expanded on the device
// (wmi_submit_ranges).  Query i of the run is at start + i * stride; its
// windows are win0 + i (plain) or win0 + 3i .. win0 + 3i + 2 (base,
// extension, union).  kind says how its windows are scheduled; the queue
// offsets are those the host planner gave the run.
enum : uint32_t {
    kRangeLocal = 0,       // plain windows <= kLocalSlots: local items of per_item windows
    kRangeSweep = 1,       // plain windows: sweep items of per_item windows
    kRangeSplit = 2,       // plain windows > kLocalSlots: a prep item and split items each
    kRangeTriple = 3,      // triples with union <= kLocalSlots: triple items of per_item triples
    kRangeTripleWide = 4,  // other triples: each window alone (local item, or prep + split items)
};

struct RangeDesc {          // 80 bytes
    const float *x;         // series a
    const float *y;         // series b
    uint64_t start;         // base start of query 0
    double tau_eff;         // noise threshold of its triples, normalised if requested
    uint32_t stride, count; // queries
    uint32_t m, e;          // base points, extension points (0 for plain windows)
    int32_t side;           // 0 plain, +1 / -1 extension side
    uint32_t kind, per_item;
    uint32_t q0, win0;      // first query and window of the run
    uint32_t item0;         // first local / triple / sweep / split item
    uint32_t item1;         // kRangeTripleWide: first split item
    uint32_t prep0;         // first prep item
    uint32_t sorted0;       // sorted-marginal offset (points) of query 0's first split window
    uint32_t pad;
};

// Window entropies (the normalised MI of Section 5.4): per query, H of its
// windows into hres (3 per query, NaN where a query has no such window; null:
// extensions only), and with set_tau the noise threshold tau * H(extension)
// into the query's descriptor.
struct EntropyArgs {
    const WinDesc *win;
    QDesc *qd;
    double *hres;
    double tau;
    uint32_t n_query;
    uint32_t set_tau;
};

}  // namespace wmi
