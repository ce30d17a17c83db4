/*
 * wmi.h -- windowed KSG mutual information on AMD MI355X (gfx950): C-ABI.
 *
 * The library evaluates, for batches of time windows over pairs of series
 * held in GPU memory, the KSG estimate of mutual information of Eq. (2)
 * (Section 4.2 of Ho et al., "A Unified Approach for Multi-Scale Synchronous
 * Correlation Search in Big Time Series"), and the noise test of
 * Definition 6.2 for a window split into an overlapping part and a newly
 * added part (Section 6.2).
 *
 * Conventions for every entry point:
 *   - returns WMI_OK (0) or a negative WMI_E* code; the message of the last
 *     failure on the calling thread is available from wmi_last_error();
 *   - pointers named host_* are host memory, d_* are device memory;
 *   - a NULL required pointer gives WMI_EINVAL;
 *   - after a HIP runtime error the store is poisoned: that call and every
 *     later call on the store return WMI_EHIP.
 *
 * Numerics: inputs are float32.  Values on the 2^-12 grid with magnitude
 * below 2^11 give exact neighbour distances and counts; other finite values
 * are evaluated after rounding to that grid and their results carry
 * WMI_F_OFFGRID.  NaN and infinities are rejected when a series is added.
 * Digamma sums are accumulated exactly in 64-bit fixed point (2^-44) and the
 * estimate is formed in double precision; the noise comparisons are done in
 * double precision.
 */
#ifndef WMI_H
#define WMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMI_VERSION_MAJOR 0
#define WMI_VERSION_MINOR 1

/* ---- return codes ------------------------------------------------------ */
#define WMI_OK 0
#define WMI_EINVAL (-1)    /* bad argument: id, window range, k, size       */
#define WMI_ENOMEM (-2)    /* can never fit the memory budget               */
#define WMI_EBUSY (-3)     /* does not fit now (non-blocking), or in use    */
#define WMI_ETIMEDOUT (-4) /* wmi_wait timed out; the batch keeps running   */
#define WMI_EHIP (-5)      /* HIP runtime error; the store is poisoned      */
#define WMI_ESTATE (-6)    /* call not valid in the object's current state  */

/* ---- limits -------------------------------------------------------------- */
#define WMI_MAX_WINDOW 4096 /* points per window, including a noise union   */
#define WMI_MAX_K 16

/* ---- result flags (wmi_result.flags) ------------------------------------- */
#define WMI_F_NOISE 1u       /* Definition 6.2 holds for the triple          */
#define WMI_F_TOO_SHORT 2u   /* some window has m <= k: its MI is NaN        */
#define WMI_F_NONPOS_BASE 4u /* I(w_o) <= 0: Definition 6.2 does not apply   */
#define WMI_F_OFFGRID 8u     /* some value was off the 2^-12 grid / range    */

/* ---- store flags ----------------------------------------------------------- */
#define WMI_STORE_STRICT_GRID 1u /* reject off-grid series at add time        */

/* ---- submit flags (wmi_params.flags) ---------------------------------------- */
#define WMI_SUBMIT_NONBLOCKING 1u /* WMI_EBUSY instead of waiting for memory  */
#define WMI_SUBMIT_PLAIN 2u       /* one kernel launch per window (baseline)   */
/* Evaluate every window on its own, without the reuse of the default batched
 * form (Section 7.1.2's incremental computation: a noise triple's base and
 * extension lists come from its union's scan, so a triple costs its union's
 * distances only).  Results are identical; for comparison. */
#define WMI_SUBMIT_NO_REUSE 4u
/* Also compute the entropy H_w of every window of every query (the
 * denominator of the normalised MI, Section 5.4; read as the entropy of the
 * window's empirical distribution of pairs, natural log):
 *     H_w = -sum_v (c_v / m) ln(c_v / m),
 * c_v the number of the window's m points equal to the pair v in both
 * coordinates; ln m when all pairs are distinct.  Read with
 * wmi_read_entropy.  Not accepted by wmi_submit_noalloc. */
#define WMI_SUBMIT_ENTROPY 8u

typedef struct wmi_store wmi_store;
typedef struct wmi_batch wmi_batch;

typedef struct {
    int device;                /* HIP device ordinal                              */
    uint32_t flags;            /* WMI_STORE_*                                     */
    uint64_t hbm_budget_bytes; /* cap on batch-owned device memory; 0 = 1 GiB      */
} wmi_store_desc;

/*
 * One query (32 bytes).  Series a supplies the first coordinate x, series b
 * the second coordinate y, at the same time indices (Definition 3.4).
 *   ext_side == 0 : one window [start, start + len).
 *   ext_side == +1: a noise triple; base w_o = [start, start + len), extension
 *                   w_d = [start + len, start + len + ext_len), union
 *                   w'' = [start, start + len + ext_len).
 *   ext_side == -1: as +1 with the extension on the left:
 *                   w_d = [start - ext_len, start), w'' = [start - ext_len,
 *                   start + len).
 * Every window must lie inside both series; len + ext_len <= WMI_MAX_WINDOW.
 */
typedef struct {
    uint32_t a, b;
    uint64_t start;
    uint32_t len;
    uint32_t ext_len;
    int32_t ext_side;
    uint32_t reserved; /* must be 0 */
} wmi_query;

/*
 * k          : neighbours, 1..WMI_MAX_K (Eq. 2); 4 is the usual choice.
 * estimator  : 0 = Eq. 2 as printed (per-dimension radii from the k
 *              neighbours, counts with <=, psi(n_x), -1/k);
 *              1 = Kraskov's first form (joint radius, counts with <,
 *              psi(n_x + 1), no -1/k).
 * tau        : noise threshold of Definition 6.2 (nats).
 * tau_normalize: how the noise threshold of Definition 6.2 is scaled by the
 *              extension's entropy (the normalised MI of Section 5.4):
 *              0 compare I(w_d) < tau;
 *              1 compare I(w_d) < tau * ln|w_d| (the entropy when every pair
 *                of w_d is distinct);
 *              2 compare I(w_d) < tau * H(w_d), H as for WMI_SUBMIT_ENTROPY
 *                (ties lower it below ln|w_d|); computed on the device by an
 *                extra pass before the estimates.
 * flags      : WMI_SUBMIT_*.
 */
typedef struct {
    uint32_t k;
    uint32_t estimator;
    double tau;
    uint32_t tau_normalize;
    uint32_t flags;
} wmi_params;

/* One result per query (32 bytes).  mi_ext and mi_union are NaN for plain
 * windows.  MI values are in nats and are not clamped (KSG can be < 0). */
typedef struct {
    double mi_base, mi_ext, mi_union;
    uint32_t flags;
    uint32_t reserved;
} wmi_result;

typedef struct {
    uint64_t windows;        /* windows evaluated (3 per noise triple)         */
    uint64_t ordered_pairs;  /* sum of m (m - 1) over those windows            */
    uint64_t launches;       /* kernel launches used                           */
    double device_ms;        /* event time from first to last launch           */
    uint32_t items;          /* work items of the main kernel                  */
    uint32_t grid;           /* workgroups of the persistent main kernel       */
    uint32_t wg_per_cu;      /* resident main-kernel workgroups per CU         */
    uint32_t cus;            /* compute units of the device                    */
} wmi_batch_stats;

/* Library version as (major << 16) | minor. */
int wmi_version(void);

/* Message of the last failure on this thread ("" if none).  Valid until the
 * next failing call on the same thread. */
const char *wmi_last_error(void);

/* Create a store on a device: uploads the digamma tables (built on the host
 * from the asymptotic series and the recurrence) and owns all device memory
 * it allocates.  *out receives the store.  Thread-safe: a store may be used
 * from several threads. */
int wmi_store_create(const wmi_store_desc *desc, wmi_store **out);

/* Wait for every batch of the store, free its device memory and the store.
 * Batches not yet destroyed become invalid. */
int wmi_store_destroy(wmi_store *store);

/*
 * Work-list and scheduling choices of a store (the tile shapes the autotuner
 * picks per window-size bucket); every choice gives the same results, only
 * the speed differs.  Buckets and ranges:
 *   local_windows[b] windows packed into one workgroup's item when the
 *                    item's largest window has at most 32, 64, 128, 256,
 *                    512 points (b = 0..4): 1..16 (default 16)
 *   triples[b]       noise triples per workgroup item, by the largest union
 *                    in the same buckets: 1..5 (default 5)
 *   sweep_windows[b] windows of a run of equally spaced windows (stride at
 *                    most m / 16, m + stride <= 256) that one workgroup
 *                    derives one from the other (Section 7.1.2), for m <= 64,
 *                    128, 255: 2..255, or 1: such runs are evaluated window
 *                    by window (default 8)
 *   stragglers[b]    for windows above 512 points (m <= 1024, 2048, 4096):
 *                    a wave stops scanning candidates for its 128 query
 *                    points together once at most this many can still gain,
 *                    and finishes those one at a time: 0..128 (default 16)
 * WMI_EINVAL for a value out of range.  Applies to later submits and newly
 * created servers of the store.
 */
typedef struct {
    uint32_t local_windows[5];
    uint32_t triples[5];
    uint32_t sweep_windows[3];
    uint32_t stragglers[3];
} wmi_tuning;

/* Set the store's choices (NULL: the defaults). */
int wmi_store_set_tuning(wmi_store *store, const wmi_tuning *tuning);

/* The store's current choices. */
int wmi_store_get_tuning(wmi_store *store, wmi_tuning *out);

/* Copy n float32 values from host memory into a new resident series; the
 * caller keeps ownership of host_values.  NaN/Inf -> WMI_EINVAL; off-grid
 * values -> WMI_EINVAL under WMI_STORE_STRICT_GRID.  *id receives the id. */
int wmi_series_add(wmi_store *store, const float *host_values, uint64_t n, uint32_t *id);

/* Register n float32 values already in device memory (e.g. a torch tensor)
 * without copying.  The caller keeps d_values alive and unchanged until the
 * series is removed or the store destroyed.  The values are validated by a
 * kernel on `stream` (a hipStream_t, or NULL for the store's stream); the
 * call returns after that check. */
int wmi_series_add_device(wmi_store *store, const float *d_values, uint64_t n, void *stream,
                          uint32_t *id);

/* Remove a series.  WMI_EBUSY if an unfinished batch reads it. */
int wmi_series_remove(wmi_store *store, uint32_t id);

/* Length of a series (WMI_EINVAL for an unknown id). */
int wmi_series_length(wmi_store *store, uint32_t id, uint64_t *n);

/*
 * Submit `count` queries (host memory, copied before return) for evaluation
 * on `stream` (hipStream_t, or NULL for the store's stream).  The batch owns
 * its device buffers until wmi_batch_destroy.  Returns after enqueueing; the
 * work is ordered after earlier work on the stream.
 * Errors: WMI_EINVAL (bad id, window outside a series, len + ext_len above
 * WMI_MAX_WINDOW, bad k or estimator, reserved field set); WMI_ENOMEM (the
 * batch needs more than the store's budget even when alone); WMI_EBUSY (the
 * batch does not fit beside batches in flight and WMI_SUBMIT_NONBLOCKING is
 * set; without that flag the call waits for memory to free up).
 */
int wmi_submit(wmi_store *store, const wmi_query *host_queries, uint64_t count,
               const wmi_params *params, void *stream, wmi_batch **out);

/*
 * A run of `count` equally spaced queries of one series pair (the sliding
 * windows of Definition 3.4, or the shifted windows of Section 6.2 split into
 * overlap and new part): query i (0 <= i < count) is
 *     { a, b, start + i * stride, len, ext_len, ext_side }
 * with the meaning of wmi_query.  40 bytes.
 */
typedef struct {
    uint32_t a, b;
    uint64_t start;
    uint32_t count;
    uint32_t stride;   /* >= 1 when count > 1                                 */
    uint32_t len;
    uint32_t ext_len;  /* 0 with ext_side 0: plain windows                    */
    int32_t ext_side;
    uint32_t reserved; /* must be 0                                           */
} wmi_range;

/*
 * wmi_submit for queries given as runs: the batch holds the queries of
 * ranges[0], then those of ranges[1], ... (total = sum of count), and gives
 * bit-identical results to wmi_submit of that list.  The host plans per run,
 * not per window: the window descriptors, query descriptors and work queue are
 * written on the device by an expansion kernel at every run of the batch
 * (submit and each replay), before the estimates, so only the run list
 * (n_ranges x 40 bytes) crosses PCIe.  A run with count 0 adds nothing.
 * Every query of a run must be valid as for wmi_submit (it suffices that the
 * first and the last are).  Flags as wmi_submit except WMI_SUBMIT_PLAIN
 * (WMI_EINVAL).  Errors as wmi_submit; WMI_EINVAL also for a reserved field
 * set, stride 0 with count > 1, or more than 2^32 - 16 queries.
 */
int wmi_submit_ranges(wmi_store *store, const wmi_range *host_ranges, uint64_t n_ranges,
                      const wmi_params *params, void *stream, wmi_batch **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as wmi_submit, without allocating.  Descriptors, sorted
 * marginals, counters and per-window estimates of the call live in a static
 * device array of WMI_NOALLOC_SCRATCH_BYTES per device, held until the process
 * ends; results (count entries of 32 bytes, as wmi_read writes them) go to
 * d_results, device memory the caller owns.  Queries are host memory, read
 * before return.  Synchronous: returns once the results are in d_results
 * (work ordered on `stream`, NULL for the store's stream).  No hipMalloc,
 * hipFree or pinned-host allocation is made; the work list is planned in
 * ordinary host memory.  Every call on a device shares that device's array
 * and overwrites it; the library serialises calls per device, so calls that
 * overlap on one GPU wait for each other.
 * Errors: as wmi_submit; WMI_EINVAL for params->flags != 0 (no plain form,
 * no budget); WMI_ENOMEM when the call needs more scratch than the array
 * holds (about 80 bytes per window, 56 per query and 12 per point of each
 * window above 512 points).
 */
#define WMI_NOALLOC_SCRATCH_BYTES (64ull << 20)
int wmi_submit_noalloc(wmi_store *store, const wmi_query *host_queries, uint64_t count,
                       const wmi_params *params, void *stream, wmi_result *d_results);

/* Wait up to timeout_us microseconds (< 0: forever) for a batch to finish.
 * WMI_ETIMEDOUT leaves the batch running. */
int wmi_wait(wmi_batch *batch, int64_t timeout_us);

/* Nonzero if the batch has finished (does not block). */
int wmi_done(wmi_batch *batch);

/* Wait for the batch, then copy its `count` results to host_out. */
int wmi_read(wmi_batch *batch, wmi_result *host_out);

/* Window entropies of a batch submitted with WMI_SUBMIT_ENTROPY: 3 doubles per
 * query (base, extension, union; a plain window fills the first, NaN in the
 * others) into host_out (3 * count doubles, caller-owned).  Waits as
 * wmi_read.  WMI_ESTATE when the batch was submitted without the flag.
 * H is exact to a few units in the last place: the sum of ln c over the
 * points is taken in 2^-44 fixed point, independent of the schedule. */
int wmi_read_entropy(wmi_batch *batch, double *host_out);

/* ---- replay flags ------------------------------------------------------------ */
#define WMI_REPLAY_DIRECT 1u /* enqueue kernel by kernel (per-kernel timing), no graph */

/*
 * Run the batch's work again, unchanged, on `stream` (NULL: the stream it was
 * submitted on): descriptor upload and kernels, which write the results
 * straight into the batch's pinned host buffer (read with wmi_read once the
 * batch is done).  By default
 * the sequence is captured once into a HIP graph and the graph is launched;
 * WMI_REPLAY_DIRECT enqueues the kernels one by one with events around each.
 * Runs may be pipelined: a replay does not wait for earlier runs, which are
 * ordered before it on the same stream; results are overwritten with the same
 * values.  WMI_SUBMIT_PLAIN batches always replay launch by launch.
 */
int wmi_batch_replay(wmi_batch *batch, void *stream, uint32_t flags);

/* Average event timings over the most recent runs of a batch (up to 16);
 * waits for the batch.  mode: 0 direct, 1 graph, 2 plain, -1 mixed. */
typedef struct {
    uint32_t runs;
    int32_t mode;
    double total_ms; /* upload + kernels (results land in host memory)            */
    double prep_ms;  /* prep (sorted marginals) kernel; NaN unless mode 0          */
    double main_ms;  /* main (neighbours, counts, digamma) kernel; NaN unless mode 0 */
} wmi_timing;

int wmi_batch_timing(wmi_batch *batch, wmi_timing *out);

/* Counters and device time of a finished batch (of its last run). */
int wmi_batch_stats_get(wmi_batch *batch, wmi_batch_stats *out);

/*
 * Distance evaluations of the batch's main kernel: runs the batch's kernels
 * once more (results are rewritten with the same values) with a per-workgroup
 * counter and writes to *evaluated the number of (query point, candidate)
 * distances the neighbour searches computed for live query points, the point
 * itself excluded, each query point counting candidates of its own window
 * only (a wave holding several short windows also scans padding past a
 * lane's window; those keys are masked and not counted).  The estimator's
 * definition (Eq. 2) asks for the k nearest of all m - 1 other points, so
 * m (m - 1) per window is the brute-force count; windows above 512 points
 * scan outwards in x order and stop early, so the count is lower there.  Synchronous on the batch's stream; allocates 8 bytes per
 * main-kernel workgroup for the call.  WMI_EINVAL for plain batches.
 */
int wmi_batch_count_evals(wmi_batch *batch, uint64_t *evaluated);

/* Wait for the batch and release it (NULL is accepted). */
int wmi_batch_destroy(wmi_batch *batch);

/*
 * Per-point export of one window for exact parity tests: evaluates the base
 * window of *query (ext fields ignored) and writes, for point i of the
 * window, the marginal counts nx[i], ny[i] and the radii eps_x[i], eps_y[i]
 * (estimator 0: largest |dx|, |dy| over the k neighbours; estimator 1: the
 * joint k-th distance in both), each host arrays of query->len elements.
 * Synchronous.
 */
int wmi_debug_window(wmi_store *store, const wmi_query *query, const wmi_params *params,
                     uint32_t *host_nx, uint32_t *host_ny, float *host_eps_x, float *host_eps_y);

/* ==========================================================================
 * Serving: continuous batching of range requests over resident series.
 *
 * A request asks for the MI of every window of w points starting at start,
 * start + stride, ... that lies inside [start, end) of the pair (a, b) -- the
 * sliding-window sweep a correlation search submits (Sections 5.1 and 5.2).
 * A scheduler thread admits requests in arrival order while their results
 * fit the server's HBM arena (the admission budget), then keeps building
 * launches from the windows of every admitted request not yet scheduled:
 * requests arriving while others run join the next launch, long requests are
 * cut across launches, and two launch slots keep the device busy while the
 * next launch is prepared.  A request completes when all its windows are
 * done and its results are back in host memory.  Results are exact and do not
 * depend on how requests were batched.
 * ========================================================================== */

typedef struct wmi_server wmi_server;

typedef struct {
    uint64_t hbm_budget_bytes;   /* result arena for admitted requests; 0 = 256 MiB */
    uint32_t k;                  /* estimator parameters of every request        */
    uint32_t estimator;
    uint32_t max_launch_windows; /* windows per launch; 0 = 65536                 */
    uint32_t flags;              /* 0                                             */
} wmi_server_desc;

typedef struct {                 /* 32 bytes */
    uint32_t a, b;               /* series pair (x from a, y from b)              */
    uint64_t start;              /* first window start                            */
    uint64_t end;                /* windows lie in [start, end); end <= lengths   */
    uint32_t w;                  /* window points, 1..WMI_MAX_WINDOW              */
    uint32_t stride;             /* >= 1                                           */
} wmi_request;

typedef struct {                 /* 16 bytes */
    double mi;                   /* nats; NaN with WMI_F_TOO_SHORT when w <= k    */
    uint32_t flags;              /* WMI_F_TOO_SHORT, WMI_F_OFFGRID                 */
    uint32_t reserved;
} wmi_window_result;

typedef struct {
    uint64_t windows;            /* windows of the request                       */
    double t_arrival_us;         /* server clock (microseconds) at submit        */
    double t_admit_us;           /* admitted into the arena                      */
    double t_first_launch_us;    /* its first windows launched                   */
    double t_complete_us;        /* results in host memory                       */
    int32_t state;               /* 0 queued, 1 admitted, 2 done, < 0 WMI_E code */
    uint32_t launches;           /* launches its windows were spread over         */
} wmi_request_info;

typedef struct {
    uint64_t requests_done;
    uint64_t windows_done;
    uint64_t ordered_pairs_done;
    uint64_t launches;
    double busy_us;              /* sum of launch durations (events); launches of
                                    the two slots overlap, so it can exceed wall time */
    uint64_t arena_bytes;        /* admission budget                             */
    uint64_t arena_peak_bytes;   /* most arena bytes held at once                */
    uint64_t queued_peak;        /* most requests waiting for admission at once   */
    double busy_union_us;        /* device time with at least one launch running
                                    (union of the launch intervals; <= wall time) */
} wmi_server_stats;

/* Start a server on a store (its series stay owned by the store; a series
 * read by a pending request cannot be removed).  Allocates the arena and two
 * launch slots and starts the scheduler thread. */
int wmi_server_create(wmi_store *store, const wmi_server_desc *desc, wmi_server **out);

/* Enqueue a request (copied); never blocks.  *ticket identifies it.
 * WMI_EINVAL for a bad series id, window or stride; WMI_ENOMEM if its results
 * alone exceed the arena. */
int wmi_server_submit(wmi_server *server, const wmi_request *request, uint64_t *ticket);

/* Wait up to timeout_us (< 0: forever) for a request to complete. */
int wmi_server_wait(wmi_server *server, uint64_t ticket, int64_t timeout_us);

/* Progress and timestamps of a request (any state). */
int wmi_server_info(wmi_server *server, uint64_t ticket, wmi_request_info *info);

/* Copy a completed request's results (info->windows entries, in window
 * order) to host_out, which holds `capacity` entries, then forget the ticket.
 * WMI_ESTATE if not complete; WMI_EINVAL if capacity is too small. */
int wmi_server_read(wmi_server *server, uint64_t ticket, wmi_window_result *host_out, uint64_t capacity,
                    wmi_request_info *info);

/* Server counters. */
int wmi_server_stats_get(wmi_server *server, wmi_server_stats *out);

/* Current server clock in microseconds (the clock of wmi_request_info). */
double wmi_server_clock_us(wmi_server *server);

/* Finish every pending request, stop the scheduler and free the server. */
int wmi_server_destroy(wmi_server *server);

/* ==========================================================================
 * Search drivers: native host code that walks one of the paper's search
 * rules over a series pair and evaluates the candidate windows in batches
 * through the path above.  A driver's result is exactly that of the rule
 * applied window by window; the batching only decides which windows are
 * evaluated together on the device.
 * ========================================================================== */

typedef struct {                 /* 24 bytes */
    uint64_t start;              /* window [start, start + len) of the pair      */
    uint32_t len;
    uint32_t layer;              /* top-down: layer (0 = s_max)                   */
    double mi;                   /* I_w in nats                                   */
} wmi_window;

typedef struct {
    uint64_t layers;             /* layers searched                               */
    uint64_t windows_visited;    /* windows the sequential rule examined          */
    uint64_t windows_evaluated;  /* windows evaluated on the device (a noise
                                    triple counts 3)                              */
    uint64_t ordered_pairs;      /* distances computed: m (m - 1) per window; a
                                    noise triple of at most 512 points counts its
                                    union's only (parts come from its scan)       */
    uint64_t noise_detections;   /* shifted windows whose new part was noise      */
    uint64_t noise_skips;        /* shifts cancelled after p detections in a row  */
    uint64_t batches;            /* batches submitted                             */
    double wall_ms;              /* whole call                                    */
    double submit_ms;            /* of which inside batch submission (planning,
                                    upload, launch)                              */
    double wait_ms;              /* of which waiting for and reading results      */
} wmi_search_stats;

/*
 * Top-down search (Algorithm 1, Section 5.1) with noise-based pruning
 * (Section 6.2).  Layer 0 slides windows of s_max points over [begin, end);
 * each later layer halves the window size, down to s_min, and slides over
 * the uncorrelated partitions the layer above left: the stretches of its
 * partitions not covered by a correlated window.  Inside a partition a window
 * w with I_w >= sigma is correlated and reported, and the next window starts
 * where w ends; otherwise the next window is w shifted by the layer's step
 * delta = max(1, s_w / step_div).  With pruning (p > 0) a shifted window is
 * split into its overlap with the previous window and its delta new points;
 * when Definition 6.2 flags the new part as noise in p consecutive shifted
 * windows, the shift is cancelled and the next window starts where the last
 * one ends.
 *   s_max, s_min : 2 <= s_min <= s_max <= WMI_MAX_WINDOW.
 *   step_div     : 0 means 8.
 *   normalize    : thresholds of the normalised MI (Section 5.4): 0 compares
 *                  I_w >= sigma and I(w_d) < tau; 1 compares I_w >= sigma *
 *                  ln|w| and I(w_d) < tau * ln|w_d| (the entropy of |w|
 *                  distinct samples); 2 takes the windows' empirical
 *                  entropies H(w), H(w_d) (WMI_SUBMIT_ENTROPY) instead.
 * Output: the correlated windows in ascending start order (non-overlapping),
 * written to host_out (capacity entries; (end - begin) / s_min + 1 always
 * suffice); *n_out receives their number.  WMI_EINVAL for bad ids, ranges or
 * parameters, or a capacity below the number found (nothing written).
 * stats may be NULL.  Synchronous; uses the store's stream.
 */
typedef struct {
    uint32_t s_max, s_min;
    uint32_t step_div;
    uint32_t p;
    double sigma;
    double tau;
    uint32_t normalize;
    uint32_t k;
    uint32_t estimator;
    uint32_t flags;              /* 0 */
} wmi_td_params;

int wmi_td_search(wmi_store *store, uint32_t a, uint32_t b, uint64_t begin, uint64_t end,
                  const wmi_td_params *params, wmi_window *host_out, uint64_t capacity, uint64_t *n_out,
                  wmi_search_stats *stats);

/*
 * Bottom-up search (Algorithm 2, Section 5.2): late-acceptance hill climbing
 * over windows, with the directional noise pruning of Section 6.3.
 * [begin, end) is cut into consecutive chunks of `chunk` points (0: one
 * chunk); each chunk is searched by its own walker, and the walkers advance
 * together, one batch per step (the partitioned form of Section 7.2 without
 * overlap, so that results never overlap).  A walker repeats, from the start
 * of the unexplored rest of its chunk:
 *   w = the s_min first points; history L_h (h entries) := I(w); idle = 0;
 *   while idle <= max_idle:
 *     N = the ring of windows whose start and end differ from w's by at most
 *         r = idle + 1 steps of delta, one of them by exactly r (8r windows),
 *         inside the unexplored rest, s_min <= |w'| <= s_max, without the
 *         directions pruning has closed;
 *     best = the neighbour of largest I (first in the order start offset,
 *         then end offset, ascending);  j = a pick of L_h;
 *     if I(best) > L_h[j] or I(best) > I(w): w = best, idle = 0
 *     else idle += 1;
 *     if I(w) > L_h[j]: L_h[j] = I(w)
 *   report w if I(w) >= sigma (normalize 1: sigma * ln|w|; 2: sigma * H(w),
 *   as for wmi_td_search); the rest starts at w's end.
 * Pruning (p > 0): the ring's pure left extension (start - r delta, same end)
 * and pure right extension are evaluated as noise triples over w; when
 * Definition 6.2 flags a direction's extension in p consecutive steps, that
 * direction (neighbours starting before w, or ending after it) is closed for
 * the rest of the climb.
 * Picks: pick number i (0, 1, ...) of the walker of chunk c is
 *   splitmix64(seed + (c * 2^32 + i + 1) * 0x9E3779B97F4A7C15) mod h,
 * where splitmix64(z) applies z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
 * z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31 (Steele, Lea and
 * Flood's SplitMix64 output function).
 * Output, capacity and errors as for wmi_td_search ((end - begin) / s_min + 1
 * entries suffice); layer is 0.
 */
typedef struct {
    uint32_t s_min, s_max;       /* 2 <= s_min <= s_max <= WMI_MAX_WINDOW        */
    uint32_t delta;              /* moving step, >= 1                             */
    uint32_t max_idle;           /* T_maxIdle                                     */
    uint32_t history;            /* h >= 1                                        */
    uint32_t p;                  /* 0: no pruning                                 */
    double sigma;
    double tau;
    uint32_t normalize;
    uint32_t k;
    uint32_t estimator;
    uint32_t chunk;              /* points per walker; 0 = the whole range        */
    uint64_t seed;
    uint32_t flags;              /* 0 */
    uint32_t reserved;           /* 0 */
} wmi_bu_params;

int wmi_bu_search(wmi_store *store, uint32_t a, uint32_t b, uint64_t begin, uint64_t end,
                  const wmi_bu_params *params, wmi_window *host_out, uint64_t capacity, uint64_t *n_out,
                  wmi_search_stats *stats);

/*
 * wmi_bu_search over several series pairs at once: the walkers of every span
 * advance together, so each step is one batch over all of them (fewer, larger
 * batches than one call per span).  Span i gives exactly the windows, in the
 * same order, that wmi_bu_search(store, a, b, begin, end, params, ...) gives:
 * chunk numbering (and so the picks) restarts at 0 in every span.  Output:
 * the windows of span 0 (ascending start), then those of span 1, ...;
 * host_span[j] (NULL: not written) receives the span of window j.  Capacity
 * and errors as for wmi_bu_search (sum over spans of (end - begin) / s_min + 1
 * entries suffice); stats sum over the spans.
 */
typedef struct {
    uint32_t a, b;
    uint64_t begin, end;
} wmi_span;

int wmi_bu_search_many(wmi_store *store, const wmi_span *spans, uint64_t n_spans, const wmi_bu_params *params,
                       wmi_window *host_out, uint32_t *host_span, uint64_t capacity, uint64_t *n_out,
                       wmi_search_stats *stats);

/* Copy the library's double-precision digamma table psi(1..n) (n <= 8192)
 * to host_out (for checks against an independent construction). */
int wmi_psi_table(uint32_t n, double *host_out);

#ifdef __cplusplus
}
#endif

#endif /* WMI_H */
