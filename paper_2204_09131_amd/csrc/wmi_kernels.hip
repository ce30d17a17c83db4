// wmi_kernels.hip -- gfx950 kernels for windowed KSG mutual information.
//
// One window = m co-indexed points (x_i, y_i) = (X_a[s + i], X_b[s + i])
// (Definitions 3.2 and 3.4).  Its estimate is Eq. (2) of Section 4.2:
//   I = psi(k) - 1/k + psi(m) - < psi(n_x) + psi(n_y) >
// with the k nearest neighbours taken in the joint space under the maximum
// norm (Section 7.1.1 and its footnote), per-dimension radii from those
// neighbours and marginal counts inside the radii (the worked example of
// Section 7.1.1: counts use <= and include the neighbours, not the point).
//
// No MFMA anywhere: a max-norm neighbour search is not a contraction; the
// bound is the 32-bit VALU.  A persistent kernel takes items from an atomic
// counter; the queue holds prep items, then local items, then split items,
// then the cheapest local items (the host's plan decides the order):
//
//   triple item up to 5 noise triples of at most 512 union points in all:
//               each point's base or extension list and its union list
//               come from one scan over the union, so a triple costs the
//               distances of its union only.
//   sweep item  up to 8 equally spaced windows of one pair (stride at most
//               m / 16): the first in full, each next one from the one
//               before by removing and adding points (influenced regions).
//   local item  up to 16 consecutive windows of at most 512 points in total
//               (whole queries where they fit).
//               One workgroup stages them in LDS, finds every point's
//               neighbours (all pairs), sorts each window's marginals in LDS
//               (bitonic), counts by binary search, sums digamma terms with
//               LDS integer atomics and writes the results: no global
//               atomics, no fences.
//   prep item   one window above 512 points: its x order as keys carrying
//               the point index with the y key of each point beside it, and
//               the sorted y integers, written to HBM before the window's
//               ready flag (the plain form launches a prep kernel instead).
//   split item  512 consecutive positions of such a window's x order.  Each
//               wave scans candidates outward from its 128 queries in x
//               order, stops once few queries can still gain, and finishes
//               those one at a time with the whole wave; then the item
//               counts by binary search over the sorted data.  Items add
//               exact fixed-point digamma sums with integer atomics and the
//               last item of a window forms its estimate.
//
// Keys.  With grid integers X = v * 2^12 and U = (X - min) << nb, 2^nb >= m,
// the key of candidate j for query i is
//   max(|Ux_i - Ux_j| + j, |Uy_i - Uy_j| + j) = (d_ij << nb) | j,
// so unsigned order is the order of (distance, index): ties go to the earlier
// time index.  Two v_sad_u32 and one v_max_u32 build a key, and the k (or
// k+1, the point itself dropped at the end) smallest stay in registers under
// a branch-free med3 insertion network.  A window whose value range does not
// fit 32 - nb bits uses 64-bit keys (d << 12 | j) and scans all candidates.
//
// Cross-workgroup values: sums, counters and estimates travel through
// returning atomics issued in order (an s_waitcnt between them); a split
// window's sorted data is published by a device-scope release fence before
// its ready flag and read after an acquire fence.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "wmi_internal.h"
#include "wmi_ranges.h"

namespace wmi {

__device__ __forceinline__ uint32_t sad_u32(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t hi = a > b ? a : b;
    uint32_t lo = a > b ? b : a;
    return (hi - lo) + c;
}

// |a - b| + c in one VALU instruction; c is wave-uniform (an SGPR).  Plain
// arithmetic (no memory access); written as asm because instruction
// selection otherwise splits it into min/max/sub/add.
__device__ __forceinline__ uint32_t sad_key(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// The same with the index c in a vector register (candidates in x order carry
// their own index).
__device__ __forceinline__ uint32_t sad_key_v(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Global loads a thread keeps in flight in the staging loops of the window
// sorts and the split items: each loop issues this many before using any, so
// a window costs one memory latency per batch rather than one per element.
constexpr int kLoadBatch = 8;

// Workgroup barrier after this wave's LDS accesses have completed.  The
// wait is explicit: the compiler's own wait before a barrier at the head of
// a loop (reached along the back edge from LDS stores) was found missing, and
// stores still in flight then raced with other waves' loads.
__device__ __forceinline__ void block_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
}

// Add a wave's distance evaluations, n_live query points times `per_query`
// candidates each, to its workgroup's counter (only when counting).  Every
// lane of the wave calls it with the same values.
__device__ __forceinline__ void count_evals(const LaunchArgs &a, int n_live, int per_query)
{
    if (a.evals && (threadIdx.x & 63) == 0 && n_live > 0 && per_query > 0)
        atomicAdd(&a.evals[blockIdx.x], (unsigned long long)n_live * (unsigned long long)per_query);
}

// Same with a per-lane count: the wave's lanes add `mine` each (only when
// counting).  Every lane of the wave calls it.
__device__ __forceinline__ void count_evals_lanes(const LaunchArgs &a, uint32_t mine)
{
    if (!a.evals)
        return;
    unsigned long long v = mine;
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v > 0)
        atomicAdd(&a.evals[blockIdx.x], v);
}

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a < b ? b : a; }
template <typename T>
__device__ __forceinline__ T med3(T a, T b, T c) { return tmax(tmin(a, b), tmin(tmax(a, b), c)); }

// Insert key into the ascending list t[0..S); the largest entry falls off.
template <int S, typename T>
__device__ __forceinline__ void insert_sorted(T (&t)[S], T key)
{
#pragma unroll
    for (int r = S - 1; r >= 1; --r)
        t[r] = med3(t[r - 1], t[r], key);
    t[0] = tmin(t[0], key);
}

// The same for 32-bit keys, one v_med3_u32 / v_min_u32 per entry.  Written
// as asm (plain arithmetic, no memory access) so that loop analysis does not
// expand the lists as nested min/max expressions: across an unrolled scan
// those grow with every insertion and made compile time explode for k >= 14.
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t min_u32(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_min_u32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

template <int S>
__device__ __forceinline__ void insert_sorted(uint32_t (&t)[S], uint32_t key)
{
#pragma unroll
    for (int r = S - 1; r >= 1; --r)
        t[r] = med3_u32(t[r - 1], t[r], key);
    t[0] = min_u32(t[0], key);
}

// Grid integer of a value; flags values off the 2^-12 grid or out of range.
__device__ __forceinline__ int32_t grid_int(float v, uint32_t &off)
{
    float s = v * 4096.0f;  // exact: power-of-two scaling
    float r = rintf(s);
    if (r != s || fabsf(r) > 8388607.0f)
        off = 1u;
    r = fminf(fmaxf(r, -8388607.0f), 8388607.0f);
    return (int32_t)r;
}

__device__ __forceinline__ uint32_t ceil_log2(uint32_t m)
{
    uint32_t b = 0;
    while ((1u << b) < m)
        ++b;
    return b;
}

// #{S[0..n) < v} for NX thresholds in sx and NX in sy (ascending arrays of n
// entries), the searches interleaved step by step so that their LDS reads
// overlap.  The trip count depends on n only.
template <int NX>
__device__ __forceinline__ void count_lt_xy(const int32_t *sx, const int32_t *sy, int n, const int32_t (&vx)[NX],
                                            const int32_t (&vy)[NX], int (&cx)[NX], int (&cy)[NX])
{
    int bx[NX], by[NX];
#pragma unroll
    for (int t = 0; t < NX; ++t)
        bx[t] = by[t] = 0;
    while (n > 1) {
        const int half = n >> 1;
        int32_t ex[NX], ey[NX];
#pragma unroll
        for (int t = 0; t < NX; ++t) {
            ex[t] = sx[bx[t] + half];
            ey[t] = sy[by[t] + half];
        }
#pragma unroll
        for (int t = 0; t < NX; ++t) {
            bx[t] = ex[t] < vx[t] ? bx[t] + half : bx[t];
            by[t] = ey[t] < vy[t] ? by[t] + half : by[t];
        }
        n -= half;
    }
#pragma unroll
    for (int t = 0; t < NX; ++t) {
        cx[t] = bx[t] + (sx[bx[t]] < vx[t] ? 1 : 0);
        cy[t] = by[t] + (sy[by[t]] < vy[t] ? 1 : 0);
    }
}

// Search thresholds of one point for count_lt_xy (two per dimension), from
// its grid integers and radii.  Estimator 0 counts |d| <= e:
// #{< v + e + 1} - #{< v - e};  estimator 1 counts |d| < e:
// #{< v + e} - #{< v - e + 1}.
__device__ __forceinline__ void count_bounds(uint32_t est, int32_t xi, int32_t yi, int32_t ex, int32_t ey,
                                             int32_t *vx, int32_t *vy)
{
    const int32_t o = est == 0 ? 1 : 0;
    vx[0] = xi + ex + o;
    vx[1] = xi - ex + 1 - o;
    vy[0] = yi + ey + o;
    vy[1] = yi - ey + 1 - o;
}

// Digamma terms of one point from its four counts (the point itself, inside
// every interval, is removed); estimator 1 counts nothing at zero radius and
// uses psi(n + 1).
__device__ __forceinline__ long long point_terms(const LaunchArgs &a, int hx, int lx, int hy, int ly, int32_t ex,
                                                 int &cx, int &cy)
{
    if (a.estimator == 0) {
        cx = hx - lx - 1;
        cy = hy - ly - 1;
        return a.psi_fix[cx] + a.psi_fix[cy];
    }
    cx = ex > 0 ? hx - lx - 1 : 0;
    cy = ex > 0 ? hy - ly - 1 : 0;
    return a.psi_fix[cx + 1] + a.psi_fix[cy + 1];
}

#ifndef WMI_MAIN_K
// --------------------------------------------------------------------------
// clear: zero the counters and accumulators of a launch
// --------------------------------------------------------------------------
__global__ void clear_kernel(LaunchArgs a)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t w = t; w < a.n_win; w += stride) {
        a.acc[w] = 0ull;
        a.wdone[w] = 0u;
        a.ready[w] = 0u;
    }
    if (t == 0)
        a.err[0] = 0u;
    for (uint32_t q = t; q < a.n_query; q += stride)
        a.qdone[q] = 0u;
    if (t == 0)
        a.counter[0] = 0u;
}
#endif  // !WMI_MAIN_K

// --------------------------------------------------------------------------
// prep: sorted marginals of a split window (one workgroup)
// --------------------------------------------------------------------------

// Ascending bitonic sort in LDS of `total` entries of array a (and of b, if
// NA == 2), as segments of P entries each (P a power of two dividing total,
// total <= 2 * R * kBlock).  Each stage pairs entry lo with lo + stride; a
// thread takes pairs tid + r * kBlock and loads all of them before any
// compare, so their LDS latencies overlap.  The 64 pairs a wave takes for one
// r cover one block of 128 consecutive entries whenever stride <= 64: two
// such stages in a row touch only the wave's own blocks, and between them
// the wave only waits for its own LDS stores to complete.  Every other stage
// starts with a workgroup barrier.  Called by the whole workgroup; ends with
// a barrier.
template <int R, int NA>
__device__ void bitonic_lds(int32_t *a, int32_t *b, uint32_t total, uint32_t P)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t npairs = total >> 1;
    bool prev_local = false;
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            const bool local = stride <= 64u;
            if (local && prev_local)
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            else
                block_sync();
            prev_local = local;
            int32_t va[R][2], vb[R][2];
            uint32_t lo[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t t = tid + (uint32_t)(r * kBlock);
                lo[r] = ((t & ~(stride - 1u)) << 1) | (t & (stride - 1u));
                if (t < npairs) {
                    va[r][0] = a[lo[r]];
                    va[r][1] = a[lo[r] + stride];
                    if (NA == 2) {
                        vb[r][0] = b[lo[r]];
                        vb[r][1] = b[lo[r] + stride];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t t = tid + (uint32_t)(r * kBlock);
                if (t < npairs) {
                    // direction from the index inside the segment: every segment ascends
                    const bool asc = ((lo[r] & (P - 1u)) & size) == 0u;
                    const int32_t mn = min(va[r][0], va[r][1]), mx = max(va[r][0], va[r][1]);
                    a[lo[r]] = asc ? mn : mx;
                    a[lo[r] + stride] = asc ? mx : mn;
                    if (NA == 2) {
                        const int32_t nn = min(vb[r][0], vb[r][1]), nx = max(vb[r][0], vb[r][1]);
                        b[lo[r]] = asc ? nn : nx;
                        b[lo[r] + stride] = asc ? nx : nn;
                    }
                }
            }
        }
    }
    block_sync();
}

// Signed median of three: med3_i32(a, b, INT32_MIN) = min(a, b) and
// med3_i32(a, b, INT32_MAX) = max(a, b), so one instruction keeps either
// side of a compare-exchange.
__device__ __forceinline__ int32_t med3_i32(int32_t a, int32_t b, int32_t c)
{
    int32_t r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// The value of lane (lane ^ X) of the wave, X < 64: a swizzle in bit-mask
// mode within each half-wave (and mask 31, xor mask X), a permute across
// halves for X = 32.
template <int X>
__device__ __forceinline__ int32_t xor_lane(int32_t v)
{
    if constexpr (X == 32)
        return __shfl_xor(v, 32, 64);
    else
        return __builtin_amdgcn_ds_swizzle(v, (X << 10) | 0x1F);
}

// One compare-exchange stage of the register bitonic sort at element
// distance 2X (lane distance X), for both arrays and both elements of the
// thread: bound INT32_MIN keeps the smaller value, INT32_MAX the larger.
template <int X>
__device__ __forceinline__ void bitonic_lane_stage(int32_t (&va)[2], int32_t (&vb)[2], int32_t bound)
{
    const int32_t pa0 = xor_lane<X>(va[0]), pa1 = xor_lane<X>(va[1]);
    const int32_t pb0 = xor_lane<X>(vb[0]), pb1 = xor_lane<X>(vb[1]);
    va[0] = med3_i32(va[0], pa0, bound);
    va[1] = med3_i32(va[1], pa1, bound);
    vb[0] = med3_i32(vb[0], pb0, bound);
    vb[1] = med3_i32(vb[1], pb1, bound);
}

// The same ascending segmented sort as bitonic_lds for total <= 2 kBlock
// entries, with the data in registers: thread t holds entries 2t and 2t + 1
// of both arrays.  A stage at distance 1 stays inside the thread, distances
// 2..128 entries (lanes 1..64 of one wave) are exchanged by swizzles, and
// only distances across waves go through LDS.  Each side of a pair computes
// the kept value itself (min or max by the entry's position), one med3 per
// entry.  Called by the whole workgroup after the arrays are staged; the
// sorted arrays are back in LDS when it returns.
__device__ void bitonic_regs(int32_t *a, int32_t *b, uint32_t total, uint32_t P)
{
    const uint32_t e = 2u * threadIdx.x;  // this thread's first entry
    const bool mine = e < total;
    int32_t va[2], vb[2];
    {
        const int2 x = reinterpret_cast<const int2 *>(a)[threadIdx.x];
        const int2 y = reinterpret_cast<const int2 *>(b)[threadIdx.x];
        va[0] = x.x;
        va[1] = x.y;
        vb[0] = y.x;
        vb[1] = y.y;
    }
    for (uint32_t size = 2; size <= P; size <<= 1) {
        const bool asc = ((e & (P - 1u)) & size) == 0u;  // the same for both entries
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride == 1u) {
                const int32_t lo = asc ? INT32_MIN : INT32_MAX, hi = asc ? INT32_MAX : INT32_MIN;
                const int32_t a0 = med3_i32(va[0], va[1], lo), a1 = med3_i32(va[0], va[1], hi);
                const int32_t b0 = med3_i32(vb[0], vb[1], lo), b1 = med3_i32(vb[0], vb[1], hi);
                va[0] = a0;
                va[1] = a1;
                vb[0] = b0;
                vb[1] = b1;
                continue;
            }
            const bool lower = (e & stride) == 0u;
            const int32_t bound = lower == asc ? INT32_MIN : INT32_MAX;
            switch (stride) {
            case 2: bitonic_lane_stage<1>(va, vb, bound); break;
            case 4: bitonic_lane_stage<2>(va, vb, bound); break;
            case 8: bitonic_lane_stage<4>(va, vb, bound); break;
            case 16: bitonic_lane_stage<8>(va, vb, bound); break;
            case 32: bitonic_lane_stage<16>(va, vb, bound); break;
            case 64: bitonic_lane_stage<32>(va, vb, bound); break;
            default: {
                // across waves: through LDS (the partner pair is adjacent too)
                block_sync();  // earlier reads of the arrays are complete
                if (mine) {
                    reinterpret_cast<int2 *>(a)[threadIdx.x] = make_int2(va[0], va[1]);
                    reinterpret_cast<int2 *>(b)[threadIdx.x] = make_int2(vb[0], vb[1]);
                }
                block_sync();
                const uint32_t pe = (e ^ stride) >> 1;  // e < 2 kBlock, stride < 2 kBlock: in the arrays
                const int2 x = reinterpret_cast<const int2 *>(a)[pe];
                const int2 y = reinterpret_cast<const int2 *>(b)[pe];
                va[0] = med3_i32(va[0], x.x, bound);
                va[1] = med3_i32(va[1], x.y, bound);
                vb[0] = med3_i32(vb[0], y.x, bound);
                vb[1] = med3_i32(vb[1], y.y, bound);
            }
            }
        }
    }
    block_sync();  // every read of the last LDS stage is complete
    if (mine) {
        reinterpret_cast<int2 *>(a)[threadIdx.x] = make_int2(va[0], va[1]);
        reinterpret_cast<int2 *>(b)[threadIdx.x] = make_int2(vb[0], vb[1]);
    }
    block_sync();
}

// Segmented ascending sort of the marginals staged in LDS (segments of P
// entries, total a multiple of P, at most kLocalSort): in registers when
// every entry has a thread, else through LDS.
__device__ __forceinline__ void sort_marginals(int32_t *a, int32_t *b, uint32_t total, uint32_t P)
{
    if (total <= 2u * kBlock)
        bitonic_regs(a, b, total, P);
    else
        bitonic_lds<kLocalSort / (2 * kBlock), 2>(a, b, total, P);
}

__device__ WinAux window_aux(const WinDesc &d, int32_t *s_red);

// Stable LSD radix sort of the n <= kMaxWindow words a[0, n) in LDS on bits
// [lo, lo + 4 passes), 4 bits a pass; bits below lo keep their order (the
// sort is stable), bits above are zero.  Wave w holds positions
// [w 64 E, (w + 1) 64 E) striped, element e of lane l at w 64 E + 64 e + l,
// so ranking lanes in order round by round is ranking positions in order.  A
// key's rank among equal digits of its wave comes from four ballots; the
// wave's running digit counts sit in lanes 0..15; one wave scans the 16 x 4
// digit-major totals in s_cnt.  Keys stay in registers across the pass, so
// the scatter writes back into a[] itself.  Positions past n sort last
// (all-ones digits, stable) and are never stored.
__device__ __forceinline__ void radix_lds(uint32_t *a, int n, int lo, int passes, uint32_t *s_cnt)
{
    constexpr int EM = kMaxWindow / kBlock;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int E = (n + kBlock - 1) / kBlock;
    const int wbase = wave * 64 * E;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t dl = (uint32_t)lane & 15u;
    for (int p = 0; p < passes; ++p) {
        const int sh = lo + 4 * p;
        uint32_t key[EM], rk[EM];
        block_sync();  // the previous pass's scatter is complete
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            const int pos = wbase + 64 * e + lane;
            key[e] = (e < E && pos < n) ? a[pos] : 0xFFFFFFFFu;
        }
        uint32_t cnt = 0;  // lane d < 16: keys of digit d met so far in this wave
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            if (e < E) {
                // one round at a time: tie this round's digit to the last
                // round's count, so rounds are not interleaved (their ballots
                // would all be live at once)
                uint32_t kk = key[e];
                asm volatile("" : "+v"(kk) : "v"(cnt));
                const uint32_t dg = (kk >> sh) & 15u;
                const unsigned long long b0 = __ballot(dg & 1u), b1 = __ballot(dg & 2u);
                const unsigned long long b2 = __ballot(dg & 4u), b3 = __ballot(dg & 8u);
                const unsigned long long same = ((dg & 1u) ? b0 : ~b0) & ((dg & 2u) ? b1 : ~b1) &
                                                ((dg & 4u) ? b2 : ~b2) & ((dg & 8u) ? b3 : ~b3);
                rk[e] = (uint32_t)__shfl((int)cnt, (int)dg, 64) + (uint32_t)__popcll(same & lt);
                const unsigned long long mine = ((dl & 1u) ? b0 : ~b0) & ((dl & 2u) ? b1 : ~b1) &
                                                ((dl & 4u) ? b2 : ~b2) & ((dl & 8u) ? b3 : ~b3);
                cnt += (uint32_t)__popcll(mine);
            }
        }
        if (lane < 16)
            s_cnt[lane * 4 + wave] = cnt;
        block_sync();  // every wave has read its keys and published its counts
        if (wave == 0) {
            const uint32_t v = s_cnt[lane];
            uint32_t incl = v;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
                if (lane >= o)
                    incl += u;
            }
            s_cnt[lane] = incl - v;
        }
        block_sync();
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            if (e < E) {
                const uint32_t dg = (key[e] >> sh) & 15u;
                const uint32_t t = s_cnt[dg * 4 + wave] + rk[e];
                if (t < (uint32_t)n)
                    a[t] = key[e];
            }
        }
    }
    block_sync();
}

// A store coherent at agent scope (a relaxed atomic store: written through
// to memory, not held in this XCD's L2), for data another CU reads after a
// flag.
__device__ __forceinline__ void store_through(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bits needed for values up to r (0 for r == 0).
__device__ __forceinline__ int value_bits(uint32_t r) { return r ? 32 - __clz((int)r) : 0; }

// Write the sorted data of split window w to HBM (layout at kSortedWords),
// make it visible to every CU, then raise the window's ready flag.  Two
// sorts, each one radix sort in LDS: x (keys ((X - min_x) << nb) | i, or with
// 64-bit keys the offsets X - min_x) and y (offsets Y - min_y).
__device__ void prep_item(const LaunchArgs &a, uint32_t w, uint32_t *buf, int32_t *s_red, uint32_t *s_cnt)
{
    const WinDesc d = a.win[w];
    const int m = (int)d.m;
    const int tid = threadIdx.x;
    int32_t *out = a.sorted + (uint64_t)kSortedWords * d.sorted_off;
    const WinAux ax = window_aux(d, s_red);
    const uint32_t mask = (1u << ax.nb) - 1u;
    for (int job = 0; job < 2; ++job) {
        const float *v = job ? d.y : d.x;
        const int32_t mn = job ? ax.min_y : ax.min_x;
        // keys carrying the index are built in index order: sorting the bits
        // from nb up stably gives the order of the whole key
        const uint32_t shift = job ? 0u : ax.nb;
        uint32_t off = 0;
        block_sync();
        for (int i0 = tid; i0 < m; i0 += kLoadBatch * kBlock) {
            float vv[kLoadBatch];
#pragma unroll
            for (int g = 0; g < kLoadBatch; ++g)
                vv[g] = v[i0 + g * kBlock < m ? i0 + g * kBlock : i0];
#pragma unroll
            for (int g = 0; g < kLoadBatch; ++g) {
                const int i = i0 + g * kBlock;
                if (i < m)
                    buf[i] = ((uint32_t)(grid_int(vv[g], off) - mn) << shift) | (shift ? (uint32_t)i : 0u);
            }
        }
        radix_lds(buf, m, (int)shift, (value_bits(job ? ax.range_y : ax.range_x) + 3) / 4, s_cnt);
        if (shift) {
            // beside each x-order key the y key of its point: a gather,
            // kLoadBatch loads in flight per thread
            for (int s0 = tid; s0 < m; s0 += kLoadBatch * kBlock) {
                uint32_t key[kLoadBatch];
                float yv[kLoadBatch];
#pragma unroll
                for (int g = 0; g < kLoadBatch; ++g)
                    key[g] = buf[s0 + g * kBlock < m ? s0 + g * kBlock : s0];
#pragma unroll
                for (int g = 0; g < kLoadBatch; ++g)
                    yv[g] = d.y[key[g] & mask];
#pragma unroll
                for (int g = 0; g < kLoadBatch; ++g) {
                    const int s = s0 + g * kBlock;
                    if (s < m) {
                        store_through(&out[s], (int32_t)key[g]);
                        store_through(&out[m + s], (int32_t)((uint32_t)(grid_int(yv[g], off) - ax.min_y) << ax.nb));
                    }
                }
            }
        } else {
            int32_t *dst = job ? out + 2 * m : out;
            for (int s = tid; s < m; s += kBlock)
                store_through(&dst[s], (int32_t)buf[s] + mn);
        }
    }
    // the sorted data went to memory with agent-scope stores: once every
    // wave's stores have completed, the flag may rise.  (A release fence
    // would also write back the whole L2 of the XCD, the other work's dirty
    // lines included; the split items still take an acquire before reading.)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    block_sync();
    if (threadIdx.x == 0)
        atomicExch(&a.ready[w], kReady | (ax.flags ? kReadyOffGrid : 0u) | (ax.nb << kReadyNbShift));
}

// --------------------------------------------------------------------------
// cross-workgroup values: returning atomics only
// --------------------------------------------------------------------------

// Wait until this thread's outstanding memory operations have returned, so a
// following atomic is performed after them.  A wait instruction only.
__device__ __forceinline__ void wait_returned() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ void publish_f64(double *p, double v)
{
    atomicExch(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ double fetch_f64(double *p)
{
    return __longlong_as_double((long long)atomicAdd(reinterpret_cast<unsigned long long *>(p), 0ull));
}

// Result of a query from its windows' estimates (Definition 6.2 for triples).
__device__ __forceinline__ Result compose_result(const QDesc &qd, const double *mi, const uint32_t *fl)
{
    Result r;
    r.reserved = 0u;
    const double nan = __builtin_nan("");
    if (qd.nwin == 1) {
        r.mi_base = mi[0];
        r.mi_ext = nan;
        r.mi_union = nan;
        r.flags = fl[0];
        return r;
    }
    uint32_t f = fl[0] | fl[1] | fl[2];
    if (!(f & kFlagTooShort)) {
        if (!(mi[0] > 0.0))
            f |= kFlagNonPos;
        else if (mi[1] < qd.tau_eff && mi[2] < mi[0])
            f |= kFlagNoise;
    }
    r.mi_base = mi[0];
    r.mi_ext = mi[1];
    r.mi_union = mi[2];
    r.flags = f;
    return r;
}

// Store a query's result: the 32-byte result array, or for serving the
// 16-byte slot of its request in the arena.
__device__ __forceinline__ void store_result(const LaunchArgs &a, uint32_t q, const Result &r)
{
    if (a.cdst) {
        CompactResult c;
        c.mi = r.mi_base;
        c.flags = r.flags;
        c.reserved = 0u;
        a.arena[a.cdst[q]] = c;
    } else {
        a.res[q] = r;
    }
}

// A window's final estimate, reported to its query by one thread.  A plain
// query is written directly; a triple whose windows finished in different
// workgroups is completed by whichever finishes last.
__device__ void report_window(const LaunchArgs &a, uint32_t w, uint32_t q, double mi, uint32_t fl)
{
    const QDesc qd = a.qd[q];
    if (qd.nwin == 1) {
        store_result(a, q, compose_result(qd, &mi, &fl));
        return;
    }
    publish_f64(&a.wmi[w], mi);
    atomicExch(&a.wflags[w], fl);
    wait_returned();
    uint32_t prev = atomicAdd(&a.qdone[q], 1u);
    if (prev + 1u == qd.nwin) {
        double m3[3];
        uint32_t f3[3];
        for (int r = 0; r < 3; ++r) {
            m3[r] = fetch_f64(&a.wmi[qd.win0 + r]);
            f3[r] = atomicAdd(&a.wflags[qd.win0 + r], 0u);
        }
        store_result(a, q, compose_result(qd, m3, f3));
    }
}

// window_estimate with psi(k) and psi(m) already at hand (fetched when the
// item starts): the same expression, so the same rounding.
template <int K>
__device__ __forceinline__ double estimate_from(uint32_t est, double psi_k, double psi_m, int m, long long S)
{
    double Sd = (double)S * 0x1p-44;
    if (est == 0)
        return (psi_k - 1.0 / (double)K + psi_m) - Sd / (double)m;
    return (psi_k + psi_m) - Sd / (double)m;
}

template <int K>
__device__ __forceinline__ double window_estimate(const LaunchArgs &a, int m, long long S)
{
    double Sd = (double)S * 0x1p-44;
    if (a.estimator == 0)
        return (a.psi_d[K] - 1.0 / (double)K + a.psi_d[m]) - Sd / (double)m;
    return (a.psi_d[K] + a.psi_d[m]) - Sd / (double)m;
}

// Radii of one query (grid units) from the keys of its k neighbours; the
// neighbours' coordinates are read back from the window's keys in LDS.
template <int K, typename T>
__device__ __forceinline__ void radii_k(const T (&nbk)[K], int shift, uint32_t mask, int m, const uint32_t *cand,
                                        uint32_t base, uint32_t qx, uint32_t qy, int dshift, uint32_t est,
                                        uint32_t &rx, uint32_t &ry)
{
    if (est == 0) {
        // in key units: coordinates carry dshift zero bits, so the distance
        // is shifted back once at the end
        uint32_t ex = 0, ey = 0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const uint32_t jj = min((uint32_t)(nbk[r] & (T)mask), (uint32_t)(m - 1));
            const uint2 c = reinterpret_cast<const uint2 *>(cand)[base + jj];
            ex = tmax(ex, sad_key(qx, c.x, 0u));
            ey = tmax(ey, sad_key(qy, c.y, 0u));
        }
        rx = ex >> dshift;
        ry = ey >> dshift;
    } else {
        rx = (uint32_t)(nbk[K - 1] >> shift);
        ry = rx;
    }
}

// Same from the k+1 smallest keys of a scan that included the point itself
// (its key is self: distance 0, index i), which is dropped first.
template <int K, typename T>
__device__ __forceinline__ void radii_from_keys(const T (&top)[K + 1], T self, int shift, uint32_t mask, int m,
                                                const uint32_t *cand, uint32_t base, uint32_t qx, uint32_t qy,
                                                int dshift, uint32_t est, uint32_t &rx, uint32_t &ry)
{
    T nbk[K];
#pragma unroll
    for (int r = 0; r < K; ++r)
        nbk[r] = top[r] < self ? top[r] : top[r + 1];
    radii_k<K, T>(nbk, shift, mask, m, cand, base, qx, qy, dshift, est, rx, ry);
}

// --------------------------------------------------------------------------
// split items: one block of up to 512 query points of a large window
// --------------------------------------------------------------------------

// Window extrema and grid check, computed by the workgroup (every item of a
// window computes the same values).
__device__ WinAux window_aux(const WinDesc &d, int32_t *s_red)
{
    const int tid = threadIdx.x;
    const int m = (int)d.m;
    if (tid == 0) {
        s_red[0] = INT32_MAX;
        s_red[1] = INT32_MIN;
        s_red[2] = INT32_MAX;
        s_red[3] = INT32_MIN;
        s_red[4] = 0;
    }
    block_sync();
    int32_t mnx = INT32_MAX, mxx = INT32_MIN, mny = INT32_MAX, mxy = INT32_MIN;
    uint32_t off = 0;
    for (int i0 = tid; i0 < m; i0 += kLoadBatch * kBlock) {
        float vx[kLoadBatch], vy[kLoadBatch];
#pragma unroll
        for (int g = 0; g < kLoadBatch; ++g) {
            const int i = i0 + g * kBlock < m ? i0 + g * kBlock : i0;  // past the end: a repeat
            vx[g] = d.x[i];
            vy[g] = d.y[i];
        }
#pragma unroll
        for (int g = 0; g < kLoadBatch; ++g) {
            const int32_t xi = grid_int(vx[g], off), yi = grid_int(vy[g], off);
            mnx = min(mnx, xi);
            mxx = max(mxx, xi);
            mny = min(mny, yi);
            mxy = max(mxy, yi);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mnx = min(mnx, __shfl_xor(mnx, o, 64));
        mxx = max(mxx, __shfl_xor(mxx, o, 64));
        mny = min(mny, __shfl_xor(mny, o, 64));
        mxy = max(mxy, __shfl_xor(mxy, o, 64));
        off |= (uint32_t)__shfl_xor((int)off, o, 64);
    }
    if ((tid & 63) == 0) {
        atomicMin(&s_red[0], mnx);
        atomicMax(&s_red[1], mxx);
        atomicMin(&s_red[2], mny);
        atomicMax(&s_red[3], mxy);
        if (off)
            atomicOr(&s_red[4], 1);
    }
    block_sync();
    WinAux ax;
    ax.min_x = s_red[0];
    ax.min_y = s_red[2];
    const uint32_t rx = (uint32_t)(s_red[1] - s_red[0]);
    const uint32_t ry = (uint32_t)(s_red[3] - s_red[2]);
    const uint32_t nb = ceil_log2((uint32_t)(m > 1 ? m : 2));
    // 32-bit keys need (range << nb) + j < 2^32
    ax.nb = (((rx | ry) >> (32 - nb)) == 0u) ? nb : 0u;
    ax.range_x = rx;
    ax.range_y = ry;
    ax.flags = s_red[4] ? kFlagOffGrid : 0u;
    block_sync();
    return ax;
}

// Wait until window w's sorted data is in HBM and return the window's
// constants: nb and the off-grid flag from its ready word, min_y as the first
// sorted y integer, min_x from the point that starts the x order (or the
// first sorted x integer with 64-bit keys).  The prep item has a lower index
// than every split item, so a running workgroup already holds it and it waits
// on nothing: the wait ends.  A poll limit turns a broken dependency into an
// error report instead of a hang.
__device__ WinAux split_window_aux(const LaunchArgs &a, uint32_t w, const WinDesc &d, int32_t *s_red)
{
    if (threadIdx.x == 0) {
        uint32_t polls = 0, v;
        while ((v = atomicAdd(&a.ready[w], 0u)) == 0u) {
            if (++polls >= kWaitLimit) {
                atomicOr(a.err, kErrWait);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        s_red[0] = (int32_t)v;
    }
    block_sync();
    // acquire only (the reader has nothing to release): later loads see
    // the prep item's stores
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const uint32_t v = (uint32_t)s_red[0];
    const int m = (int)d.m;
    const int32_t *base = a.sorted + (uint64_t)kSortedWords * d.sorted_off;
    WinAux ax;
    ax.nb = (v >> kReadyNbShift) & 31u;
    ax.flags = (v & kReadyOffGrid) ? kFlagOffGrid : 0u;
    ax.min_y = base[2 * m];
    if (ax.nb) {
        uint32_t off = 0;
        ax.min_x = grid_int(d.x[(uint32_t)base[0] & ((1u << ax.nb) - 1u)], off);
    } else {
        ax.min_x = base[0];
    }
    ax.range_x = ax.range_y = 0u;  // not needed by split items
    block_sync();  // s_red is reused
    return ax;
}

constexpr int kChunk = 2048;  // candidates (and sorted-marginal entries) staged in LDS at a time

// (X - min) << nb for point i of a window: a 32-bit key coordinate (nb > 0)
// or the offset grid integer (nb == 0, 64-bit key path).
__device__ __forceinline__ uint32_t key_coord(const float *v, int i, int32_t mn, uint32_t nb)
{
    uint32_t off = 0;
    return (uint32_t)(grid_int(v[i], off) - mn) << nb;
}

// Scan candidates [c0, c0 + cn) (LDS holds their grid-integer pairs) with
// 64-bit keys (d << 12 | j) into (k+1)-entry lists.
template <int K, int Q>
__device__ __forceinline__ void scan_wide(const uint32_t *__restrict__ cand, int c0, int cn,
                                          const uint32_t (&qx)[Q], const uint32_t (&qy)[Q],
                                          unsigned long long (&top)[Q][K + 1])
{
    constexpr int S = K + 1;
    for (int j = 0; j < cn; ++j) {
        const uint32_t cx = cand[2 * j], cy = cand[2 * j + 1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t d = tmax(sad_u32(qx[q], cx, 0u), sad_u32(qy[q], cy, 0u));
            unsigned long long key = ((unsigned long long)d << 12) | (unsigned long long)(c0 + j);
            if (key < top[q][S - 1])
                insert_sorted<S>(top[q], key);
        }
    }
}

// Radii of a query from the keys of its k neighbours; neighbour coordinates
// are re-read from the series (k loads per dimension).
template <int K, typename T>
__device__ __forceinline__ void split_radii_k(const T (&nbk)[K], int shift, uint32_t mask, const WinDesc &d,
                                              const WinAux &ax, uint32_t qx, uint32_t qy, uint32_t est,
                                              uint32_t &rx, uint32_t &ry)
{
    const uint32_t nb = ax.nb;
    if (est == 0) {
        uint32_t ex = 0, ey = 0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int jj = (int)min((uint32_t)(nbk[r] & (T)mask), d.m - 1u);
            ex = tmax(ex, sad_u32(qx, key_coord(d.x, jj, ax.min_x, nb), 0u) >> nb);
            ey = tmax(ey, sad_u32(qy, key_coord(d.y, jj, ax.min_y, nb), 0u) >> nb);
        }
        rx = ex;
        ry = ey;
    } else {
        rx = (uint32_t)(nbk[K - 1] >> shift);
        ry = rx;
    }
}

// Same from the k+1 smallest keys of a scan that included the point itself.
template <int K, typename T>
__device__ __forceinline__ void split_radii(const T (&top)[K + 1], T self, int shift, uint32_t mask,
                                            const WinDesc &d, const WinAux &ax, uint32_t qx, uint32_t qy,
                                            uint32_t est, uint32_t &rx, uint32_t &ry)
{
    T nbk[K];
#pragma unroll
    for (int r = 0; r < K; ++r)
        nbk[r] = top[r] < self ? top[r] : top[r + 1];
    split_radii_k<K, T>(nbk, shift, mask, d, ax, qx, qy, est, rx, ry);
}

// Split item of a window whose value range needs 64-bit keys (nb == 0): Q
// query points per thread (points q0 + tid + q * kBlock), all m candidates
// streamed through LDS as grid integers, then counts over the sorted
// marginals.
template <int K, int Q>
__device__ __forceinline__ long long split_body_wide(const LaunchArgs &a, uint32_t w, const WinDesc &d,
                                                     const WinAux &ax, int q0, uint32_t *buf)
{
    constexpr int S = K + 1;
    const int m = (int)d.m;
    const int tid = threadIdx.x;
    uint32_t qx[Q], qy[Q], rx[Q], ry[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = min(q0 + tid + q * kBlock, m - 1);
        qx[q] = key_coord(d.x, i, ax.min_x, 0u);
        qy[q] = key_coord(d.y, i, ax.min_y, 0u);
    }
    // ---- neighbours: candidates stream through LDS in chunks
    unsigned long long top[Q][S];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int r = 0; r < S; ++r)
            top[q][r] = ~0ull;
    for (int c0 = 0; c0 < m; c0 += kChunk) {
        const int cn = min(kChunk, m - c0);
        block_sync();
        for (int i = tid; i < cn; i += kBlock) {
            buf[2 * i] = key_coord(d.x, c0 + i, ax.min_x, 0u);
            buf[2 * i + 1] = key_coord(d.y, c0 + i, ax.min_y, 0u);
        }
        block_sync();
        scan_wide<K, Q>(buf, c0, cn, qx, qy, top);
    }
    {
        int n_live = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            n_live += __popcll(__ballot(q0 + tid + q * kBlock < m));
        count_evals(a, n_live, m - 1);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
        split_radii<K, unsigned long long>(top[q], (unsigned long long)min(q0 + tid + q * kBlock, m - 1), 12,
                                           0xFFFu, d, ax, qx[q], qy[q], a.estimator, rx[q], ry[q]);
    // ---- marginal counts over the sorted marginals, chunk by chunk
    int32_t xi[Q], yi[Q];
    int hx[Q], lx[Q], hy[Q], ly[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        xi[q] = (int32_t)qx[q] + ax.min_x;
        yi[q] = (int32_t)qy[q] + ax.min_y;
        hx[q] = lx[q] = hy[q] = ly[q] = 0;
    }
    const int32_t *src = a.sorted + (uint64_t)kSortedWords * d.sorted_off;
    int32_t *sx = reinterpret_cast<int32_t *>(buf);
    int32_t *sy = sx + kChunk;
    int32_t vx[2 * Q], vy[2 * Q];
#pragma unroll
    for (int q = 0; q < Q; ++q)
        count_bounds(a.estimator, xi[q], yi[q], (int32_t)rx[q], (int32_t)ry[q], vx + 2 * q, vy + 2 * q);
    for (int c0 = 0; c0 < m; c0 += kChunk) {
        const int cn = min(kChunk, m - c0);
        block_sync();
        for (int i = tid; i < cn; i += kBlock) {
            sx[i] = src[c0 + i];
            sy[i] = src[2 * m + c0 + i];
        }
        block_sync();
        int cxs[2 * Q], cys[2 * Q];
        count_lt_xy<2 * Q>(sx, sy, cn, vx, vy, cxs, cys);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            hx[q] += cxs[2 * q];
            lx[q] += cxs[2 * q + 1];
            hy[q] += cys[2 * q];
            ly[q] += cys[2 * q + 1];
        }
    }
    long long part = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = q0 + tid + q * kBlock;
        if (i >= m)
            continue;
        int cx, cy;
        part += point_terms(a, hx[q], lx[q], hy[q], ly[q], (int32_t)rx[q], cx, cy);
        if (a.dbg_nx) {
            a.dbg_nx[i] = (uint32_t)cx;
            a.dbg_ny[i] = (uint32_t)cy;
            a.dbg_ex[i] = (float)rx[q] * (1.0f / 4096.0f);
            a.dbg_ey[i] = (float)ry[q] * (1.0f / 4096.0f);
        }
    }
    return part;
}

// --------------------------------------------------------------------------
// split items over the x order: neighbours by an outward scan
// --------------------------------------------------------------------------
// A split item takes 512 consecutive positions of its window's x order, two
// adjacent ones per thread, so a wave holds 128 queries adjacent in x.  Each
// wave scans candidates in x order: its own block first (the queries' own
// points masked), then outwards, a chunk to the right and a chunk to the left
// in turn.  A candidate with |dx| larger than a query's current k-th distance
// cannot enter its list, and |dx| only grows further out, so a side stops once
// every query of the wave is past that point; the k smallest keys, and so the
// results, are those of the full scan.  Candidates travel through a private
// LDS chunk of the wave as (Ux, Uy, index); no workgroup barrier is involved.
constexpr int kWaveChunk = 128;

__device__ __forceinline__ void stage_wave(uint4 *wb, const uint32_t *KX, const uint32_t *YS, int c0, int cnt,
                                           uint32_t mask)
{
    const int lane = threadIdx.x & 63;
    asm volatile("" ::: "memory");
    static_assert(kWaveChunk == 128, "two candidates per lane");
    uint32_t key[2], ys[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int i = lane + 64 * g < cnt ? lane + 64 * g : 0;  // cnt >= 1
        key[g] = KX[c0 + i];
        ys[g] = YS[c0 + i];
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
        if (lane + 64 * g < cnt)
            wb[lane + 64 * g] = make_uint4(key[g] & ~mask, ys[g], key[g] & mask, 0u);
    // the chunk is written by the whole wave before any lane reads it
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
}

template <int K, bool SELF>
__device__ __forceinline__ void scan_wave(const uint4 *__restrict__ wb, int cnt, const uint32_t (&qx)[2],
                                          const uint32_t (&qy)[2], const uint32_t (&qj)[2], uint32_t (&top)[2][K])
{
    // four candidates a step: their LDS reads are in flight together
    int i = 0;
    for (; i + 4 <= cnt; i += 4) {
        uint4 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            c[u] = wb[i + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                uint32_t k = tmax(sad_key_v(qx[t], c[u].x, c[u].z), sad_key_v(qy[t], c[u].y, c[u].z));
                if (SELF)
                    k = c[u].z == qj[t] ? 0xFFFFFFFFu : k;
                insert_sorted<K>(top[t], k);
            }
        }
    }
    for (; i < cnt; ++i) {
        const uint4 c = wb[i];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            uint32_t k = tmax(sad_key_v(qx[t], c.x, c.z), sad_key_v(qy[t], c.y, c.z));
            if (SELF)
                k = c.z == qj[t] ? 0xFFFFFFFFu : k;
            insert_sorted<K>(top[t], k);
        }
    }
}

// Does some live query of the wave still need candidates at x-distance
// dist[t] (in key units) on a side?  dist > (k-th key | mask) means its
// distance exceeds the k-th neighbour's.
template <int K>
__device__ __forceinline__ bool side_open(const bool (&live)[2], const uint32_t (&dist)[2], const uint32_t (&top)[2][K],
                                          uint32_t mask)
{
    bool need = false;
#pragma unroll
    for (int t = 0; t < 2; ++t)
        need = need || (live[t] && dist[t] <= (top[t][K - 1] | mask));
    return __ballot(need) != 0ull;
}

// #{S[0..n) < v} for ascending 32-bit keys (thresholds up to 2^32) and
// #{T[0..n) < u} for ascending integers, NX of each, interleaved.
template <int NX>
__device__ __forceinline__ void count_lt_keys(const uint32_t *sx, const int32_t *sy, int n, const uint64_t (&vx)[NX],
                                              const int32_t (&vy)[NX], int (&cx)[NX], int (&cy)[NX])
{
    int bx[NX], by[NX];
#pragma unroll
    for (int t = 0; t < NX; ++t)
        bx[t] = by[t] = 0;
    while (n > 1) {
        const int half = n >> 1;
        uint32_t ex[NX];
        int32_t ey[NX];
#pragma unroll
        for (int t = 0; t < NX; ++t) {
            ex[t] = sx[bx[t] + half];
            ey[t] = sy[by[t] + half];
        }
#pragma unroll
        for (int t = 0; t < NX; ++t) {
            bx[t] = (uint64_t)ex[t] < vx[t] ? bx[t] + half : bx[t];
            by[t] = ey[t] < vy[t] ? by[t] + half : by[t];
        }
        n -= half;
    }
#pragma unroll
    for (int t = 0; t < NX; ++t) {
        cx[t] = bx[t] + ((uint64_t)sx[bx[t]] < vx[t] ? 1 : 0);
        cy[t] = by[t] + (sy[by[t]] < vy[t] ? 1 : 0);
    }
}

// Key threshold of "X - min_x < v" for keys ((X - min_x) << nb) | i.
__device__ __forceinline__ uint64_t key_below(int64_t v, uint32_t nb)
{
    if (v <= 0)
        return 0ull;
    if (v >= (1ll << (32 - nb)))
        return 1ull << 32;
    return (uint64_t)v << nb;
}


// One straggler's scan of one side, by the whole wave: candidates from `edge`
// outwards (RIGHT: edge, edge + 1, ...; left: edge - 1, edge - 2, ...), 256
// a round, one per lane per group of 64, into per-lane k-lists.  `bound` is
// the query's current k-th key with the index bits set: a candidate whose x
// distance exceeds it cannot enter, nor can any further out, so the side ends
// after the round whose outermost candidate is past it.  Returns the
// candidates evaluated.
template <int K, bool RIGHT>
__device__ __forceinline__ int straggler_side(const uint32_t *__restrict__ KX, const uint32_t *__restrict__ YS,
                                              int edge, int m, uint32_t sx, uint32_t sy, uint32_t bound,
                                              uint32_t mask, uint32_t (&pt)[K])
{
    const int lane = threadIdx.x & 63;
    const int avail = RIGHT ? m - edge : edge;  // candidates on this side
    int done = 0;
    while (done < avail) {
        const int n = min(256, avail - done);
        uint32_t kx[4], ky[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int off = done + 64 * g + lane;
            const int o = min(off, done + n - 1);  // past the end: repeat the round's last candidate
            const int p = RIGHT ? edge + o : edge - 1 - o;
            kx[g] = KX[p];
            ky[g] = YS[p];
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t cx = kx[g] & ~mask, cj = kx[g] & mask;
            uint32_t key = tmax(sad_key_v(sx, cx, cj), sad_key_v(sy, ky[g], cj));
            key = 64 * g + lane < n ? key : 0xFFFFFFFFu;
            insert_sorted<K>(pt, key);
        }
        done += n;
        const int pf = RIGHT ? edge + done - 1 : edge - done;  // the outermost candidate so far
        const uint32_t fx = (uint32_t)__builtin_amdgcn_readfirstlane((int)(KX[pf] & ~mask));
        if ((RIGHT ? fx - sx : sx - fx) > bound)
            break;
    }
    return min(done, avail);
}

template <int K>
__device__ long long split_body_sorted(const LaunchArgs &a, uint32_t w, const WinDesc &d, const WinAux &ax, int q0,
                                       uint32_t *buf)
{
    const int m = (int)d.m;
    const int tid = threadIdx.x;
    const uint32_t nb = ax.nb, mask = (1u << nb) - 1u;
    const uint32_t *KX = reinterpret_cast<const uint32_t *>(a.sorted + (uint64_t)kSortedWords * d.sorted_off);
    const uint32_t *YS = KX + m;
    const int32_t *SY = reinterpret_cast<const int32_t *>(KX + 2 * m);
    uint32_t qx[2], qy[2], qj[2], top[2][K];
    bool live[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int p = q0 + 2 * tid + t;
        live[t] = p < m;
        const int pc = min(p, m - 1);
        const uint32_t key = KX[pc];
        qx[t] = key & ~mask;
        qj[t] = key & mask;
        qy[t] = YS[pc];
#pragma unroll
        for (int r = 0; r < K; ++r)
            top[t][r] = 0xFFFFFFFFu;
    }
    // ---- neighbours, wave by wave
    {
        const int wave = tid >> 6;
        const int lane = tid & 63;
        uint4 *wb = reinterpret_cast<uint4 *>(buf) + wave * kWaveChunk;
        const int w_lo = __builtin_amdgcn_readfirstlane(q0 + 128 * wave);
        if (w_lo < m) {
            const int w_hi = min(m, w_lo + 128);
            stage_wave(wb, KX, YS, w_lo, w_hi - w_lo, mask);
            scan_wave<K, true>(wb, w_hi - w_lo, qx, qy, qj, top);
            int scanned = w_hi - w_lo;
            // x keys of the outermost candidates scanned on each side
            uint32_t er = wb[w_hi - w_lo - 1].x, el = wb[0].x;
            int r = w_hi, l = w_lo;
            bool nr[2], nl[2];
            for (;;) {
                // which queries can still gain from each side
                int needy = 0;
                bool any_r = false, any_l = false;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const uint32_t lim = top[t][K - 1] | mask;
                    nr[t] = live[t] && r < m && er - qx[t] <= lim;
                    nl[t] = live[t] && l > 0 && qx[t] - el <= lim;
                    needy += __popcll(__ballot(nr[t] || nl[t]));
                    any_r = any_r || __ballot(nr[t]) != 0ull;
                    any_l = any_l || __ballot(nl[t]) != 0ull;
                }
                // a few queries still open: they finish alone below
                // a few open slots left (the launch's threshold for this
                // window size): they finish one at a time below
                if (needy <= (int)a.strag[split_bucket((uint32_t)m)])
                    break;
                if (any_r) {
                    const int cnt = min(kWaveChunk, m - r);
                    stage_wave(wb, KX, YS, r, cnt, mask);
                    scan_wave<K, false>(wb, cnt, qx, qy, qj, top);
                    er = wb[cnt - 1].x;
                    r += cnt;
                    scanned += cnt;
                }
                if (any_l) {
                    const int cnt = min(kWaveChunk, l);
                    stage_wave(wb, KX, YS, l - cnt, cnt, mask);
                    scan_wave<K, false>(wb, cnt, qx, qy, qj, top);
                    el = wb[0].x;
                    l -= cnt;
                    scanned += cnt;
                }
            }
            const int n_live = __popcll(__ballot(live[0])) + __popcll(__ballot(live[1]));
            count_evals(a, n_live, scanned - 1);  // the own point is masked, not evaluated
            // stragglers, one at a time: the whole wave scans the sides the
            // query still needs, then merges the lanes' lists into its own
            unsigned long long s0 = __ballot(nr[0] || nl[0]), s1 = __ballot(nr[1] || nl[1]);
            while ((s0 | s1) != 0ull) {
                const int t = s0 != 0ull ? 0 : 1;
                const int L = __ffsll((long long)(t == 0 ? s0 : s1)) - 1;
                if (t == 0)
                    s0 &= s0 - 1ull;
                else
                    s1 &= s1 - 1ull;
                const uint32_t sx = __builtin_amdgcn_readlane(t == 0 ? qx[0] : qx[1], L);
                const uint32_t sy = __builtin_amdgcn_readlane(t == 0 ? qy[0] : qy[1], L);
                const uint32_t bound =
                    __builtin_amdgcn_readlane(t == 0 ? top[0][K - 1] : top[1][K - 1], L) | mask;
                const int need_r = __builtin_amdgcn_readlane((int)(t == 0 ? nr[0] : nr[1]), L);
                const int need_l = __builtin_amdgcn_readlane((int)(t == 0 ? nl[0] : nl[1]), L);
                uint32_t pt[K];
#pragma unroll
                for (int q = 0; q < K; ++q)
                    pt[q] = 0xFFFFFFFFu;
                int cand = 0;
                if (need_r)
                    cand += straggler_side<K, true>(KX, YS, r, m, sx, sy, bound, mask, pt);
                if (need_l)
                    cand += straggler_side<K, false>(KX, YS, l, m, sx, sy, bound, mask, pt);
                // after the butterfly every lane holds the k smallest of all lists
                for (int o = 32; o > 0; o >>= 1) {
                    uint32_t other[K];
#pragma unroll
                    for (int q = 0; q < K; ++q)
                        other[q] = (uint32_t)__shfl_xor((int)pt[q], o, 64);
#pragma unroll
                    for (int q = 0; q < K; ++q)
                        insert_sorted<K>(pt, other[q]);
                }
                if (lane == L) {
#pragma unroll
                    for (int q = 0; q < K; ++q) {
                        if (t == 0)
                            insert_sorted<K>(top[0], pt[q]);
                        else
                            insert_sorted<K>(top[1], pt[q]);
                    }
                }
                count_evals(a, 1, cand);
            }
        }
    }
    uint32_t rx[2], ry[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
        split_radii_k<K, uint32_t>(top[t], (int)nb, mask, d, ax, qx[t], qy[t], a.estimator, rx[t], ry[t]);
    // ---- marginal counts: x over the keys, y over the sorted integers
    uint64_t vx[4];
    int32_t vy[4];
    const int64_t o = a.estimator == 0 ? 1 : 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int64_t xr = (int64_t)(qx[t] >> nb), e = (int64_t)rx[t];
        vx[2 * t] = key_below(xr + e + o, nb);
        vx[2 * t + 1] = key_below(xr - e + 1 - o, nb);
        const int32_t yi = (int32_t)(qy[t] >> nb) + ax.min_y, ey = (int32_t)ry[t];
        vy[2 * t] = yi + ey + (int32_t)o;
        vy[2 * t + 1] = yi - ey + 1 - (int32_t)o;
    }
    int hx[2] = {0, 0}, lx[2] = {0, 0}, hy[2] = {0, 0}, ly[2] = {0, 0};
    uint32_t *sx = buf;
    int32_t *sy = reinterpret_cast<int32_t *>(buf + kChunk);
    for (int c0 = 0; c0 < m; c0 += kChunk) {
        const int cn = min(kChunk, m - c0);
        block_sync();
        for (int i0 = tid; i0 < cn; i0 += kLoadBatch * kBlock) {
            uint32_t kx[kLoadBatch];
            int32_t ky[kLoadBatch];
#pragma unroll
            for (int g = 0; g < kLoadBatch; ++g) {
                const int i = i0 + g * kBlock < cn ? i0 + g * kBlock : i0;
                kx[g] = KX[c0 + i];
                ky[g] = SY[c0 + i];
            }
#pragma unroll
            for (int g = 0; g < kLoadBatch; ++g) {
                if (i0 + g * kBlock < cn) {
                    sx[i0 + g * kBlock] = kx[g];
                    sy[i0 + g * kBlock] = ky[g];
                }
            }
        }
        block_sync();
        int cxs[4], cys[4];
        count_lt_keys<4>(sx, sy, cn, vx, vy, cxs, cys);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            hx[t] += cxs[2 * t];
            lx[t] += cxs[2 * t + 1];
            hy[t] += cys[2 * t];
            ly[t] += cys[2 * t + 1];
        }
    }
    long long part = 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!live[t])
            continue;
        int cx, cy;
        part += point_terms(a, hx[t], lx[t], hy[t], ly[t], (int32_t)rx[t], cx, cy);
        if (a.dbg_nx) {
            a.dbg_nx[qj[t]] = (uint32_t)cx;
            a.dbg_ny[qj[t]] = (uint32_t)cy;
            a.dbg_ex[qj[t]] = (float)rx[t] * (1.0f / 4096.0f);
            a.dbg_ey[qj[t]] = (float)ry[t] * (1.0f / 4096.0f);
        }
    }
    return part;
}

template <int K>
__device__ void split_item(const LaunchArgs &a, uint32_t w, int q0, uint32_t *buf, long long *s_part,
                           int32_t *s_red)
{
    const WinDesc d = a.win[w];
    const WinAux ax = split_window_aux(a, w, d, s_red);
    const int m = (int)d.m;
    const int tid = threadIdx.x;
    long long part = 0;
    if (m > K) {
        if (ax.nb)
            part = split_body_sorted<K>(a, w, d, ax, q0, buf);
        else if (m - q0 <= kBlock)
            part = split_body_wide<K, 1>(a, w, d, ax, q0, buf);
        else
            part = split_body_wide<K, 2>(a, w, d, ax, q0, buf);
    }
    // workgroup sum of the fixed-point terms (exact, order-free)
    for (int o = 32; o > 0; o >>= 1)
        part += __shfl_xor(part, o, 64);
    if ((tid & 63) == 0)
        s_part[tid >> 6] = part;
    block_sync();
    if (tid == 0) {
        long long tot = 0;
        for (int wv = 0; wv < kBlock / 64; ++wv)
            tot += s_part[wv];
        if (m > K)
            atomicAdd(&a.acc[w], (unsigned long long)tot);
        wait_returned();
        uint32_t prev = atomicAdd(&a.wdone[w], 1u);
        if (prev + 1u == d.n_items) {
            double mi;
            uint32_t fl = ax.flags;
            if (m <= K) {
                mi = __builtin_nan("");
                fl |= kFlagTooShort;
            } else {
                long long S = (long long)atomicAdd(&a.acc[w], 0ull);
                mi = window_estimate<K>(a, m, S);
            }
            a.wmi[w] = mi;
            a.wflags[w] = fl;
            report_window(a, w, d.query, mi, fl);
        }
    }
}

// --------------------------------------------------------------------------
// local items: up to 16 consecutive windows, all inside one workgroup
// --------------------------------------------------------------------------

// Digamma sums are split over this many LDS words per window, picked by the
// lane, so that the atomics of a wave's lanes meet at most 8-way on one word
// (the sum is exact integer arithmetic: the split changes nothing).
constexpr int kAccSplit = 8;

__device__ __forceinline__ unsigned long long acc_sum(const unsigned long long (&v)[kAccSplit])
{
    unsigned long long s = 0ull;
#pragma unroll
    for (int r = 0; r < kAccSplit; ++r)
        s += v[r];
    return s;
}

struct LocalShared {
    const float *x[kLocalWindows];
    const float *y[kLocalWindows];
    unsigned long long acc[kLocalWindows][kAccSplit];
    QDesc qd[kLocalWindows];      // each window's query, fetched when the item starts
    double psi_m[kLocalWindows];  // psi(m) of each window, likewise
    double psi_k;
    double mi[kLocalWindows];
    uint32_t off[kLocalWindows + 1];
    uint32_t m[kLocalWindows];
    uint32_t nb[kLocalWindows];
    uint32_t flags[kLocalWindows];
    uint32_t query[kLocalWindows];
    int32_t mn[2][kLocalWindows];
    int32_t mx[2][kLocalWindows];
    uint32_t P, log2P;
};

// Scan candidates [jlo, jhi) of one window (cand: its keys, two words per
// point, jlo even) for a thread's two consecutive query points (slot 2t and
// 2t+1: points self and self+1, self even) into S-entry lists t0, t1.
// MASKM: j >= m is padding beyond this lane's window (the loop runs to the
// wave's longest window); SELF: the queries' own points are masked (keys set
// to the maximum) so k-entry lists hold neighbours only.
template <int S, bool MASKM, bool SELF>
__device__ __forceinline__ void local_scan2(const uint32_t *__restrict__ cand, int jlo, int jhi, int m, uint32_t self,
                                            uint32_t qx0, uint32_t qy0, uint32_t qx1, uint32_t qy1,
                                            uint32_t (&t0)[S], uint32_t (&t1)[S])
{
    const uint4 *c4 = reinterpret_cast<const uint4 *>(cand);
    int j = jlo;
    for (; j + 1 < jhi; j += 2) {
        const uint4 c = c4[j >> 1];
        const uint32_t j0 = (uint32_t)j;
        uint32_t a0 = tmax(sad_key(qx0, c.x, j0), sad_key(qy0, c.y, j0));
        uint32_t a1 = tmax(sad_key(qx0, c.z, j0 + 1u), sad_key(qy0, c.w, j0 + 1u));
        uint32_t b0 = tmax(sad_key(qx1, c.x, j0), sad_key(qy1, c.y, j0));
        uint32_t b1 = tmax(sad_key(qx1, c.z, j0 + 1u), sad_key(qy1, c.w, j0 + 1u));
        if (MASKM) {
            a0 = (int)j0 < m ? a0 : 0xFFFFFFFFu;
            b0 = (int)j0 < m ? b0 : 0xFFFFFFFFu;
            a1 = (int)j0 + 1 < m ? a1 : 0xFFFFFFFFu;
            b1 = (int)j0 + 1 < m ? b1 : 0xFFFFFFFFu;
        }
        if (SELF) {
            // j0 even: only (query 0, j0 == self) and (query 1, j0 + 1 == self + 1)
            const bool hit = j0 == self;
            a0 = hit ? 0xFFFFFFFFu : a0;
            b1 = hit ? 0xFFFFFFFFu : b1;
        }
        insert_sorted<S>(t0, a0);
        insert_sorted<S>(t0, a1);
        insert_sorted<S>(t1, b0);
        insert_sorted<S>(t1, b1);
    }
    if (j < jhi) {
        const uint32_t cx = cand[2 * j], cy = cand[2 * j + 1], j0 = (uint32_t)j;
        uint32_t a0 = tmax(sad_key(qx0, cx, j0), sad_key(qy0, cy, j0));
        uint32_t b0 = tmax(sad_key(qx1, cx, j0), sad_key(qy1, cy, j0));
        if (MASKM) {
            a0 = (int)j0 < m ? a0 : 0xFFFFFFFFu;
            b0 = (int)j0 < m ? b0 : 0xFFFFFFFFu;
        }
        if (SELF) {
            a0 = j0 == self ? 0xFFFFFFFFu : a0;
            b0 = j0 == self + 1u ? 0xFFFFFFFFu : b0;
        }
        insert_sorted<S>(t0, a0);
        insert_sorted<S>(t1, b0);
    }
}

// Neighbour search of a thread's two slots inside a local item (points i0
// and i0 + 1 of the window at slot offset base).  Wave-uniform mode:
//   0  the whole wave is inside one window (32-bit keys): k-entry lists,
//      the points themselves masked inside the wave's band of 128 points
//   1  lanes in several windows of the same m (32-bit keys): k+1 entries,
//      the point itself dropped at the end
//   2  lanes in windows of different m (32-bit keys): as 1, candidates past
//      a lane's own window masked
//   3  some window needs 64-bit keys: one slot at a time
// m_loop is the wave's longest window; band0 (mode 0) its first point.
template <int K>
__device__ __forceinline__ void local_knn2(const uint32_t *__restrict__ cand, uint32_t base, int m, int i0,
                                           uint32_t nb, int mode, int m_loop, int band0, uint32_t est,
                                           uint32_t (&rx)[2], uint32_t (&ry)[2])
{
    constexpr int S = K + 1;
    const uint32_t *cw = cand + 2 * base;
    const uint32_t qx0 = cw[2 * i0], qy0 = cw[2 * i0 + 1];
    const uint32_t qx1 = cw[2 * i0 + 2], qy1 = cw[2 * i0 + 3];
    const uint32_t mask = (1u << nb) - 1u;
    if (mode == 0) {
        uint32_t t0[K], t1[K];
#pragma unroll
        for (int r = 0; r < K; ++r)
            t0[r] = t1[r] = 0xFFFFFFFFu;
        const int b1 = min(band0 + 128, m_loop);
        local_scan2<K, false, false>(cw, 0, band0, m, (uint32_t)i0, qx0, qy0, qx1, qy1, t0, t1);
        local_scan2<K, false, true>(cw, band0, b1, m, (uint32_t)i0, qx0, qy0, qx1, qy1, t0, t1);
        local_scan2<K, false, false>(cw, b1, m_loop, m, (uint32_t)i0, qx0, qy0, qx1, qy1, t0, t1);
        radii_k<K, uint32_t>(t0, (int)nb, mask, m, cand, base, qx0, qy0, (int)nb, est, rx[0], ry[0]);
        radii_k<K, uint32_t>(t1, (int)nb, mask, m, cand, base, qx1, qy1, (int)nb, est, rx[1], ry[1]);
    } else if (mode == 1 || mode == 2) {
        uint32_t t0[S], t1[S];
#pragma unroll
        for (int r = 0; r < S; ++r)
            t0[r] = t1[r] = 0xFFFFFFFFu;
        if (mode == 1)
            local_scan2<S, false, false>(cw, 0, m_loop, m, (uint32_t)i0, qx0, qy0, qx1, qy1, t0, t1);
        else
            local_scan2<S, true, false>(cw, 0, m_loop, m, (uint32_t)i0, qx0, qy0, qx1, qy1, t0, t1);
        radii_from_keys<K, uint32_t>(t0, (uint32_t)i0, (int)nb, mask, m, cand, base, qx0, qy0, (int)nb, est, rx[0],
                                     ry[0]);
        radii_from_keys<K, uint32_t>(t1, (uint32_t)i0 + 1u, (int)nb, mask, m, cand, base, qx1, qy1, (int)nb, est,
                                     rx[1], ry[1]);
    } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = i0 + q;
            unsigned long long top[S];
#pragma unroll
            for (int r = 0; r < S; ++r)
                top[r] = ~0ull;
            const uint32_t px = cw[2 * i] >> nb, py = cw[2 * i + 1] >> nb;
            for (int j = 0; j < m_loop; ++j) {
                uint32_t cx = cw[2 * j] >> nb, cy = cw[2 * j + 1] >> nb;
                uint32_t d = tmax(sad_u32(px, cx, 0u), sad_u32(py, cy, 0u));
                unsigned long long key = ((unsigned long long)d << 12) | (unsigned long long)j;
                if (j < m && key < top[S - 1])
                    insert_sorted<S>(top, key);
            }
            radii_from_keys<K, unsigned long long>(top, (unsigned long long)i, 12, 0xFFFu, m, cand, base,
                                                   cw[2 * i], cw[2 * i + 1], (int)nb, est, rx[q], ry[q]);
        }
    }
}

template <int K>
__device__ void local_item(const LaunchArgs &a, uint32_t w0, uint32_t nwin, uint32_t *buf, LocalShared &L)
{
    const int tid = threadIdx.x;
    uint32_t *cand = buf;                                       // 2 x 1024 words: keys, by slot
    int32_t *srt_x = reinterpret_cast<int32_t *>(buf + 2 * 1024);  // kLocalSort: sorted marginals
    int32_t *srt_y = srt_x + kLocalSort;

    // descriptors, each window's query and psi values (fetched now, so that
    // the results at the end wait on no load), and the window offsets: an
    // exclusive scan of the even-rounded sizes (even offsets keep 16-byte
    // candidate reads aligned) in the lanes of wave 0
    uint32_t vm = 0u;
    if (tid < (int)nwin) {
        const WinDesc d = a.win[w0 + tid];
        L.x[tid] = d.x;
        L.y[tid] = d.y;
        L.m[tid] = d.m;
        L.query[tid] = d.query;
        L.qd[tid] = a.qd[d.query];
        L.psi_m[tid] = a.psi_d[min(d.m, (uint32_t)kMaxWindow)];
        for (int r = 0; r < kAccSplit; ++r)
            L.acc[tid][r] = 0ull;
        L.flags[tid] = 0u;
        vm = d.m;
    }
    if (tid < 64) {
        static_assert(kLocalWindows <= 16, "one scan over 16 lanes");
        const uint32_t v = (vm + 1u) & ~1u;
        uint32_t incl = v, mmax = max(vm, 2u);
        for (int o = 1; o < 16; o <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 16);
            if ((tid & 15) >= o)
                incl += u;
            mmax = max(mmax, (uint32_t)__shfl_xor((int)mmax, o, 16));
        }
        if (tid < (int)nwin)
            L.off[tid] = incl - v;
        if (tid == (int)nwin - 1)
            L.off[nwin] = incl;
        if (tid == 0) {
            const uint32_t lp = ceil_log2(mmax);
            L.P = 1u << lp;
            L.log2P = lp;
            L.psi_k = a.psi_d[K];
        }
    }
    block_sync();
    const uint32_t total = L.off[nwin];
    const uint32_t P = L.P, lp = L.log2P;

    // ---- stage: grid integers into the sort segments, per-window extrema
    int32_t X[2], Y[2];
    uint32_t W[2];
    int I[2];
    bool act[2];
    // slots 2t and 2t+1: window offsets are even, so both lie in one window,
    // the number of later window starts at or below slot 2t
    uint32_t w_t = 0;
#pragma unroll
    for (int r = 1; r < kLocalWindows; ++r)
        w_t += (r < (int)nwin && L.off[r] <= 2u * (uint32_t)tid) ? 1u : 0u;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint32_t s = 2u * (uint32_t)tid + (uint32_t)q;
        const uint32_t w = w_t;
        const int i = (int)s - (int)L.off[w];
        act[q] = s < total && i < (int)L.m[w];
        W[q] = w;
        I[q] = act[q] ? i : 0;
        X[q] = 0;
        Y[q] = 0;
        if (act[q]) {
            uint32_t off = 0;
            X[q] = grid_int(L.x[w][i], off);
            Y[q] = grid_int(L.y[w][i], off);
            srt_x[(w << lp) + i] = X[q];
            srt_y[(w << lp) + i] = Y[q];
            if (off)
                atomicOr(&L.flags[w], kFlagOffGrid);
        }
    }
    for (uint32_t t = tid; t < (nwin << lp); t += kBlock) {
        const uint32_t w = t >> lp, i = t & (P - 1u);
        if (i >= L.m[w]) {
            srt_x[t] = INT32_MAX;
            srt_y[t] = INT32_MAX;
        }
    }
    block_sync();

    // ---- sort every window's marginals (segments of P, padded with INT32_MAX):
    // the counts search them, and their ends are the window's extrema
    sort_marginals(srt_x, srt_y, nwin << lp, P);
    if (tid < (int)nwin) {
        const uint32_t m = L.m[tid];
        const uint32_t last = m > 0u ? m - 1u : 0u;
        L.mn[0][tid] = srt_x[tid << lp];
        L.mx[0][tid] = srt_x[(tid << lp) + last];
        L.mn[1][tid] = srt_y[tid << lp];
        L.mx[1][tid] = srt_y[(tid << lp) + last];
        const uint32_t nb = ceil_log2(m > 1 ? m : 2u);
        const uint32_t rxr = (uint32_t)(L.mx[0][tid] - L.mn[0][tid]);
        const uint32_t ryr = (uint32_t)(L.mx[1][tid] - L.mn[1][tid]);
        L.nb[tid] = (((rxr | ryr) >> (32 - nb)) == 0u) ? nb : 0u;
    }
    block_sync();
    // ---- keys (or X - min for the 64-bit path), by slot
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (act[q]) {
            const uint32_t s = 2u * (uint32_t)tid + (uint32_t)q;
            const uint32_t w = W[q], nb = L.nb[w];
            cand[2 * s] = (uint32_t)(X[q] - L.mn[0][w]) << nb;
            cand[2 * s + 1] = (uint32_t)(Y[q] - L.mn[1][w]) << nb;
        }
    }
    block_sync();

    // ---- neighbours: one pass over the window for both slots of the thread
    uint32_t RX[2] = {0u, 0u}, RY[2] = {0u, 0u};
    {
        // slot 2t+1 is live only if slot 2t is (a pad slot is always the second)
        const bool live = act[0] && (int)L.m[W[0]] > K;
        const unsigned long long bal = __ballot(live);
        if (bal != 0ull) {  // wave-uniform
            // lanes without a live slot follow the first live lane's window
            const int first = __ffsll((long long)bal) - 1;
            const uint32_t lead_w = (uint32_t)__shfl((int)W[0], first, 64);
            const int lead_i = __shfl(I[0], first, 64);
            const uint32_t wl = live ? W[0] : lead_w;
            const int il = live ? I[0] : lead_i;
            const int m = (int)L.m[wl];
            const uint32_t nb = L.nb[wl];
            // wave-wide: one window?  same m everywhere?  any 64-bit window?
            // (against lane 0, which holds a live slot's window); slots rise
            // with the lane inside a window, so with one window the wave's
            // lowest slot is the first live lane's
            const bool one_win = __ballot(wl != (uint32_t)__builtin_amdgcn_readfirstlane((int)wl)) == 0ull;
            const bool one_m = __ballot(m != __builtin_amdgcn_readfirstlane(m)) == 0ull;
            const int mode = __ballot(nb == 0u) != 0ull ? 3 : (one_win ? 0 : (one_m ? 1 : 2));
            const int band0 = __builtin_amdgcn_readfirstlane(lead_i);
            int m_max = m;
            if (!one_m) {
                for (int o = 32; o > 0; o >>= 1)
                    m_max = max(m_max, __shfl_xor(m_max, o, 64));
            }
            m_max = __builtin_amdgcn_readfirstlane(m_max);
            local_knn2<K>(cand, L.off[wl], m, il, nb, mode, m_max, band0, a.estimator, RX, RY);
            // each live slot needs the m - 1 other points of its own window;
            // candidates a wave scans past a lane's window are padding
            count_evals_lanes(a, live ? (uint32_t)(m - 1) * (act[1] ? 2u : 1u) : 0u);
        }
    }
    block_sync();

    // ---- counts and digamma terms: both slots of a thread lie in one window,
    // so their eight searches run interleaved over the same sorted marginals
    if (act[0] && (int)L.m[W[0]] > K) {
        const uint32_t w = W[0];
        const int m = (int)L.m[w];
        int32_t vx[4], vy[4];
        int cxs[4], cys[4];
#pragma unroll
        for (int q = 0; q < 2; ++q)
            count_bounds(a.estimator, X[q], Y[q], (int32_t)RX[q], (int32_t)RY[q], vx + 2 * q, vy + 2 * q);
        count_lt_xy<4>(srt_x + (w << lp), srt_y + (w << lp), m, vx, vy, cxs, cys);
        long long t = 0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (!act[q])
                continue;
            int cx, cy;
            t += point_terms(a, cxs[2 * q], cxs[2 * q + 1], cys[2 * q], cys[2 * q + 1], (int32_t)RX[q], cx, cy);
            if (a.dbg_nx) {
                a.dbg_nx[I[q]] = (uint32_t)cx;
                a.dbg_ny[I[q]] = (uint32_t)cy;
                a.dbg_ex[I[q]] = (float)RX[q] * (1.0f / 4096.0f);
                a.dbg_ey[I[q]] = (float)RY[q] * (1.0f / 4096.0f);
            }
        }
        atomicAdd(&L.acc[w][tid & (kAccSplit - 1)], (unsigned long long)t);
    }
    block_sync();

    // ---- estimates, then results
    if (tid < (int)nwin) {
        const int m = (int)L.m[tid];
        uint32_t fl = L.flags[tid];
        double mi;
        if (m <= K) {
            mi = __builtin_nan("");
            fl |= kFlagTooShort;
        } else {
            mi = estimate_from<K>(a.estimator, L.psi_k, L.psi_m[tid], m, (long long)acc_sum(L.acc[tid]));
        }
        L.mi[tid] = mi;
        L.flags[tid] = fl;
        a.wmi[w0 + tid] = mi;
        a.wflags[w0 + tid] = fl;
    }
    block_sync();
    if (tid < (int)nwin) {
        const uint32_t w = w0 + tid, q = L.query[tid];
        const QDesc qd = L.qd[tid];
        const bool inside = qd.win0 >= w0 && qd.win0 + qd.nwin <= w0 + nwin;
        if (inside) {
            if (qd.win0 == w)
                store_result(a, q, compose_result(qd, &L.mi[tid], &L.flags[tid]));
        } else {
            report_window(a, w, q, L.mi[tid], L.flags[tid]);
        }
    }
}

// --------------------------------------------------------------------------
// triple items: noise triples evaluated through their union
// --------------------------------------------------------------------------
// The base w_o and the extension w_d of a noise triple partition its union
// w'' (Definition 6.2 as applied in Section 6.2).  A point's k nearest
// neighbours inside its own part are the k smallest keys among that part's
// candidates, and the k smallest of a set do not depend on the order they
// are inserted in, so one scan over the union gives both of a point's lists:
// the base's candidates first, after which a base point's list is its base
// list (kept), then the extension's, which complete every union list and,
// inserted into a second list, give an extension point its extension list.
// A triple costs the distances of its union only.
//
// Counts inside a part: with S the smaller part, a point of S counts over S
// by brute force; a point of the other part counts over the union (binary
// searches in the sorted union marginals, as the union's own counts) and
// subtracts its count over S.  Up to kTripleMax triples (whole queries) with
// at most kLocalSlots union points in total share a workgroup.

struct TripleShared {
    const float *x[kTripleMax];
    const float *y[kTripleMax];
    uint32_t off[kTripleMax + 1];             // first slot of each union (even)
    uint32_t m[kTripleMax];                   // union points
    uint32_t a0[kTripleMax], na[kTripleMax];  // base part [a0, a0 + na) of the union
    uint32_t b0[kTripleMax], nb[kTripleMax];  // extension part [b0, b0 + nb)
    uint32_t bits[kTripleMax];                // index bits of 32-bit keys; 0: 64-bit keys
    uint32_t flags[kTripleMax];
    int32_t mn[2][kTripleMax];
    int32_t mx[2][kTripleMax];
    unsigned long long acc[kTripleMax][3][kAccSplit];  // base, extension, union
    QDesc qd[kTripleMax];                     // each triple's query, fetched when the item starts
    double psi[kTripleMax][4];                // psi(k), psi of the base, extension and union sizes
    uint32_t query[kTripleMax];
    uint32_t P, log2P;
    uint32_t njobs;                           // part counts handed to other threads
};

// Part counts of the larger part's points whose part radii differ from their
// union radii (their part list lost a neighbour to the other part) are
// searched by other threads, one job per thread: four words per job (the
// point as t | i << 8, its part radii; then its four counts), in the LDS words
// the union keys leave free.  The other points reuse their union counts.
constexpr int kTripJobs = kBlock;

// Scan candidates j = j0 + jj, jj in [0, n), of a thread's union (cw: its
// keys, two words per point) for the thread's two query points into the
// S-entry union lists u0, u1; with PART the keys also enter the part lists
// p0, p1 of the queries whose in0 / in1 is set.  MASK: jj >= n_lane is past
// this lane's range (the wave's loop runs to its longest range) and j0 is
// per lane; otherwise j0 and n are wave-uniform.
template <int S, bool MASK, bool PART>
__device__ __forceinline__ void trip_scan(const uint32_t *__restrict__ cw, int j0, int n, int n_lane, uint32_t qx0,
                                          uint32_t qy0, uint32_t qx1, uint32_t qy1, bool in0, bool in1,
                                          uint32_t (&u0)[S], uint32_t (&u1)[S], uint32_t (&p0)[S], uint32_t (&p1)[S])
{
    const uint2 *c2 = reinterpret_cast<const uint2 *>(cw);
    const int jlast = j0 + n_lane - 1;  // MASK: reads past the lane's range stay on its last candidate
    int jj = 0;
    for (; jj + 4 <= n; jj += 4) {
        uint2 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            c[u] = c2[MASK ? min(j0 + jj + u, jlast) : j0 + jj + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t j = (uint32_t)(j0 + jj + u);
            uint32_t k0, k1;
            if (MASK) {
                k0 = tmax(sad_key_v(qx0, c[u].x, j), sad_key_v(qy0, c[u].y, j));
                k1 = tmax(sad_key_v(qx1, c[u].x, j), sad_key_v(qy1, c[u].y, j));
                k0 = jj + u < n_lane ? k0 : 0xFFFFFFFFu;
                k1 = jj + u < n_lane ? k1 : 0xFFFFFFFFu;
            } else {
                k0 = tmax(sad_key(qx0, c[u].x, j), sad_key(qy0, c[u].y, j));
                k1 = tmax(sad_key(qx1, c[u].x, j), sad_key(qy1, c[u].y, j));
            }
            insert_sorted<S>(u0, k0);
            insert_sorted<S>(u1, k1);
            if (PART) {
                insert_sorted<S>(p0, in0 ? k0 : 0xFFFFFFFFu);
                insert_sorted<S>(p1, in1 ? k1 : 0xFFFFFFFFu);
            }
        }
    }
    for (; jj < n; ++jj) {
        const uint2 c = c2[MASK ? min(j0 + jj, jlast) : j0 + jj];
        const uint32_t j = (uint32_t)(j0 + jj);
        uint32_t k0, k1;
        if (MASK) {
            k0 = tmax(sad_key_v(qx0, c.x, j), sad_key_v(qy0, c.y, j));
            k1 = tmax(sad_key_v(qx1, c.x, j), sad_key_v(qy1, c.y, j));
            k0 = jj < n_lane ? k0 : 0xFFFFFFFFu;
            k1 = jj < n_lane ? k1 : 0xFFFFFFFFu;
        } else {
            k0 = tmax(sad_key(qx0, c.x, j), sad_key(qy0, c.y, j));
            k1 = tmax(sad_key(qx1, c.x, j), sad_key(qy1, c.y, j));
        }
        insert_sorted<S>(u0, k0);
        insert_sorted<S>(u1, k1);
        if (PART) {
            insert_sorted<S>(p0, in0 ? k0 : 0xFFFFFFFFu);
            insert_sorted<S>(p1, in1 ? k1 : 0xFFFFFFFFu);
        }
    }
}

// The same with 64-bit keys (d << 12 | j), one query point, for unions whose
// value range does not fit 32-bit keys.
template <int S>
__device__ __forceinline__ void trip_scan_wide(const uint32_t *__restrict__ cw, int j0, int n, uint32_t qx, uint32_t qy,
                                               bool in, bool part, unsigned long long (&u)[S],
                                               unsigned long long (&p)[S])
{
    for (int jj = 0; jj < n; ++jj) {
        const uint32_t j = (uint32_t)(j0 + jj);
        const uint32_t d = tmax(sad_u32(qx, cw[2 * j], 0u), sad_u32(qy, cw[2 * j + 1], 0u));
        const unsigned long long key = ((unsigned long long)d << 12) | (unsigned long long)j;
        insert_sorted<S>(u, key);
        if (part)
            insert_sorted<S>(p, in ? key : ~0ull);
    }
}

// #{j in [s0, s0 + ns) of the union : |c_i - c_j| <= e} (estimator 0) or
// < e (estimator 1) in both coordinates, from the union's keys (key units:
// coordinates shifted left by the index bits, e likewise).
__device__ __forceinline__ void trip_count_part(const uint32_t *__restrict__ cw, int s0, int ns, uint32_t qx,
                                                uint32_t qy, uint32_t ex, uint32_t ey, uint32_t est, int &cx, int &cy)
{
    // |d| < e is |d| + 1 <= e on integers: the absolute difference carries
    // the 1 for estimator 1 (no wrap: key coordinates stay below 2^32 - 1)
    const uint32_t o = est == 0 ? 0u : 1u;
    const uint2 *c2 = reinterpret_cast<const uint2 *>(cw);
    int nx = 0, ny = 0;
    for (int j = s0; j < s0 + ns; ++j) {
        const uint2 c = c2[j];
        nx += sad_key(qx, c.x, o) <= ex ? 1 : 0;
        ny += sad_key(qy, c.y, o) <= ey ? 1 : 0;
    }
    cx = nx;
    cy = ny;
}

template <int K>
__device__ void triple_item(const LaunchArgs &a, uint32_t w0, uint32_t ntrip, uint32_t *buf, TripleShared &T)
{
    constexpr int S = K + 1;
    const int tid = threadIdx.x;
    uint32_t *cand = buf;                                          // keys, two words per union point
    int32_t *srt_x = reinterpret_cast<int32_t *>(buf + 2 * 1024);  // sorted union marginals
    int32_t *srt_y = srt_x + kLocalSort;

    if (tid < (int)ntrip) {
        const uint32_t wb = w0 + 3u * (uint32_t)tid;  // base, extension, union
        const WinDesc db = a.win[wb], de = a.win[wb + 1], du = a.win[wb + 2];
        T.x[tid] = du.x;
        T.y[tid] = du.y;
        T.m[tid] = du.m;
        T.a0[tid] = (uint32_t)(db.x - du.x);
        T.na[tid] = db.m;
        T.b0[tid] = (uint32_t)(de.x - du.x);
        T.nb[tid] = de.m;
        T.flags[tid] = 0u;
        // the query and the psi values of its three sizes, fetched now so
        // that the result at the end waits on no load
        T.query[tid] = db.query;
        T.qd[tid] = a.qd[db.query];
        T.psi[tid][0] = a.psi_d[K];
        T.psi[tid][1] = a.psi_d[min(db.m, (uint32_t)kMaxWindow)];
        T.psi[tid][2] = a.psi_d[min(de.m, (uint32_t)kMaxWindow)];
        T.psi[tid][3] = a.psi_d[min(du.m, (uint32_t)kMaxWindow)];
        if (tid == 0)
            T.njobs = 0u;
        for (int r = 0; r < 3; ++r)
            for (int l = 0; l < kAccSplit; ++l)
                T.acc[tid][r][l] = 0ull;
    }
    block_sync();
    if (tid == 0) {
        uint32_t off = 0, mmax = 2;
        for (uint32_t t = 0; t < ntrip; ++t) {
            T.off[t] = off;
            off += (T.m[t] + 1u) & ~1u;
            mmax = max(mmax, T.m[t]);
        }
        T.off[ntrip] = off;
        const uint32_t lp = ceil_log2(mmax);
        T.P = 1u << lp;
        T.log2P = lp;
    }
    block_sync();
    const uint32_t total = T.off[ntrip];
    const uint32_t P = T.P, lp = T.log2P;

    // ---- stage: grid integers into the sort segments, per-union extrema
    int32_t X[2], Y[2];
    uint32_t W[2];
    int I[2];
    bool act[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint32_t s = 2u * (uint32_t)tid + (uint32_t)q;
        uint32_t t = 0;
        while (t + 1 < ntrip && T.off[t + 1] <= s)
            ++t;
        const int i = (int)s - (int)T.off[t];
        act[q] = s < total && i < (int)T.m[t];
        W[q] = t;
        I[q] = act[q] ? i : 0;
        X[q] = 0;
        Y[q] = 0;
        if (act[q]) {
            uint32_t off = 0;
            X[q] = grid_int(T.x[t][i], off);
            Y[q] = grid_int(T.y[t][i], off);
            srt_x[(t << lp) + i] = X[q];
            srt_y[(t << lp) + i] = Y[q];
            if (off)
                atomicOr(&T.flags[t], kFlagOffGrid);
        }
    }
    for (uint32_t e = tid; e < (ntrip << lp); e += kBlock) {
        const uint32_t t = e >> lp, i = e & (P - 1u);
        if (i >= T.m[t]) {
            srt_x[e] = INT32_MAX;
            srt_y[e] = INT32_MAX;
        }
    }
    block_sync();

    // ---- sort every union's marginals (segments of P, padded with INT32_MAX):
    // the counts search them, and their ends are the union's extrema
    sort_marginals(srt_x, srt_y, ntrip << lp, P);
    if (tid < (int)ntrip) {
        const uint32_t m = T.m[tid];
        const uint32_t last = m > 0u ? m - 1u : 0u;
        T.mn[0][tid] = srt_x[tid << lp];
        T.mx[0][tid] = srt_x[(tid << lp) + last];
        T.mn[1][tid] = srt_y[tid << lp];
        T.mx[1][tid] = srt_y[(tid << lp) + last];
        const uint32_t nb = ceil_log2(m > 1 ? m : 2u);
        const uint32_t rxr = (uint32_t)(T.mx[0][tid] - T.mn[0][tid]);
        const uint32_t ryr = (uint32_t)(T.mx[1][tid] - T.mn[1][tid]);
        T.bits[tid] = (((rxr | ryr) >> (32 - nb)) == 0u) ? nb : 0u;
    }
    block_sync();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (act[q]) {
            const uint32_t s = 2u * (uint32_t)tid + (uint32_t)q;
            const uint32_t t = W[q], nb = T.bits[t];
            cand[2 * s] = (uint32_t)(X[q] - T.mn[0][t]) << nb;
            cand[2 * s + 1] = (uint32_t)(Y[q] - T.mn[1][t]) << nb;
        }
    }
    block_sync();

    // ---- neighbours: union and part lists of both slots in one scan
    const uint32_t t = W[0];
    const int m = (int)T.m[t];
    const bool live = act[0] && m > K;
    const uint32_t base = T.off[t];
    const uint32_t *cw = cand + 2 * base;
    const int a0 = (int)T.a0[t], na = (int)T.na[t], b0 = (int)T.b0[t], nbp = (int)T.nb[t];
    const bool inA0 = I[0] >= a0 && I[0] < a0 + na, inA1 = I[0] + 1 >= a0 && I[0] + 1 < a0 + na;
    const uint32_t bits = T.bits[t];
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t RXu[2] = {0u, 0u}, RYu[2] = {0u, 0u}, RXp[2] = {0u, 0u}, RYp[2] = {0u, 0u};
    {
        const unsigned long long bal = __ballot(live);
        if (bal != 0ull) {  // wave-uniform
            // lanes without a live slot follow the first live lane's union
            const int first = __ffsll((long long)bal) - 1;
            const uint32_t tl = live ? t : (uint32_t)__shfl((int)t, first, 64);
            const int ml = (int)T.m[tl], a0l = (int)T.a0[tl], nal = (int)T.na[tl];
            const int b0l = (int)T.b0[tl], nbl = (int)T.nb[tl];
            const uint32_t bitsl = T.bits[tl];
            const uint32_t *cwl = cand + 2 * T.off[tl];
            const int il = live ? I[0] : __shfl(I[0], first, 64);
            // one shape in the whole wave (every triple of the wave alike as
            // lane 0's, which holds a live slot's union)?  any 64-bit union?
            const bool alike = ml == __builtin_amdgcn_readfirstlane(ml) &&
                               a0l == __builtin_amdgcn_readfirstlane(a0l) &&
                               nal == __builtin_amdgcn_readfirstlane(nal) &&
                               b0l == __builtin_amdgcn_readfirstlane(b0l) &&
                               nbl == __builtin_amdgcn_readfirstlane(nbl);
            const int mode = __ballot(bitsl == 0u) != 0ull ? 2 : (__ballot(!alike) == 0ull ? 0 : 1);
            const bool in0 = il >= a0l && il < a0l + nal, in1 = il + 1 >= a0l && il + 1 < a0l + nal;
            const uint32_t maskl = (1u << bitsl) - 1u;
            if (mode != 2) {
                const uint32_t qx0 = cwl[2 * il], qy0 = cwl[2 * il + 1];
                const uint32_t qx1 = cwl[2 * il + 2], qy1 = cwl[2 * il + 3];
                uint32_t u0[S], u1[S], p0[S], p1[S];
#pragma unroll
                for (int r = 0; r < S; ++r)
                    u0[r] = u1[r] = p0[r] = p1[r] = 0xFFFFFFFFu;
                if (mode == 0) {
                    const int A0 = __builtin_amdgcn_readfirstlane(a0l), NA = __builtin_amdgcn_readfirstlane(nal);
                    const int B0 = __builtin_amdgcn_readfirstlane(b0l), NB = __builtin_amdgcn_readfirstlane(nbl);
                    trip_scan<S, false, false>(cwl, A0, NA, NA, qx0, qy0, qx1, qy1, false, false, u0, u1, p0, p1);
#pragma unroll
                    for (int r = 0; r < S; ++r) {
                        p0[r] = in0 ? u0[r] : 0xFFFFFFFFu;
                        p1[r] = in1 ? u1[r] : 0xFFFFFFFFu;
                    }
                    trip_scan<S, false, true>(cwl, B0, NB, NB, qx0, qy0, qx1, qy1, !in0, !in1, u0, u1, p0, p1);
                } else {
                    // the wave's loops run to its longest part
                    int na_max = nal, nb_max = nbl;
                    for (int o = 32; o > 0; o >>= 1) {
                        na_max = max(na_max, __shfl_xor(na_max, o, 64));
                        nb_max = max(nb_max, __shfl_xor(nb_max, o, 64));
                    }
                    na_max = __builtin_amdgcn_readfirstlane(na_max);
                    nb_max = __builtin_amdgcn_readfirstlane(nb_max);
                    trip_scan<S, true, false>(cwl, a0l, na_max, nal, qx0, qy0, qx1, qy1, false, false, u0, u1, p0,
                                              p1);
#pragma unroll
                    for (int r = 0; r < S; ++r) {
                        p0[r] = in0 ? u0[r] : 0xFFFFFFFFu;
                        p1[r] = in1 ? u1[r] : 0xFFFFFFFFu;
                    }
                    trip_scan<S, true, true>(cwl, b0l, nb_max, nbl, qx0, qy0, qx1, qy1, !in0, !in1, u0, u1, p0, p1);
                }
                const uint32_t bb = T.off[tl];
                radii_from_keys<K, uint32_t>(u0, (uint32_t)il, (int)bitsl, maskl, ml, cand, bb, qx0, qy0, (int)bitsl,
                                             a.estimator, RXu[0], RYu[0]);
                radii_from_keys<K, uint32_t>(u1, (uint32_t)il + 1u, (int)bitsl, maskl, ml, cand, bb, qx1, qy1,
                                             (int)bitsl, a.estimator, RXu[1], RYu[1]);
                radii_from_keys<K, uint32_t>(p0, (uint32_t)il, (int)bitsl, maskl, ml, cand, bb, qx0, qy0, (int)bitsl,
                                             a.estimator, RXp[0], RYp[0]);
                radii_from_keys<K, uint32_t>(p1, (uint32_t)il + 1u, (int)bitsl, maskl, ml, cand, bb, qx1, qy1,
                                             (int)bitsl, a.estimator, RXp[1], RYp[1]);
            } else {
                // some union of the wave needs 64-bit keys: one slot at a time
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int i = il + q;
                    const bool inq = q == 0 ? in0 : in1;
                    unsigned long long u[S], p[S];
#pragma unroll
                    for (int r = 0; r < S; ++r)
                        u[r] = p[r] = ~0ull;
                    const uint32_t qx = cwl[2 * i], qy = cwl[2 * i + 1];
                    trip_scan_wide<S>(cwl, a0l, nal, qx, qy, false, false, u, p);
#pragma unroll
                    for (int r = 0; r < S; ++r)
                        p[r] = inq ? u[r] : ~0ull;
                    trip_scan_wide<S>(cwl, b0l, nbl, qx, qy, !inq, true, u, p);
                    const uint32_t bb = T.off[tl];
                    radii_from_keys<K, unsigned long long>(u, (unsigned long long)i, 12, 0xFFFu, ml, cand, bb, qx, qy,
                                                           (int)bitsl, a.estimator, RXu[q], RYu[q]);
                    radii_from_keys<K, unsigned long long>(p, (unsigned long long)i, 12, 0xFFFu, ml, cand, bb, qx, qy,
                                                           (int)bitsl, a.estimator, RXp[q], RYp[q]);
                }
            }
            count_evals_lanes(a, live ? (uint32_t)(ml - 1) * (act[1] ? 2u : 1u) : 0u);
        }
    }
    block_sync();

    // ---- counts and digamma terms
    // union counts: two searches per dimension and point; a larger-part
    // point's part counts equal them when its part radii equal its union
    // radii, else they come from a job
    const bool small_a = na <= nbp;
    const int s0 = small_a ? a0 : b0, ns = small_a ? na : nbp;
    int cx[8], cy[8];
    int job[2] = {-1, -1};
    uint32_t *jobs = buf + 2 * kLocalSlots;  // the words after the union keys
    if (live) {
        const int32_t *sx = srt_x + (t << lp), *sy = srt_y + (t << lp);
        int32_t vx[4], vy[4];
        int ux[4], uy[4];
#pragma unroll
        for (int q = 0; q < 2; ++q)
            count_bounds(a.estimator, X[q], Y[q], (int32_t)RXu[q], (int32_t)RYu[q], vx + 2 * q, vy + 2 * q);
        count_lt_xy<4>(sx, sy, m, vx, vy, ux, uy);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            cx[4 * q] = ux[2 * q];
            cx[4 * q + 1] = ux[2 * q + 1];
            cy[4 * q] = uy[2 * q];
            cy[4 * q + 1] = uy[2 * q + 1];
            cx[4 * q + 2] = cx[4 * q];
            cx[4 * q + 3] = cx[4 * q + 1];
            cy[4 * q + 2] = cy[4 * q];
            cy[4 * q + 3] = cy[4 * q + 1];
            const bool inA = q == 0 ? inA0 : inA1;
            const bool in_small = small_a ? inA : !inA;
            const int part_m = inA ? na : nbp;
            if (act[q] && part_m > K && !in_small && (RXp[q] != RXu[q] || RYp[q] != RYu[q])) {
                const uint32_t j = atomicAdd(&T.njobs, 1u);
                if (j < (uint32_t)kTripJobs) {
                    jobs[4 * j] = t | ((uint32_t)(I[0] + q) << 8);
                    jobs[4 * j + 1] = RXp[q];
                    jobs[4 * j + 2] = RYp[q];
                    job[q] = (int)j;
                } else {
                    // more jobs than threads: search here
                    int32_t wx[2], wy[2];
                    int px[2], py[2];
                    count_bounds(a.estimator, X[q], Y[q], (int32_t)RXp[q], (int32_t)RYp[q], wx, wy);
                    count_lt_xy<2>(sx, sy, m, wx, wy, px, py);
                    cx[4 * q + 2] = px[0];
                    cx[4 * q + 3] = px[1];
                    cy[4 * q + 2] = py[0];
                    cy[4 * q + 3] = py[1];
                }
            }
        }
    }
    block_sync();
    if ((uint32_t)tid < min(T.njobs, (uint32_t)kTripJobs)) {
        const uint32_t w0 = jobs[4 * tid], jt = w0 & 0xFFu, ji = w0 >> 8;
        const uint32_t nbj = T.bits[jt];
        const uint32_t *cj = cand + 2 * (T.off[jt] + ji);
        const int32_t xj = (int32_t)(cj[0] >> nbj) + T.mn[0][jt], yj = (int32_t)(cj[1] >> nbj) + T.mn[1][jt];
        int32_t wx[2], wy[2];
        int px[2], py[2];
        count_bounds(a.estimator, xj, yj, (int32_t)jobs[4 * tid + 1], (int32_t)jobs[4 * tid + 2], wx, wy);
        count_lt_xy<2>(srt_x + (jt << lp), srt_y + (jt << lp), (int)T.m[jt], wx, wy, px, py);
        jobs[4 * tid] = (uint32_t)px[0];
        jobs[4 * tid + 1] = (uint32_t)px[1];
        jobs[4 * tid + 2] = (uint32_t)py[0];
        jobs[4 * tid + 3] = (uint32_t)py[1];
    }
    block_sync();
    if (live) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (job[q] >= 0) {
                cx[4 * q + 2] = (int)jobs[4 * job[q]];
                cx[4 * q + 3] = (int)jobs[4 * job[q] + 1];
                cy[4 * q + 2] = (int)jobs[4 * job[q] + 2];
                cy[4 * q + 3] = (int)jobs[4 * job[q] + 3];
            }
        }
        long long tu = 0, tpa = 0, tpb = 0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (!act[q])
                continue;
            const int i = I[0] + q;
            const bool inA = q == 0 ? inA0 : inA1;
            const bool in_small = small_a ? inA : !inA;
            const int part_m = inA ? na : nbp;
            int ux, uy;
            tu += point_terms(a, cx[4 * q], cx[4 * q + 1], cy[4 * q], cy[4 * q + 1], (int32_t)RXu[q], ux, uy);
            if (part_m > K) {
                int sx_n, sy_n;
                trip_count_part(cw, s0, ns, cw[2 * i], cw[2 * i + 1], RXp[q] << bits, RYp[q] << bits, a.estimator,
                                sx_n, sy_n);
                int nx, ny;
                if (a.estimator == 0) {
                    nx = in_small ? sx_n - 1 : (cx[4 * q + 2] - cx[4 * q + 3] - 1) - sx_n;
                    ny = in_small ? sy_n - 1 : (cy[4 * q + 2] - cy[4 * q + 3] - 1) - sy_n;
                    const long long v = a.psi_fix[nx] + a.psi_fix[ny];
                    tpa += inA ? v : 0;
                    tpb += inA ? 0 : v;
                } else {
                    const bool pos = RXp[q] > 0u;
                    nx = !pos ? 0 : (in_small ? sx_n - 1 : (cx[4 * q + 2] - cx[4 * q + 3] - 1) - sx_n);
                    ny = !pos ? 0 : (in_small ? sy_n - 1 : (cy[4 * q + 2] - cy[4 * q + 3] - 1) - sy_n);
                    const long long v = a.psi_fix[nx + 1] + a.psi_fix[ny + 1];
                    tpa += inA ? v : 0;
                    tpb += inA ? 0 : v;
                }
            }
        }
        const int sl = tid & (kAccSplit - 1);
        atomicAdd(&T.acc[t][2][sl], (unsigned long long)tu);
        if (tpa)
            atomicAdd(&T.acc[t][0][sl], (unsigned long long)tpa);
        if (tpb)
            atomicAdd(&T.acc[t][1][sl], (unsigned long long)tpb);
    }
    block_sync();

    // ---- estimates of the three windows, then the query's result
    if (tid < (int)ntrip) {
        const uint32_t mw[3] = {T.na[tid], T.nb[tid], T.m[tid]};
        const uint32_t wb = w0 + 3u * (uint32_t)tid;
        double mi3[3];
        uint32_t f3[3];
        for (int r = 0; r < 3; ++r) {
            uint32_t fl = T.flags[tid];
            double mi;
            if ((int)mw[r] <= K) {
                mi = __builtin_nan("");
                fl |= kFlagTooShort;
            } else {
                mi = estimate_from<K>(a.estimator, T.psi[tid][0], T.psi[tid][1 + r], (int)mw[r],
                                      (long long)acc_sum(T.acc[tid][r]));
            }
            mi3[r] = mi;
            f3[r] = fl;
            a.wmi[wb + r] = mi;
            a.wflags[wb + r] = fl;
        }
        store_result(a, T.query[tid], compose_result(T.qd[tid], mi3, f3));
    }
}

// --------------------------------------------------------------------------
// sweep items: a run of equally spaced windows, updated point by point
// --------------------------------------------------------------------------
// Windows [c s, c s + m) (c = 0 .. C-1, indices relative to the run's first
// point) of one series pair share m - s points with their neighbour.  The
// first window is evaluated in full; each later one is derived from the one
// before by removing its first s points and adding the next s, with the
// influenced regions of Section 7.1.2 (Definitions 7.1-7.2, Lemmas 1-4):
//   - a point whose list holds a removed point (the removed point lay in its
//     influenced region) searches the new window again;
//   - any other point keeps its list and inserts the added points' keys,
//     which enter exactly when they lie in its influenced region;
//   - added points search the whole window;
//   - a point whose radii did not change updates its marginal counts by the
//     removed and added points inside its influenced marginal regions; the
//     others, and the added points, count again.
// The points that search and count again are the step's jobs: a group of 8
// lanes takes one (each lane an eighth of the window's candidates, then a
// butterfly merge and a sum), three workgroup barriers a step.  Keys are (d << ib) | j with j the run-relative index (the same
// order as the window-relative index) and 2^ib >= the run's span.  The
// run's points (at most kSweepSpan) are read into LDS once; a window point
// of index j is owned by thread j mod R, R = pow2(m + s) <= 256, which keeps
// its list, radii and counts in registers.  Results equal those of a full scan of every window.

struct SweepShared {
    int32_t mn[2], mx[2];
    uint32_t nwork[2];   // job counters of even and odd windows
    uint32_t offc;       // off-grid points of the current window
    unsigned long long acc;
};

// Radii of a point from its k-list (key units): estimator 0 the largest
// |dx|, |dy| over its neighbours (their coordinates from the ring), 1 the
// joint k-th distance in both.
template <int K>
__device__ __forceinline__ void sweep_radii(const uint32_t (&t)[K], const uint32_t *ring, uint32_t rmask, uint32_t ib,
                                            uint32_t qx, uint32_t qy, uint32_t est, uint32_t &ex, uint32_t &ey)
{
    if (est == 0) {
        uint32_t rx = 0, ry = 0;
        const uint32_t imask = (1u << ib) - 1u;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const uint32_t s = (t[r] & imask) & rmask;
            rx = tmax(rx, sad_u32(qx, ring[2 * s], 0u));
            ry = tmax(ry, sad_u32(qy, ring[2 * s + 1], 0u));
        }
        ex = rx;
        ey = ry;
    } else {
        ex = ey = (t[K - 1] >> ib) << ib;
    }
}

__device__ __forceinline__ int sweep_pred(uint32_t d, uint32_t e, uint32_t est)
{
    return est == 0 ? (d <= e ? 1 : 0) : (d < e ? 1 : 0);
}

constexpr int kSweepGroup = 8;  // lanes sharing one point's search and count

// One point's update by a group of kSweepGroup consecutive lanes: its k
// nearest among the window's candidates [lo, lo + m) (the point itself,
// index self, excluded; lane g takes candidates lo + g, lo + g + 8, ...; a
// three-step butterfly merges the lanes' lists), its radii, then its marginal
// counts (lanes count their candidates, a butterfly sums).  Every lane of
// the group ends with the list and the counts.
template <int K>
__device__ __forceinline__ void sweep_group_update(const uint32_t *__restrict__ ring, uint32_t rmask, uint32_t ib,
                                                   int lo, int m, int self, uint32_t est, uint32_t (&t)[K], int &cx,
                                                   int &cy)
{
    const int g = (int)threadIdx.x & (kSweepGroup - 1);
    const uint32_t sq = (uint32_t)self & rmask;
    const uint32_t qx = ring[2 * sq], qy = ring[2 * sq + 1];
#pragma unroll
    for (int r = 0; r < K; ++r)
        t[r] = 0xFFFFFFFFu;
    for (int i = g; i < m; i += kSweepGroup) {
        const int j = lo + i;
        const uint32_t sl = (uint32_t)j & rmask;
        uint32_t key = tmax(sad_key_v(qx, ring[2 * sl], (uint32_t)j), sad_key_v(qy, ring[2 * sl + 1], (uint32_t)j));
        key = j == self ? 0xFFFFFFFFu : key;
        insert_sorted<K>(t, key);
    }
#pragma unroll
    for (int o = kSweepGroup / 2; o > 0; o >>= 1) {
        uint32_t other[K];
#pragma unroll
        for (int r = 0; r < K; ++r)
            other[r] = (uint32_t)__shfl_xor((int)t[r], o, 64);
#pragma unroll
        for (int r = 0; r < K; ++r)
            insert_sorted<K>(t, other[r]);
    }
    uint32_t ex, ey;
    sweep_radii<K>(t, ring, rmask, ib, qx, qy, est, ex, ey);
    int nx = 0, ny = 0;
    for (int i = g; i < m; i += kSweepGroup) {
        const int j = lo + i;
        const uint32_t sl = (uint32_t)j & rmask;
        if (j != self) {
            nx += sweep_pred(sad_u32(qx, ring[2 * sl], 0u), ex, est);
            ny += sweep_pred(sad_u32(qy, ring[2 * sl + 1], 0u), ey, est);
        }
    }
#pragma unroll
    for (int o = kSweepGroup / 2; o > 0; o >>= 1) {
        nx += __shfl_xor(nx, o, 64);
        ny += __shfl_xor(ny, o, 64);
    }
    cx = nx;
    cy = ny;
}

// Returns false, having evaluated nothing, when the run's value range does not
// fit 32-bit keys (the caller then evaluates its windows as local items).
template <int K>
__device__ bool sweep_item(const LaunchArgs &a, uint32_t w0, uint32_t nwin, uint32_t *buf, SweepShared &W)
{
    const int tid = threadIdx.x;
    const WinDesc d0 = a.win[w0];
    const int m = (int)d0.m;
    const int s = (int)(a.win[w0 + 1].x - d0.x);  // the plan gives C >= 2 windows at a constant stride
    const int N = (int)(nwin - 1u) * s + m;        // the run's points
    const float *X = d0.x, *Y = d0.y;

    // ---- the run's extrema and key width
    if (tid == 0) {
        W.mn[0] = W.mn[1] = INT32_MAX;
        W.mx[0] = W.mx[1] = INT32_MIN;
        W.acc = 0ull;
        W.offc = 0u;
        W.nwork[0] = W.nwork[1] = 0u;
    }
    block_sync();
    // the run's points, read from HBM once: grid integers (then keys) in
    // span, off-grid marks in offb
    uint32_t *span = buf;                                                // 2 words per point
    uint8_t *offb = reinterpret_cast<uint8_t *>(buf + 2 * kSweepSpan);  // kSweepSpan bytes
    {
        int32_t mnx = INT32_MAX, mxx = INT32_MIN, mny = INT32_MAX, mxy = INT32_MIN;
        for (int i = tid; i < N; i += kBlock) {
            uint32_t off = 0;
            const int32_t xi = grid_int(X[i], off), yi = grid_int(Y[i], off);
            span[2 * i] = (uint32_t)xi;
            span[2 * i + 1] = (uint32_t)yi;
            offb[i] = off ? 1 : 0;
            mnx = min(mnx, xi);
            mxx = max(mxx, xi);
            mny = min(mny, yi);
            mxy = max(mxy, yi);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mnx = min(mnx, __shfl_xor(mnx, o, 64));
            mxx = max(mxx, __shfl_xor(mxx, o, 64));
            mny = min(mny, __shfl_xor(mny, o, 64));
            mxy = max(mxy, __shfl_xor(mxy, o, 64));
        }
        if ((tid & 63) == 0) {
            atomicMin(&W.mn[0], mnx);
            atomicMax(&W.mx[0], mxx);
            atomicMin(&W.mn[1], mny);
            atomicMax(&W.mx[1], mxy);
        }
    }
    block_sync();
    const int32_t mnx = W.mn[0], mny = W.mn[1];
    const uint32_t ib = ceil_log2((uint32_t)N);
    const uint32_t range = (uint32_t)(W.mx[0] - mnx) | (uint32_t)(W.mx[1] - mny);
    if ((range >> (32 - ib)) != 0u)
        return false;  // 32-bit keys do not fit
    const uint32_t est = a.estimator;
    // ownership of the window's points: slot r = index mod R, R = pow2(m + s)
    const int R = (int)(1u << ceil_log2((uint32_t)(m + s)));
    const uint32_t rmask = (uint32_t)R - 1u;
    const uint32_t imask = (1u << ib) - 1u;
    for (int i = tid; i < N; i += kBlock) {
        span[2 * i] = (uint32_t)((int32_t)span[2 * i] - mnx) << ib;
        span[2 * i + 1] = (uint32_t)((int32_t)span[2 * i + 1] - mny) << ib;
    }
    // LDS after the span: the step's jobs (slots) and their results (k keys
    // and two counts each)
    constexpr int RW = K + 2;
    constexpr int kSpanWords = 2 * kSweepSpan + kSweepSpan / 4;
    constexpr int kJobs = (2 * kChunk - kSpanWords) / (RW + 1);
    const uint32_t *ring = span;  // indexed by run-relative point index
    constexpr uint32_t kAll = 0xFFFFFFFFu;
    uint32_t *job = buf + kSpanWords;
    uint32_t *res = job + kJobs;

    // the ring slot owned by this thread (R <= 256): its point's state
    const int r = tid;
    uint32_t Lk[K], QX = 0u, QY = 0u, EX = 0u, EY = 0u;
    int NX = 0, NY = 0, JI = -1;
    bool OFF = false;
#pragma unroll
    for (int e = 0; e < K; ++e)
        Lk[e] = 0xFFFFFFFFu;
    auto stage = [&](int j) {
        QX = ring[2 * j];
        QY = ring[2 * j + 1];
        OFF = offb[j] != 0;
    };
    block_sync();  // keys in place
    if (r < m)
        stage(r);

    int lo = 0;  // the current window is [lo, lo + m)
    for (int c = 0;; ++c) {
        // ---- which points search and count in full: all of the first
        // window; later the added points, the points whose list held a
        // removed one, and the points whose radii the added points changed
        int cat = 0;  // 0 empty, 2 in the window, 3 just added
        uint32_t J;
        const int j_own = lo + ((r - lo) & (int)rmask);
        if (c == 0) {
            cat = r < m ? 3 : 0;
            JI = r < m ? r : -1;
            J = (uint32_t)m;
        } else {
            const int plo = lo - s;  // the previous window's first point
            cat = r >= R ? 0 : (j_own < lo ? 0 : (j_own < plo + m ? 2 : (j_own < lo + m ? 3 : 0)));
            JI = -1;
            uint32_t ins = 0;
            bool full = cat == 3;
            if (cat == 2) {
                bool stale = false;
#pragma unroll
                for (int e = 0; e < K; ++e)
                    stale = stale || (int)(Lk[e] & imask) < lo;
                if (stale) {
                    full = true;
                } else {
                    for (int j = plo + m; j < lo + m; ++j) {
                        const uint32_t sl = (uint32_t)j;
                        const uint32_t key =
                            tmax(sad_key_v(QX, ring[2 * sl], (uint32_t)j), sad_key_v(QY, ring[2 * sl + 1], (uint32_t)j));
                        insert_sorted<K>(Lk, key);
                    }
                    ins = (uint32_t)s;
                    uint32_t ex, ey;
                    sweep_radii<K>(Lk, ring, kAll, ib, QX, QY, est, ex, ey);
                    if (ex != EX || ey != EY) {
                        full = true;
                    } else {
                        // the same radii: the counts move by the removed and
                        // added points inside the marginal regions
                        int dxn = 0, dyn = 0;
                        for (int j = plo; j < lo; ++j) {
                            const uint32_t sl = (uint32_t)j;
                            dxn -= sweep_pred(sad_u32(QX, ring[2 * sl], 0u), ex, est);
                            dyn -= sweep_pred(sad_u32(QY, ring[2 * sl + 1], 0u), ey, est);
                        }
                        for (int j = plo + m; j < lo + m; ++j) {
                            const uint32_t sl = (uint32_t)j;
                            dxn += sweep_pred(sad_u32(QX, ring[2 * sl], 0u), ex, est);
                            dyn += sweep_pred(sad_u32(QY, ring[2 * sl + 1], 0u), ey, est);
                        }
                        NX += dxn;
                        NY += dyn;
                    }
                }
            }
            if (full) {
                const uint32_t ji = atomicAdd(&W.nwork[c & 1], 1u);
                JI = (int)ji;
                if (ji < (uint32_t)kJobs)
                    job[ji] = (uint32_t)r;
            }
            count_evals_lanes(a, ins);
            block_sync();  // the job list is complete
            J = W.nwork[c & 1];
        }
        // the next window's counter: its last use (two windows back) ended
        // at that window's job-list barrier, its next use starts after this
        // window's last barrier
        if (tid == 0)
            W.nwork[(c + 1) & 1] = 0u;
        // ---- the jobs: groups of kSweepGroup lanes, or each owner alone
        if (J <= (uint32_t)kJobs) {
            const uint32_t grp = (uint32_t)tid / kSweepGroup;
            for (uint32_t jb = grp; jb < J; jb += kBlock / kSweepGroup) {
                const uint32_t sl = c == 0 ? jb : job[jb];
                const int jq = lo + (int)((sl - (uint32_t)lo) & rmask);
                uint32_t t[K];
                int cx, cy;
                sweep_group_update<K>(ring, kAll, ib, lo, m, jq, est, t, cx, cy);
                if ((tid & (kSweepGroup - 1)) == 0) {
#pragma unroll
                    for (int e = 0; e < K; ++e)
                        res[jb * RW + e] = t[e];
                    res[jb * RW + K] = (uint32_t)cx;
                    res[jb * RW + K + 1] = (uint32_t)cy;
                    if (a.evals)
                        atomicAdd(&a.evals[blockIdx.x], (unsigned long long)(m - 1));
                }
            }
            block_sync();  // the jobs' results are in LDS
            if (JI >= 0) {
#pragma unroll
                for (int e = 0; e < K; ++e)
                    Lk[e] = res[JI * RW + e];
                NX = (int)res[JI * RW + K];
                NY = (int)res[JI * RW + K + 1];
                sweep_radii<K>(Lk, ring, kAll, ib, QX, QY, est, EX, EY);
            }
        } else {
            // more jobs than LDS room (many ties on the removed points)
            const bool need = JI >= 0;
            if (__ballot(need) != 0ull) {
                uint32_t t[K];
#pragma unroll
                for (int e = 0; e < K; ++e)
                    t[e] = 0xFFFFFFFFu;
                for (int j = lo; j < lo + m; ++j) {
                    const uint32_t sl = (uint32_t)j;
                    uint32_t key =
                        tmax(sad_key_v(QX, ring[2 * sl], (uint32_t)j), sad_key_v(QY, ring[2 * sl + 1], (uint32_t)j));
                    key = j == j_own ? 0xFFFFFFFFu : key;
                    insert_sorted<K>(t, key);
                }
                uint32_t ex, ey;
                sweep_radii<K>(t, ring, kAll, ib, QX, QY, est, ex, ey);
                int nx = 0, ny = 0;
                for (int j = lo; j < lo + m; ++j) {
                    const uint32_t sl = (uint32_t)j;
                    if (j != j_own) {
                        nx += sweep_pred(sad_u32(QX, ring[2 * sl], 0u), ex, est);
                        ny += sweep_pred(sad_u32(QY, ring[2 * sl + 1], 0u), ey, est);
                    }
                }
                count_evals_lanes(a, need ? (uint32_t)(m - 1) : 0u);
                if (need) {
#pragma unroll
                    for (int e = 0; e < K; ++e)
                        Lk[e] = t[e];
                    EX = ex;
                    EY = ey;
                    NX = nx;
                    NY = ny;
                }
            }
        }

        // ---- window c: digamma terms; the next window's added points
        long long term = 0;
        uint32_t offn = 0;
        if (cat != 0) {
            int nx = NX, ny = NY;
            if (est != 0 && EX == 0u)
                nx = ny = 0;
            term = est == 0 ? a.psi_fix[nx] + a.psi_fix[ny] : a.psi_fix[nx + 1] + a.psi_fix[ny + 1];
            offn = OFF ? 1u : 0u;
        }
        const bool more = c + 1 < (int)nwin;
        if (more) {
            // they take the slots of points that left before this window
            const int jn = (lo + s) + ((r - (lo + s)) & (int)rmask);
            if (r < R && jn >= lo + m && jn < lo + m + s)
                stage(jn);
        }
        for (int o = 32; o > 0; o >>= 1) {
            term += __shfl_xor(term, o, 64);
            offn += (uint32_t)__shfl_xor((int)offn, o, 64);
        }
        if ((tid & 63) == 0) {
            atomicAdd(&W.acc, (unsigned long long)term);
            if (offn)
                atomicAdd(&W.offc, offn);
        }
        block_sync();  // sums complete, added points staged
        if (tid == 0) {
            const uint32_t w = w0 + (uint32_t)c;
            const double mi = window_estimate<K>(a, m, (long long)W.acc);
            const uint32_t fl = W.offc ? kFlagOffGrid : 0u;
            a.wmi[w] = mi;
            a.wflags[w] = fl;
            const uint32_t qi = a.win[w].query;
            store_result(a, qi, compose_result(a.qd[qi], &mi, &fl));
            W.acc = 0ull;
            W.offc = 0u;
        }
        if (!more)
            break;
        lo += s;
    }
    return true;
}

// --------------------------------------------------------------------------
// main: persistent loop over items
// --------------------------------------------------------------------------
// Two compilations per k: every item kind, at four workgroups per CU for k <=
// 5; and, for queues of local and triple items only, those two paths alone,
// whose smaller register need allows eight workgroups per CU (k <= 5).
template <int K, bool LOCAL_ONLY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(K <= 5 ? (LOCAL_ONLY ? 8 : 4) : 1))) void
main_kernel(LaunchArgs a)
{
    __shared__ __align__(16) uint32_t buf[2 * kChunk];  // 16 KB, shared by both item kinds
    __shared__ LocalShared L;
    __shared__ TripleShared T;
    __shared__ SweepShared SW;
    __shared__ long long s_part[kBlock / 64];
    __shared__ int32_t s_red[5];
    __shared__ uint32_t s_cnt[64];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;

    if (a.persistent) {
        if (tid == 0)
            s_item = atomicAdd(a.counter, 1u);
        block_sync();
    }
    for (uint32_t iter = 0;; ++iter) {
        uint32_t it;
        if (a.persistent) {
            it = s_item;
        } else {
            if (iter > 0)
                break;
            it = blockIdx.x;
        }
        if (it >= a.n_items)
            break;
        const Item itm = a.item[a.item_begin + it];
        if (LOCAL_ONLY) {
            if (itm.info & kItemTriple)
                triple_item<K>(a, itm.win, itm.info & 0xFFu, buf, T);
            else if (itm.info & kItemLocal)
                local_item<K>(a, itm.win, itm.info & 0xFFu, buf, L);
            else if (tid == 0)
                atomicOr(a.err, kErrItemKind);  // the host chose the wrong variant: report, skip
        } else if (itm.info & kItemSweep) {
            if (!sweep_item<K>(a, itm.win, itm.info & 0xFFu, buf, SW)) {
                // values too widely spread for 32-bit keys: every window on its own
                for (uint32_t c = 0; c < (itm.info & 0xFFu); ++c) {
                    block_sync();
                    local_item<K>(a, itm.win + c, 1u, buf, L);
                }
            }
        } else if (itm.info & kItemTriple) {
            triple_item<K>(a, itm.win, itm.info & 0xFFu, buf, T);
        } else if (itm.info & kItemLocal) {
            local_item<K>(a, itm.win, itm.info & 0xFFu, buf, L);
        } else if (itm.info & kItemPrep) {
            // a sort that split items of the window will wait for: its waves
            // issue ahead of theirs
            __builtin_amdgcn_s_setprio(3);
            prep_item(a, itm.win, buf, s_red, s_cnt);
            __builtin_amdgcn_s_setprio(0);
        } else {
            // split items are the largest, taken first: let their waves issue
            // ahead of the short local items sharing the CU, so they are not
            // the last to finish
            __builtin_amdgcn_s_setprio(2);
            split_item<K>(a, itm.win, (int)itm.info, buf, s_part, s_red);
            __builtin_amdgcn_s_setprio(0);
        }
        block_sync();
        // take the next item only now: a workgroup still busy must not hold
        // one (items are largest first); other workgroups keep the CU busy
        if (a.persistent && tid == 0)
            s_item = atomicAdd(a.counter, 1u);
        block_sync();
    }
}

#ifndef WMI_MAIN_K
// --------------------------------------------------------------------------
// serving: expand range parts into windows, queries and queue items
// --------------------------------------------------------------------------
// One workgroup per part.  Window w of the part: descriptor, a one-window
// query writing to arena index dst + w.  Split windows (m > kLocalSlots): a
// prep item each, then ceil(m / kSplitPoints) split items each.  Local
// windows: items of per_item consecutive windows.
__global__ __launch_bounds__(kBlock) void expand_kernel(LaunchArgs a, const PartDesc *parts, uint32_t n_parts,
                                                        Item *queue, WinDesc *win, QDesc *qd, uint64_t *cdst)
{
    const uint32_t pi = blockIdx.x;
    if (pi >= n_parts)
        return;
    const PartDesc P = parts[pi];
    const bool split = P.m > (uint32_t)kLocalSlots;
    const uint32_t nsplit = (P.m + kSplitPoints - 1) / kSplitPoints;
    for (uint32_t i = threadIdx.x; i < P.count; i += kBlock) {
        const uint32_t w = P.win0 + i;
        WinDesc d;
        d.x = P.x + P.start + (uint64_t)i * P.stride;
        d.y = P.y + P.start + (uint64_t)i * P.stride;
        d.m = P.m;
        d.query = w;
        d.sorted_off = split ? P.sorted0 + i * P.m : 0u;
        d.n_items = split ? nsplit : 1u;
        win[w] = d;
        QDesc q;
        q.win0 = w;
        q.nwin = 1u;
        q.tau_eff = 0.0;
        qd[w] = q;
        cdst[w] = P.dst + i;
        if (split) {
            queue[P.prep0 + i] = Item{w, kItemPrep};
            for (uint32_t t = 0; t < nsplit; ++t)
                queue[P.item0 + i * nsplit + t] = Item{w, t * (uint32_t)kSplitPoints};
        } else if (i % P.per_item == 0) {
            const uint32_t n = min(P.per_item, P.count - i);
            queue[P.item0 + i / P.per_item] = Item{w, kItemLocal | n};
        }
    }
}

// runs of queries: one thread per query writes its window and query
// descriptors and the queue entries its windows start (expand_query)
__global__ __launch_bounds__(kBlock) void expand_ranges_kernel(const RangeDesc *rd, uint32_t n_rd, uint32_t n_query,
                                                               WinDesc *win, QDesc *qd, Item *queue)
{
    const uint32_t t = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
    if (t >= n_query)
        return;
    uint32_t lo = 0, hi = n_rd - 1u;  // the last run whose first query is at or before t
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (rd[mid].q0 <= t)
            lo = mid;
        else
            hi = mid - 1u;
    }
    expand_query(rd[lo], t - rd[lo].q0, win, qd, queue);
}

// plain form: one workgroup per split window, before that window's items
__global__ __launch_bounds__(kBlock) void prep_kernel(LaunchArgs a)
{
    __shared__ __align__(16) uint32_t buf[kMaxWindow];
    __shared__ int32_t s_red[5];
    __shared__ uint32_t s_cnt[64];
    const uint32_t pi = a.win_begin + blockIdx.x;
    if (pi < a.n_prep)
        prep_item(a, a.prep_list[pi], buf, s_red, s_cnt);
}

// --------------------------------------------------------------------------
// validate: count non-finite and off-grid values of a device series
// --------------------------------------------------------------------------
__global__ void validate_kernel(const float *v, uint64_t n, unsigned long long *bad)
{
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long nonfinite = 0, off = 0;
    for (uint64_t i = t; i < n; i += stride) {
        float x = v[i];
        if (!isfinite(x)) {
            ++nonfinite;
        } else {
            uint32_t o = 0;
            (void)grid_int(x, o);
            off += o;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        nonfinite += __shfl_xor(nonfinite, o, 64);
        off += __shfl_xor(off, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (nonfinite)
            atomicAdd(&bad[0], nonfinite);
        if (off)
            atomicAdd(&bad[1], off);
    }
}

// --------------------------------------------------------------------------
// window entropy (Section 5.4: the denominator of the normalised MI)
// --------------------------------------------------------------------------
// H_w is the entropy of the window's empirical distribution of pairs: with
// c_v the number of points equal to the pair v in both coordinates,
//   H_w = - sum_v (c_v/m) ln(c_v/m) = ln m - (1/m) sum_i ln c_(i),
// the last sum over the points, c_(i) the multiplicity of point i's pair.
// One workgroup per query (grid-stride): each wanted window's pairs become
// 64-bit keys (float bits of x above those of y, -0 folded into +0), sorted
// in LDS by a bitonic network; each point then finds its run of equal keys
// by two binary searches.  The ln c terms are summed in 2^-44 fixed point,
// so the sum does not depend on the order of the additions.

__device__ __forceinline__ uint32_t pair_bits(float v)
{
    const uint32_t b = __float_as_uint(v);
    return (b << 1) == 0u ? 0u : b;  // +0 and -0 are one value
}

// Ascending bitonic sort of k[0..P), P a power of two, by the workgroup.
__device__ void bitonic_u64(unsigned long long *k, uint32_t P)
{
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            block_sync();
            for (uint32_t t = threadIdx.x; t < (P >> 1); t += kBlock) {
                const uint32_t lo = ((t & ~(stride - 1u)) << 1) | (t & (stride - 1u));
                const unsigned long long u = k[lo], v = k[lo + stride];
                if ((u > v) == ((lo & size) == 0u)) {
                    k[lo] = v;
                    k[lo + stride] = u;
                }
            }
        }
    }
    block_sync();
}

// First index in k[0..n) whose key is not below v (upper: above v).
__device__ __forceinline__ uint32_t key_bound(const unsigned long long *k, uint32_t n, unsigned long long v,
                                              bool upper)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (upper ? k[mid] <= v : k[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ double window_entropy(const WinDesc &d, unsigned long long *key, long long *s_part)
{
    const uint32_t m = d.m;
    const uint32_t P = 1u << ceil_log2(m > 1u ? m : 2u);
    block_sync();  // the previous window's keys are no longer read
    for (uint32_t i = threadIdx.x; i < P; i += kBlock)
        key[i] = i < m ? ((unsigned long long)pair_bits(d.x[i]) << 32) | pair_bits(d.y[i]) : ~0ull;
    bitonic_u64(key, P);
    long long part = 0;
    for (uint32_t i = threadIdx.x; i < m; i += kBlock) {
        const unsigned long long v = key[i];
        const uint32_t c = key_bound(key, m, v, true) - key_bound(key, m, v, false);
        part += c > 1u ? (long long)rint(log((double)c) * 0x1p44) : 0ll;
    }
    for (int o = 32; o > 0; o >>= 1)
        part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63u) == 0u)
        s_part[threadIdx.x >> 6] = part;
    block_sync();
    long long S = 0;
    for (int v = 0; v < kBlock / 64; ++v)
        S += s_part[v];
    return log((double)m) - (double)S * 0x1p-44 / (double)m;
}

__global__ __launch_bounds__(kBlock) void entropy_kernel(EntropyArgs a)
{
    __shared__ unsigned long long key[kMaxWindow];
    __shared__ long long s_part[kBlock / 64];
    const double nan = __builtin_nan("");
    for (uint32_t q = blockIdx.x; q < a.n_query; q += gridDim.x) {
        const QDesc qd = a.qd[q];
        for (uint32_t r = 0; r < 3u; ++r) {
            if (r >= qd.nwin) {
                if (a.hres && threadIdx.x == 0)
                    a.hres[3u * q + r] = nan;
                continue;
            }
            if (!a.hres && r != 1u)
                continue;  // only the extension's entropy is wanted
            const double h = window_entropy(a.win[qd.win0 + r], key, s_part);
            if (threadIdx.x == 0) {
                if (a.hres)
                    a.hres[3u * q + r] = h;
                if (r == 1u && a.set_tau)
                    a.qd[q].tau_eff = a.tau * h;
            }
        }
    }
}

// --------------------------------------------------------------------------
// host-side launchers
// --------------------------------------------------------------------------

hipError_t launch_expand(const LaunchArgs &a, const PartDesc *parts, uint32_t n_parts, Item *queue, WinDesc *win,
                         QDesc *qd, uint64_t *cdst, hipStream_t s)
{
    if (n_parts == 0)
        return hipSuccess;
    hipLaunchKernelGGL(expand_kernel, dim3(n_parts), dim3(kBlock), 0, s, a, parts, n_parts, queue, win, qd, cdst);
    return hipGetLastError();
}

hipError_t launch_expand_ranges(const RangeDesc *rd, uint32_t n_rd, uint32_t n_query, WinDesc *win, QDesc *qd,
                                Item *queue, hipStream_t s)
{
    if (n_rd == 0 || n_query == 0)
        return hipSuccess;
    const uint32_t blocks = (n_query + (uint32_t)kBlock - 1u) / (uint32_t)kBlock;
    hipLaunchKernelGGL(expand_ranges_kernel, dim3(blocks), dim3(kBlock), 0, s, rd, n_rd, n_query, win, qd, queue);
    return hipGetLastError();
}

hipError_t launch_validate(const float *v, uint64_t n, unsigned long long *bad, hipStream_t s)
{
    uint64_t blocks = (n + 255u) / 256u;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 2048)
        blocks = 2048;
    hipLaunchKernelGGL(validate_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, v, n, bad);
    return hipGetLastError();
}

hipError_t launch_clear(const LaunchArgs &a, hipStream_t s)
{
    uint32_t n = a.n_win > a.n_query ? a.n_win : a.n_query;
    uint32_t blocks = (n + 255u) / 256u;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(clear_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_entropy(const EntropyArgs &a, hipStream_t s)
{
    if (a.n_query == 0)
        return hipSuccess;
    const uint32_t blocks = a.n_query < 65536u ? a.n_query : 65536u;
    hipLaunchKernelGGL(entropy_kernel, dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prep(const LaunchArgs &a, uint32_t n_windows, hipStream_t s)
{
    if (n_windows == 0)
        return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3(n_windows), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// scratch of the allocation-free entry point
// --------------------------------------------------------------------------
// One static array per device, held until the process ends.  Host code never
// passes the array's name to a kernel or a copy: it takes the device address
// from noalloc_scratch(), looked up once per device with that device current.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void **ptr)
{
    static std::mutex mu;
    static std::vector<void *> addr;  // per device ordinal
    std::lock_guard<std::mutex> lk(mu);
    if (device < 0)
        return hipErrorInvalidDevice;
    if ((size_t)device >= addr.size())
        addr.resize((size_t)device + 1, nullptr);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != device)
            return hipErrorInvalidDevice;  // the caller makes the device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}
#endif  // !WMI_MAIN_K

// The main kernel is instantiated once per k, each in its own translation
// unit (this file compiled with WMI_MAIN_K = k), so the sixteen variants
// compile in parallel; the unit without WMI_MAIN_K dispatches on k.
#define WMI_PASTE2(a, b) a##b
#define WMI_PASTE(a, b) WMI_PASTE2(a, b)
#define WMI_K_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

#ifdef WMI_MAIN_K
hipError_t WMI_PASTE(launch_main_k, WMI_MAIN_K)(const LaunchArgs &a, uint32_t grid, hipStream_t s)
{
    if (a.local_only)
        hipLaunchKernelGGL((main_kernel<WMI_MAIN_K, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((main_kernel<WMI_MAIN_K, false>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int WMI_PASTE(main_occupancy_k, WMI_MAIN_K)(bool local_only)
{
    int n = 0;
    const hipError_t e =
        local_only ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, main_kernel<WMI_MAIN_K, true>, kBlock, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, main_kernel<WMI_MAIN_K, false>, kBlock, 0);
    if (e != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}
#else
#define X(KK)                                                                      \
    hipError_t launch_main_k##KK(const LaunchArgs &a, uint32_t grid, hipStream_t s); \
    int main_occupancy_k##KK(bool local_only);
WMI_K_CASES(X)
#undef X

hipError_t launch_main(const LaunchArgs &a, uint32_t grid, hipStream_t s)
{
    if (grid == 0)
        return hipSuccess;
    switch (a.k) {
#define X(KK)  \
    case KK:   \
        return launch_main_k##KK(a, grid, s);
        WMI_K_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

int main_occupancy(uint32_t k, bool local_only)
{
    switch (k) {
#define X(KK) \
    case KK:  \
        return main_occupancy_k##KK(local_only);
        WMI_K_CASES(X)
#undef X
    default:
        return 1;
    }
}
#endif

}  // namespace wmi
