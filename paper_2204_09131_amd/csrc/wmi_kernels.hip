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
// Work split (no MFMA anywhere: a max-norm neighbour search is not a
// contraction; the bound is the 32-bit VALU):
//   prep_kernel  one workgroup per window: converts the window to grid
//                integers (v * 2^12), finds its minima, checks the grid, and
//                sorts each marginal in LDS (bitonic) into HBM.
//   main_kernel  persistent: workgroups take (window, query block) items from
//                an atomic counter, largest first.  Per item the window is
//                staged in LDS as 32-bit keys; each lane scans all m
//                candidates for up to Q query points, keeping the k+1
//                smallest keys in registers with a med3 insertion network
//                (no sort, no branch); the point itself is dropped at the end.
//                Marginal counts come from two binary searches per dimension
//                in the sorted marginals.  Digamma terms are summed exactly in
//                64-bit fixed point with integer atomics, so the result does
//                not depend on how the window was split or scheduled.  The
//                last item of a window forms the estimate in double precision;
//                the last window of a query applies Definition 6.2.
//
// Keys.  With grid integers X = v * 2^12 and U = (X - min) << nb, where
// 2^nb >= m, the key of candidate j for query i is
//   max(|Ux_i - Ux_j| + j, |Uy_i - Uy_j| + j) = (d_ij << nb) | j,
// so unsigned order is the lexicographic order of (distance, index): ties
// go to the earlier time index.  Two v_sad_u32 and one v_max_u32 build it.
// A window whose value range does not fit 32 - nb bits uses 64-bit keys.
#include <hip/hip_runtime.h>

#include "wmi_internal.h"

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

// #{S[0..n) < v} and #{S[0..n) <= v} for ascending S; the loop trip count
// depends on n only, so lanes stay converged.
__device__ __forceinline__ int count_lt(const int32_t *S, int n, int32_t v)
{
    int base = 0;
    while (n > 1) {
        int half = n >> 1;
        base = (S[base + half] < v) ? base + half : base;
        n -= half;
    }
    return base + (S[base] < v ? 1 : 0);
}

__device__ __forceinline__ int count_le(const int32_t *S, int n, int32_t v)
{
    int base = 0;
    while (n > 1) {
        int half = n >> 1;
        base = (S[base + half] <= v) ? base + half : base;
        n -= half;
    }
    return base + (S[base] <= v ? 1 : 0);
}

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
    }
    for (uint32_t q = t; q < a.n_query; q += stride)
        a.qdone[q] = 0u;
    if (t == 0)
        a.counter[0] = 0u;
}

// --------------------------------------------------------------------------
// prep: grid integers, minima, grid check, sorted marginals (one WG / window)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void prep_kernel(LaunchArgs a)
{
    __shared__ int32_t sx[kMaxWindow];
    __shared__ int32_t sy[kMaxWindow];
    __shared__ int32_t s_red[5];

    const uint32_t w = a.win_begin + blockIdx.x;
    if (w >= a.n_win)
        return;
    const WinDesc d = a.win[w];
    const int m = (int)d.m;
    const int tid = threadIdx.x;
    int P = 1;
    while (P < m)
        P <<= 1;

    if (tid == 0) {
        s_red[0] = INT32_MAX;
        s_red[1] = INT32_MIN;
        s_red[2] = INT32_MAX;
        s_red[3] = INT32_MIN;
        s_red[4] = 0;
    }
    __syncthreads();

    int32_t mnx = INT32_MAX, mxx = INT32_MIN, mny = INT32_MAX, mxy = INT32_MIN;
    uint32_t off = 0;
    for (int i = tid; i < P; i += kBlock) {
        if (i < m) {
            int32_t xi = grid_int(d.x[i], off);
            int32_t yi = grid_int(d.y[i], off);
            sx[i] = xi;
            sy[i] = yi;
            mnx = min(mnx, xi);
            mxx = max(mxx, xi);
            mny = min(mny, yi);
            mxy = max(mxy, yi);
        } else {
            sx[i] = INT32_MAX;
            sy[i] = INT32_MAX;
        }
    }
    atomicMin(&s_red[0], mnx);
    atomicMax(&s_red[1], mxx);
    atomicMin(&s_red[2], mny);
    atomicMax(&s_red[3], mxy);
    if (off)
        atomicOr(&s_red[4], 1);

    // bitonic sort of both marginals, P = next power of two >= m
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = tid; t < (P >> 1); t += kBlock) {
                int lo = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));
                int hi = lo + stride;
                bool asc = (lo & size) == 0;
                int32_t a0 = sx[lo], a1 = sx[hi];
                if ((a0 > a1) == asc) {
                    sx[lo] = a1;
                    sx[hi] = a0;
                }
                int32_t b0 = sy[lo], b1 = sy[hi];
                if ((b0 > b1) == asc) {
                    sy[lo] = b1;
                    sy[hi] = b0;
                }
            }
        }
    }
    __syncthreads();

    int32_t *out = a.sorted + 2ull * d.sorted_off;
    for (int i = tid; i < m; i += kBlock) {
        out[i] = sx[i];
        out[m + i] = sy[i];
    }
    if (tid == 0) {
        WinAux ax;
        ax.min_x = s_red[0];
        ax.min_y = s_red[2];
        uint32_t rx = (uint32_t)(s_red[1] - s_red[0]);
        uint32_t ry = (uint32_t)(s_red[3] - s_red[2]);
        uint32_t nb = ceil_log2((uint32_t)(m > 1 ? m : 2));
        // 32-bit keys need (range << nb) + j < 2^32
        bool fits = m > 0 && nb < 32 && ((rx | ry) >> (32 - nb)) == 0u;
        ax.nb = fits ? nb : 0u;
        ax.flags = s_red[4] ? kFlagOffGrid : 0u;
        a.aux[w] = ax;
    }
}

// --------------------------------------------------------------------------
// main: k nearest neighbours, marginal counts, digamma sums, completion
// --------------------------------------------------------------------------

// 32-bit keys.  Lane query i = q0 + tid + q * kBlock.  Outputs the radii in
// grid units (estimator 0: per dimension; 1: the joint k-th distance).
template <int K, int Q>
__device__ __forceinline__ void knn_narrow(const uint32_t *__restrict__ cand, int m, uint32_t nb,
                                           int q0, int tid, uint32_t est, uint32_t (&rx)[Q],
                                           uint32_t (&ry)[Q])
{
    constexpr int S = K + 1;
    uint32_t qx[Q], qy[Q];
    uint32_t top[Q][S];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int i = min(q0 + tid + q * kBlock, m - 1);
        qx[q] = cand[2 * i];
        qy[q] = cand[2 * i + 1];
#pragma unroll
        for (int r = 0; r < S; ++r)
            top[q][r] = 0xFFFFFFFFu;
    }
    const uint4 *c4 = reinterpret_cast<const uint4 *>(cand);
    int j = 0;
#pragma unroll 2
    for (; j + 1 < m; j += 2) {
        uint4 c = c4[j >> 1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t k0 = tmax(sad_key(qx[q], c.x, (uint32_t)j), sad_key(qy[q], c.y, (uint32_t)j));
            insert_sorted<S>(top[q], k0);
            uint32_t k1 = tmax(sad_key(qx[q], c.z, (uint32_t)j + 1u), sad_key(qy[q], c.w, (uint32_t)j + 1u));
            insert_sorted<S>(top[q], k1);
        }
    }
    if (j < m) {
        uint32_t cx = cand[2 * j], cy = cand[2 * j + 1];
#pragma unroll
        for (int q = 0; q < Q; ++q)
            insert_sorted<S>(top[q], tmax(sad_u32(qx[q], cx, (uint32_t)j), sad_u32(qy[q], cy, (uint32_t)j)));
    }
    const uint32_t mask = (1u << nb) - 1u;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        // the point itself has key (0 << nb) | i; drop it if it is in the list
        uint32_t self = (uint32_t)min(q0 + tid + q * kBlock, m - 1);
        uint32_t nbk[K];
#pragma unroll
        for (int r = 0; r < K; ++r)
            nbk[r] = top[q][r] < self ? top[q][r] : top[q][r + 1];
        if (est == 0) {
            uint32_t ex = 0, ey = 0;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                uint32_t jj = nbk[r] & mask;
                ex = tmax(ex, sad_u32(qx[q], cand[2 * jj], 0u));
                ey = tmax(ey, sad_u32(qy[q], cand[2 * jj + 1], 0u));
            }
            rx[q] = ex >> nb;
            ry[q] = ey >> nb;
        } else {
            rx[q] = nbk[K - 1] >> nb;
            ry[q] = rx[q];
        }
    }
}

// 64-bit keys (d << 12 | j) for windows whose range does not fit 32-bit keys;
// the staged values are the raw grid integers.
template <int K, int Q>
__device__ __forceinline__ void knn_wide(const uint32_t *__restrict__ cand, int m, int q0, int tid,
                                         uint32_t est, uint32_t (&rx)[Q], uint32_t (&ry)[Q])
{
    constexpr int S = K + 1;
    int32_t qx[Q], qy[Q];
    unsigned long long top[Q][S];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int i = min(q0 + tid + q * kBlock, m - 1);
        qx[q] = (int32_t)cand[2 * i];
        qy[q] = (int32_t)cand[2 * i + 1];
#pragma unroll
        for (int r = 0; r < S; ++r)
            top[q][r] = ~0ull;
    }
    for (int j = 0; j < m; ++j) {
        int32_t cx = (int32_t)cand[2 * j], cy = (int32_t)cand[2 * j + 1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t d = (uint32_t)max(abs(qx[q] - cx), abs(qy[q] - cy));
            unsigned long long key = ((unsigned long long)d << 12) | (unsigned long long)j;
            if (key < top[q][S - 1])
                insert_sorted<S>(top[q], key);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        unsigned long long self = (unsigned long long)min(q0 + tid + q * kBlock, m - 1);
        unsigned long long nbk[K];
#pragma unroll
        for (int r = 0; r < K; ++r)
            nbk[r] = top[q][r] < self ? top[q][r] : top[q][r + 1];
        if (est == 0) {
            uint32_t ex = 0, ey = 0;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                uint32_t jj = (uint32_t)(nbk[r] & 0xFFFull);
                ex = tmax(ex, (uint32_t)abs(qx[q] - (int32_t)cand[2 * jj]));
                ey = tmax(ey, (uint32_t)abs(qy[q] - (int32_t)cand[2 * jj + 1]));
            }
            rx[q] = ex;
            ry[q] = ey;
        } else {
            rx[q] = (uint32_t)(nbk[K - 1] >> 12);
            ry[q] = rx[q];
        }
    }
}

template <int K, int Q>
__device__ __forceinline__ long long item_body(const LaunchArgs &a, const WinDesc &d, const WinAux &ax,
                                               int q0, uint32_t *cand)
{
    const int m = (int)d.m;
    const int tid = threadIdx.x;
    uint32_t rx[Q], ry[Q];
    if (ax.nb)
        knn_narrow<K, Q>(cand, m, ax.nb, q0, tid, a.estimator, rx, ry);
    else
        knn_wide<K, Q>(cand, m, q0, tid, a.estimator, rx, ry);

    // query grid integers, from the staged values, before they are replaced
    int32_t xi[Q], yi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int i = min(q0 + tid + q * kBlock, m - 1);
        if (ax.nb) {
            xi[q] = (int32_t)(cand[2 * i] >> ax.nb) + ax.min_x;
            yi[q] = (int32_t)(cand[2 * i + 1] >> ax.nb) + ax.min_y;
        } else {
            xi[q] = (int32_t)cand[2 * i];
            yi[q] = (int32_t)cand[2 * i + 1];
        }
    }
    __syncthreads();
    // stage the sorted marginals over the candidates
    int32_t *sx = reinterpret_cast<int32_t *>(cand);
    int32_t *sy = sx + kMaxWindow;
    const int32_t *src = a.sorted + 2ull * d.sorted_off;
    for (int i = tid; i < m; i += kBlock) {
        sx[i] = src[i];
        sy[i] = src[m + i];
    }
    __syncthreads();

    long long part = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int i = q0 + tid + q * kBlock;
        if (i >= m)
            continue;
        int cx, cy;
        int32_t ex = (int32_t)rx[q], ey = (int32_t)ry[q];
        if (a.estimator == 0) {
            cx = count_le(sx, m, xi[q] + ex) - count_lt(sx, m, xi[q] - ex) - 1;
            cy = count_le(sy, m, yi[q] + ey) - count_lt(sy, m, yi[q] - ey) - 1;
            part += a.psi_fix[cx] + a.psi_fix[cy];
        } else {
            // strict counts inside the joint radius; a zero radius counts nothing
            // (the open interval is empty), otherwise the point itself is inside
            if (ex > 0) {
                cx = count_lt(sx, m, xi[q] + ex) - count_le(sx, m, xi[q] - ex) - 1;
                cy = count_lt(sy, m, yi[q] + ey) - count_le(sy, m, yi[q] - ey) - 1;
            } else {
                cx = 0;
                cy = 0;
            }
            part += a.psi_fix[cx + 1] + a.psi_fix[cy + 1];
        }
        if (a.dbg_nx) {
            a.dbg_nx[i] = (uint32_t)cx;
            a.dbg_ny[i] = (uint32_t)cy;
            a.dbg_ex[i] = (float)ex * (1.0f / 4096.0f);
            a.dbg_ey[i] = (float)ey * (1.0f / 4096.0f);
        }
    }
    return part;
}

__device__ void finalize_query(const LaunchArgs &a, uint32_t query)
{
    const QDesc qd = a.qd[query];
    Result r;
    r.reserved = 0u;
    const double nan = __builtin_nan("");
    if (qd.nwin == 1) {
        r.mi_base = a.wmi[qd.win0];
        r.mi_ext = nan;
        r.mi_union = nan;
        r.flags = a.wflags[qd.win0];
    } else {
        double b = a.wmi[qd.win0], e = a.wmi[qd.win0 + 1], u = a.wmi[qd.win0 + 2];
        uint32_t f = a.wflags[qd.win0] | a.wflags[qd.win0 + 1] | a.wflags[qd.win0 + 2];
        if (!(f & kFlagTooShort)) {
            if (!(b > 0.0))
                f |= kFlagNonPos;
            else if (e < qd.tau_eff && u < b)
                f |= kFlagNoise;
        }
        r.mi_base = b;
        r.mi_ext = e;
        r.mi_union = u;
        r.flags = f;
    }
    a.res[query] = r;
}

template <int K>
__device__ void finalize_window(const LaunchArgs &a, uint32_t w, const WinDesc &d, const WinAux &ax)
{
    const int m = (int)d.m;
    double mi;
    uint32_t f = ax.flags;
    if (m <= K) {
        mi = __builtin_nan("");
        f |= kFlagTooShort;
    } else {
        long long S = (long long)atomicAdd(&a.acc[w], 0ull);
        double Sd = (double)S * 0x1p-44;
        if (a.estimator == 0)
            mi = (a.psi_d[K] - 1.0 / (double)K + a.psi_d[m]) - Sd / (double)m;
        else
            mi = (a.psi_d[K] + a.psi_d[m]) - Sd / (double)m;
    }
    a.wmi[w] = mi;
    a.wflags[w] = f;
    __threadfence();
    uint32_t prev = atomicAdd(&a.qdone[d.query], 1u);
    if (prev + 1u == a.qd[d.query].nwin) {
        __threadfence();
        finalize_query(a, d.query);
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void main_kernel(LaunchArgs a)
{
    __shared__ __align__(16) uint32_t cand[2 * kMaxWindow];
    __shared__ long long s_part[kBlock / 64];
    __shared__ uint32_t s_item, s_last;
    const int tid = threadIdx.x;

    for (uint32_t iter = 0;; ++iter) {
        uint32_t it;
        if (a.persistent) {
            if (tid == 0)
                s_item = atomicAdd(a.counter, 1u);
            __syncthreads();
            it = s_item;
        } else {
            if (iter > 0)
                break;
            it = blockIdx.x;
        }
        if (it >= a.n_items)
            break;
        const Item itm = a.item[a.item_begin + it];
        const WinDesc d = a.win[itm.win];
        const WinAux ax = a.aux[itm.win];
        const int m = (int)d.m;
        long long part = 0;
        if (m > K) {
            // stage the window as keys (32-bit) or raw grid integers (64-bit path)
            uint32_t off = 0;
            for (int i = tid; i < m; i += kBlock) {
                int32_t xi = grid_int(d.x[i], off);
                int32_t yi = grid_int(d.y[i], off);
                if (ax.nb) {
                    cand[2 * i] = (uint32_t)(xi - ax.min_x) << ax.nb;
                    cand[2 * i + 1] = (uint32_t)(yi - ax.min_y) << ax.nb;
                } else {
                    cand[2 * i] = (uint32_t)xi;
                    cand[2 * i + 1] = (uint32_t)yi;
                }
            }
            __syncthreads();
            const int q0 = (int)itm.q0;
            if (m - q0 <= kBlock)
                part = item_body<K, 1>(a, d, ax, q0, cand);
            else
                part = item_body<K, 2>(a, d, ax, q0, cand);
        }
        // workgroup sum of the fixed-point terms (exact, order-free)
        for (int o = 32; o > 0; o >>= 1)
            part += __shfl_xor(part, o, 64);
        if ((tid & 63) == 0)
            s_part[tid >> 6] = part;
        __syncthreads();
        if (tid == 0) {
            long long tot = 0;
            for (int wv = 0; wv < kBlock / 64; ++wv)
                tot += s_part[wv];
            if (m > K)
                atomicAdd(&a.acc[itm.win], (unsigned long long)tot);
            __threadfence();
            uint32_t prev = atomicAdd(&a.wdone[itm.win], 1u);
            s_last = (prev + 1u == d.n_items) ? 1u : 0u;
            if (s_last) {
                __threadfence();
                finalize_window<K>(a, itm.win, d, ax);
            }
        }
        __syncthreads();
    }
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
// host-side launchers
// --------------------------------------------------------------------------

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

hipError_t launch_prep(const LaunchArgs &a, uint32_t n_windows, hipStream_t s)
{
    if (n_windows == 0)
        return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3(n_windows), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_main_k(const LaunchArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(main_kernel<K>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int K>
static int occupancy_k()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, main_kernel<K>, kBlock, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

#define WMI_K_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_main(const LaunchArgs &a, uint32_t grid, hipStream_t s)
{
    if (grid == 0)
        return hipSuccess;
    switch (a.k) {
#define X(KK)  \
    case KK:   \
        return launch_main_k<KK>(a, grid, s);
        WMI_K_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

int main_occupancy(uint32_t k)
{
    switch (k) {
#define X(KK) \
    case KK:  \
        return occupancy_k<KK>();
        WMI_K_CASES(X)
#undef X
    default:
        return 1;
    }
}

}  // namespace wmi
