/*
 * ksg_oracle.c -- plain CPU reference for windowed KSG mutual information.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (Ho et al., "A Unified Approach for Multi-Scale
 * Synchronous Correlation Search in Big Time Series"):
 *
 *   - a window is a contiguous index range shared by both series
 *     (Definitions 3.2 and 3.4); window [s, s+m) here, half-open;
 *   - its MI is the KSG estimate of Eq. (2) (Section 4.2): for each point the
 *     k nearest neighbours in the joint space under the maximum norm
 *     (Section 7.1.1 footnote), the per-dimension distances to those
 *     neighbours, the marginal counts inside those distances, then
 *         I = psi(k) - 1/k + psi(n) - < psi(n_x) + psi(n_y) >
 *     with n the number of points in the window;
 *   - the count semantics follow the worked example of Section 7.1.1:
 *     the marginal counts include the k neighbours themselves (<=) and
 *     exclude the point itself;
 *   - the noise test of Definition 6.2, applied to the split of a window into
 *     its overlapping part and its newly added part (Section 6.2).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - ties among equal distances are broken by the smaller index j, so the
 *     neighbour set is the first k of (d_ij, j) in lexicographic order;
 *   - psi is evaluated at integers only, from psi(1) = -gamma and
 *     psi(n+1) = psi(n) + 1/n, summed in long double and rounded once;
 *   - a window with m <= k has no estimate (NaN) and sets TOO_SHORT;
 *   - estimator 1 is Kraskov's first estimator (joint radius d_k, strict <,
 *     psi(n+1) terms, no -1/k), offered for the looser "within d_k" wording.
 *
 * Arithmetic: inputs are float32; everything here is done in double.  On the
 * 2^-12 grid with |v| < 2^11 every coordinate difference is exact in both
 * float and double, so neighbour sets and counts are exact.
 *
 * Deliberately slow: the k neighbours are found by k successive minimum
 * searches over all other points (no sorting, no spatial index, no
 * blocking), and the sums run in ascending point order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PSI_MAX (1 << 16)
#define ORACLE_K_MAX 16

#define FLAG_NOISE 1u
#define FLAG_TOO_SHORT 2u
#define FLAG_NONPOS_BASE 4u
#define FLAG_OFFGRID 8u

/* Euler-Mascheroni constant, 30 significant digits. */
static const long double EULER_GAMMA = 0.577215664901532860606512090082L;

static double psi_tab[ORACLE_PSI_MAX + 1];
static int psi_ready = 0;

__attribute__((constructor)) static void build_psi(void)
{
    /* psi(1) = -gamma, psi(n + 1) = psi(n) + 1/n  (integer arguments only). */
    long double acc = -EULER_GAMMA;
    psi_tab[0] = NAN;
    for (int n = 1; n <= ORACLE_PSI_MAX; ++n) {
        psi_tab[n] = (double)acc;
        acc += 1.0L / (long double)n;
    }
    psi_ready = 1;
}

static double psi(long n)
{
    if (!psi_ready)
        build_psi();
    if (n < 1 || n > ORACLE_PSI_MAX)
        return NAN;
    return psi_tab[n];
}

double oracle_psi(long n) { return psi(n); }

int oracle_psi_table(int n_max, double *out)
{
    if (n_max < 1 || n_max > ORACLE_PSI_MAX)
        return -1;
    for (int n = 1; n <= n_max; ++n)
        out[n - 1] = psi(n);
    return 0;
}

/* Maximum-norm distance between points i and j of the window. */
static double dist(const float *x, const float *y, int i, int j)
{
    double dx = fabs((double)x[i] - (double)x[j]);
    double dy = fabs((double)y[i] - (double)y[j]);
    return dx > dy ? dx : dy;
}

/*
 * Per-point quantities of one window.
 *   nbr[i*k + r] : index of the (r+1)-th neighbour of i in (d, j) order
 *   nx, ny       : marginal counts as defined by the estimator
 *   ex, ey       : estimator 0: max |x_i - x_j| and max |y_i - y_j| over the
 *                  k neighbours; estimator 1: both hold the joint d_k(i)
 * Returns 0, or -1 if m <= k or k is out of range.
 */
int oracle_window_counts(const float *x, const float *y, int m, int k, int estimator,
                         uint32_t *nx, uint32_t *ny, double *ex, double *ey, int32_t *nbr)
{
    if (k < 1 || k > ORACLE_K_MAX || m <= k)
        return -1;
    for (int i = 0; i < m; ++i) {
        int chosen[ORACLE_K_MAX];
        double prev_d = -1.0;
        int prev_j = -1;
        /* k successive minimum searches over (d_ij, j), each strictly after
         * the previous pick in lexicographic order. */
        for (int r = 0; r < k; ++r) {
            int best_j = -1;
            double best_d = 0.0;
            for (int j = 0; j < m; ++j) {
                if (j == i)
                    continue;
                double d = dist(x, y, i, j);
                int after_prev = (d > prev_d) || (d == prev_d && j > prev_j);
                if (!after_prev)
                    continue;
                if (best_j < 0 || d < best_d || (d == best_d && j < best_j)) {
                    best_j = j;
                    best_d = d;
                }
            }
            chosen[r] = best_j;
            prev_d = best_d;
            prev_j = best_j;
        }
        if (nbr)
            for (int r = 0; r < k; ++r)
                nbr[(size_t)i * k + r] = chosen[r];

        uint32_t cx = 0, cy = 0;
        double rx, ry;
        if (estimator == 0) {
            rx = 0.0;
            ry = 0.0;
            for (int r = 0; r < k; ++r) {
                double dx = fabs((double)x[i] - (double)x[chosen[r]]);
                double dy = fabs((double)y[i] - (double)y[chosen[r]]);
                if (dx > rx) rx = dx;
                if (dy > ry) ry = dy;
            }
            for (int j = 0; j < m; ++j) {
                if (j == i)
                    continue;
                if (fabs((double)x[i] - (double)x[j]) <= rx) ++cx;
                if (fabs((double)y[i] - (double)y[j]) <= ry) ++cy;
            }
        } else {
            double dk = dist(x, y, i, chosen[k - 1]);
            rx = dk;
            ry = dk;
            for (int j = 0; j < m; ++j) {
                if (j == i)
                    continue;
                if (fabs((double)x[i] - (double)x[j]) < dk) ++cx;
                if (fabs((double)y[i] - (double)y[j]) < dk) ++cy;
            }
        }
        nx[i] = cx;
        ny[i] = cy;
        if (ex) ex[i] = rx;
        if (ey) ey[i] = ry;
    }
    return 0;
}

/* KSG estimate of one window (Eq. 2); NaN when m <= k. */
double oracle_window_mi(const float *x, const float *y, int m, int k, int estimator)
{
    if (k < 1 || k > ORACLE_K_MAX || m <= k)
        return NAN;
    uint32_t *nx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)m);
    uint32_t *ny = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)m);
    if (!nx || !ny) {
        free(nx);
        free(ny);
        return NAN;
    }
    oracle_window_counts(x, y, m, k, estimator, nx, ny, NULL, NULL, NULL);
    double s = 0.0;
    double mi;
    if (estimator == 0) {
        for (int i = 0; i < m; ++i)
            s += psi(nx[i]) + psi(ny[i]);
        mi = (psi(k) - 1.0 / (double)k + psi(m)) - s / (double)m;
    } else {
        for (int i = 0; i < m; ++i)
            s += psi((long)nx[i] + 1) + psi((long)ny[i] + 1);
        mi = (psi(k) + psi(m)) - s / (double)m;
    }
    free(nx);
    free(ny);
    return mi;
}

/* ---------------------------------------------------------------------- */
/* window entropy for the normalised MI of Section 5.4                     */
/* ---------------------------------------------------------------------- */

/*
 * H_w of Eq. (normalizedMI)'s denominator, read as the entropy of the
 * window's empirical distribution (the printed formula lacks its minus sign
 * and names p^(x_i, y_i), the relative frequency of a sample pair):
 *     H_w = - sum over the distinct pairs v of p_v ln p_v,  p_v = c_v / m,
 * with c_v the number of points of the window equal to v in both
 * coordinates.  Written out directly: each distinct pair is taken at its
 * first occurrence, its multiplicity counted over the whole window.
 * Natural logarithm; 0 for m = 1; ln m when every pair is distinct.
 */
double oracle_window_entropy(const float *x, const float *y, int m)
{
    if (m < 1)
        return NAN;
    double h = 0.0;
    for (int i = 0; i < m; ++i) {
        int first = 1;
        for (int j = 0; j < i && first; ++j)
            if (x[j] == x[i] && y[j] == y[i])
                first = 0;
        if (!first)
            continue;
        int c = 0;
        for (int j = 0; j < m; ++j)
            if (x[j] == x[i] && y[j] == y[i])
                ++c;
        const double p = (double)c / (double)m;
        h -= p * log(p);
    }
    return h;
}

/* ---------------------------------------------------------------------- */
/* batches of queries over a set of series                                 */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint32_t a, b;
    uint64_t start;
    uint32_t len;
    uint32_t ext_len;
    int32_t ext_side; /* 0 plain window, +1 extension on the right, -1 on the left */
    uint32_t pad;
} oracle_query;

typedef struct {
    double mi_base, mi_ext, mi_union;
    uint32_t flags;
    uint32_t pad;
} oracle_result;

static int value_on_grid(float v)
{
    double s = (double)v * 4096.0;
    return isfinite(s) && s == nearbyint(s) && fabs(s) <= 8388607.0;
}

static double window_of(const float *const *series, const oracle_query *q, uint64_t s,
                        uint32_t m, int k, int estimator, uint32_t *flags)
{
    const float *xa = series[q->a] + s;
    const float *yb = series[q->b] + s;
    for (uint32_t i = 0; i < m; ++i)
        if (!value_on_grid(xa[i]) || !value_on_grid(yb[i]))
            *flags |= FLAG_OFFGRID;
    if ((int)m <= k) {
        *flags |= FLAG_TOO_SHORT;
        return NAN;
    }
    return oracle_window_mi(xa, yb, (int)m, k, estimator);
}

/*
 * Evaluate queries.  A query with ext_side == 0 is one window [start,
 * start+len).  A query with ext_side != 0 is a noise triple (Definition 6.2
 * as applied in Section 6.2): base w_o = [start, start+len), extension w_d
 * of ext_len samples adjacent on the given side, union w'' = w_o with w_d.
 *   noise  <=>  I(w_o) > 0  and  I(w_d) < tau_eff  and  I(w'') < I(w_o)
 * with tau_eff = tau (tau_normalize 0), tau * ln(ext_len) (1: the window
 * entropy of Section 5.4 when every pair of w_d is distinct), or tau * H(w_d)
 * with H the empirical entropy of oracle_window_entropy (2).
 * Series bounds are not checked here; callers pass valid queries.
 * Queries are independent; they are spread over threads with OpenMP.
 */
int oracle_batch(const float *const *series, const oracle_query *qs, int64_t count, int k,
                 int estimator, double tau, int tau_normalize, oracle_result *out)
{
    if (k < 1 || k > ORACLE_K_MAX || tau_normalize < 0 || tau_normalize > 2)
        return -1;
    if (!psi_ready)
        build_psi();
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < count; ++t) {
        const oracle_query *q = &qs[t];
        oracle_result r;
        memset(&r, 0, sizeof(r));
        uint32_t f = 0;
        r.mi_base = window_of(series, q, q->start, q->len, k, estimator, &f);
        if (q->ext_side == 0) {
            r.mi_ext = NAN;
            r.mi_union = NAN;
        } else {
            uint64_t ext_start = q->ext_side > 0 ? q->start + q->len : q->start - q->ext_len;
            uint64_t uni_start = q->ext_side > 0 ? q->start : q->start - q->ext_len;
            r.mi_ext = window_of(series, q, ext_start, q->ext_len, k, estimator, &f);
            r.mi_union = window_of(series, q, uni_start, q->len + q->ext_len, k, estimator, &f);
            if (!(f & FLAG_TOO_SHORT)) {
                double tau_eff = tau;
                if (tau_normalize == 1)
                    tau_eff = tau * log((double)q->ext_len);
                else if (tau_normalize == 2)
                    tau_eff = tau * oracle_window_entropy(series[q->a] + ext_start, series[q->b] + ext_start,
                                                          (int)q->ext_len);
                if (!(r.mi_base > 0.0))
                    f |= FLAG_NONPOS_BASE;
                else if (r.mi_ext < tau_eff && r.mi_union < r.mi_base)
                    f |= FLAG_NOISE;
            }
        }
        r.flags = f;
        out[t] = r;
    }
    return 0;
}

/* Set the OpenMP thread count (n > 0) and return the count in effect. */
int oracle_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
