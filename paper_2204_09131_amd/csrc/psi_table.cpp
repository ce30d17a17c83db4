// psi_table.cpp -- digamma at integer arguments for the device tables.
//
// The estimate of Eq. (2) needs psi(k), psi(m) and psi(n_x), psi(n_y) at
// positive integers only.  The tables are built here on the host, once per
// store, and uploaded; no transcendental function runs on the device.
//
// Construction: for n >= 64 the asymptotic expansion of the digamma function
// (Abramowitz & Stegun 6.3.18)
//   psi(x) ~ ln x - 1/(2x) - sum_{j>=1} B_{2j} / (2j x^{2j})
// truncated after x^-14 (error below 1e-29 at x = 64); for n < 64 the
// recurrence psi(n) = psi(n + 1) - 1/n, stepping down from psi(64).  All in
// long double, rounded once to double.  The fixed-point table holds
// round(psi(n) * 2^44) for exact integer accumulation on the device.
#include <cmath>
#include <vector>

namespace wmi {

static long double psi_asymptotic(long double x)
{
    const long double x2 = 1.0L / (x * x);
    // B_{2j} / (2j) for j = 1..7
    const long double c[7] = {1.0L / 12.0L,   -1.0L / 120.0L,     1.0L / 252.0L, -1.0L / 240.0L,
                              1.0L / 132.0L,  -691.0L / 32760.0L, 1.0L / 12.0L};
    long double s = 0.0L, p = x2;
    for (int j = 0; j < 7; ++j) {
        s += c[j] * p;
        p *= x2;
    }
    return logl(x) - 0.5L / x - s;
}

void build_psi_tables(int n_max, std::vector<double> &psi_d, std::vector<long long> &psi_fix)
{
    const int n0 = 64;
    std::vector<long double> v((size_t)n_max + 1 > (size_t)n0 + 1 ? (size_t)n_max + 1 : (size_t)n0 + 1);
    for (int n = n0; n < (int)v.size(); ++n)
        v[(size_t)n] = psi_asymptotic((long double)n);
    for (int n = n0 - 1; n >= 1; --n)
        v[(size_t)n] = v[(size_t)n + 1] - 1.0L / (long double)n;
    psi_d.assign((size_t)n_max + 1, 0.0);
    psi_fix.assign((size_t)n_max + 1, 0);
    for (int n = 1; n <= n_max; ++n) {
        psi_d[(size_t)n] = (double)v[(size_t)n];
        psi_fix[(size_t)n] = llroundl(v[(size_t)n] * 17592186044416.0L);  // 2^44
    }
}

}  // namespace wmi
