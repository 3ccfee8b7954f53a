// Device helpers for the symmetric tridiagonal matrices of Lanczos runs:
// Sturm counts, extreme eigenvalues by multisection, and a pivoted solve.
#pragma once

#include <hip/hip_runtime.h>

namespace hoscf {

// ---------------------------------------------------------------------------
// Symmetric tridiagonal helpers (Lanczos matrix T_m: diag al, off-diag be).
// ---------------------------------------------------------------------------

// Number of eigenvalues of T_m smaller than x (Sturm sequence of the LDL'
// pivots).
// The quotient b2/d uses the hardware reciprocal refined by two Newton
// steps (relative error ~1e-16, well inside what the count needs) instead
// of a correctly rounded division.
__device__ inline double fast_div(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    r = fma(fma(-b, r, 1.0), r, r);
    return a * r;
}

__device__ inline int sturm_count(const double* al, const double* b2, int m, double x, double pivmin) {
    int cnt = 0;
    double d = al[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    cnt += d < 0.0;
    for (int k = 1; k < m; ++k) {
        d = (al[k] - x) - fast_div(b2[k - 1], d);
        if (fabs(d) < pivmin) d = -pivmin;
        cnt += d < 0.0;
    }
    return cnt;
}

// Extreme eigenvalues of T_m by 32-way multisection per end (wave 0 only;
// lanes 0-31 bracket the smallest, lanes 32-63 the largest).
__device__ inline void extreme_eigs(const double* al, const double* b2, const double* be, int m, double* out_lo,
                             double* out_hi) {
    const int lane = threadIdx.x & 63;
    double glo = 1e300, ghi = -1e300, bmax = 0.0;
    for (int k = 0; k < m; ++k) {
        const double r = (k > 0 ? fabs(be[k - 1]) : 0.0) + (k < m - 1 ? fabs(be[k]) : 0.0);
        glo = fmin(glo, al[k] - r);
        ghi = fmax(ghi, al[k] + r);
        if (k < m - 1) bmax = fmax(bmax, b2[k]);
    }
    const double scale = fmax(fabs(glo), fabs(ghi));
    const double pivmin = 1e-290 * fmax(1.0, bmax);
    const double pad = 2.0 * 2.220446049250313e-16 * scale + pivmin;
    double lo0 = glo - pad, hi0 = ghi + pad;  // interval for the smallest eigenvalue
    double lo1 = glo - pad, hi1 = ghi + pad;  // interval for the largest
    const bool low_half = lane < 32;
    const int sub = lane & 31;
    for (int round = 0; round < 14; ++round) {
        const double lo = low_half ? lo0 : lo1, hi = low_half ? hi0 : hi1;
        const double x = lo + (hi - lo) * (double)(sub + 1) / 33.0;
        const int c = sturm_count(al, b2, m, x, pivmin);
        // smallest: first point with count >= 1; largest: first point with count == m
        const bool hit = low_half ? (c >= 1) : (c >= m);
        const unsigned long long bal = __ballot(hit);
        const unsigned lo_bits = (unsigned)(bal & 0xffffffffull);
        const unsigned hi_bits = (unsigned)(bal >> 32);
        // lane-uniform update of both intervals
        const double xs_lo_step = (hi0 - lo0) / 33.0;
        const double xs_hi_step = (hi1 - lo1) / 33.0;
        if (lo_bits) {
            const int f = __ffs(lo_bits) - 1;
            const double nhi = lo0 + xs_lo_step * (f + 1);
            const double nlo = f > 0 ? lo0 + xs_lo_step * f : lo0;
            lo0 = nlo;
            hi0 = nhi;
        } else {
            lo0 = lo0 + xs_lo_step * 32;
        }
        if (hi_bits) {
            const int f = __ffs(hi_bits) - 1;
            const double nhi = lo1 + xs_hi_step * (f + 1);
            const double nlo = f > 0 ? lo1 + xs_hi_step * f : lo1;
            lo1 = nlo;
            hi1 = nhi;
        } else {
            lo1 = lo1 + xs_hi_step * 32;
        }
        const double tol = 4.0 * 2.220446049250313e-16 * scale + pivmin;
        if (hi0 - lo0 <= tol && hi1 - lo1 <= tol) break;
    }
    *out_lo = 0.5 * (lo0 + hi0);
    *out_hi = 0.5 * (lo1 + hi1);
}

// Solve (T_m - shift I) y = rhs by Gaussian elimination with partial
// pivoting on the tridiagonal (single thread).  Zero pivots are replaced by
// `zrep` when zrep > 0; otherwise the call reports singularity (returns false).
__device__ inline bool tri_solve(const double* al, const double* be, int m, double shift, double* y, double zrep,
                          double* d, double* du, double* du2, double* dl) {
    for (int i = 0; i < m; ++i) {
        d[i] = al[i] - shift;
        if (i < m - 1) {
            du[i] = be[i];
            dl[i] = be[i];
            du2[i] = 0.0;
        }
    }
    for (int i = 0; i < m - 1; ++i) {
        if (fabs(d[i]) >= fabs(dl[i])) {
            if (d[i] == 0.0) {
                if (zrep <= 0.0) return false;
                d[i] = zrep;
            }
            const double f = dl[i] / d[i];
            d[i + 1] -= f * du[i];
            y[i + 1] -= f * y[i];
        } else {
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            const double t = du[i];
            du[i] = d[i + 1];
            d[i + 1] = t - f * d[i + 1];
            if (i < m - 2) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
            const double yt = y[i];
            y[i] = y[i + 1];
            y[i + 1] = yt - f * y[i + 1];
        }
    }
    if (d[m - 1] == 0.0) {
        if (zrep <= 0.0) return false;
        d[m - 1] = zrep;
    }
    y[m - 1] /= d[m - 1];
    if (m >= 2) y[m - 2] = (y[m - 2] - du[m - 2] * y[m - 1]) / d[m - 2];
    for (int i = m - 3; i >= 0; --i) y[i] = (y[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / d[i];
    return true;
}

}  // namespace hoscf
