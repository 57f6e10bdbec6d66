// Host eigensolver for the Lanczos tridiagonal matrix T (diagonal d,
// off-diagonal e): all eigenvalues by the implicit QL method with Wilkinson
// shifts (Bowdler, Martin, Reinsch and Wilkinson, 1968), and the eigenvector
// of one eigenvalue by inverse iteration with a pivoted tridiagonal solve.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace ecut {

// Eigenvalues of T, ascending.  d: n entries, e: n-1 entries (copied).
inline std::vector<double> tridiag_eigenvalues(const std::vector<double> &d_in, const std::vector<double> &e_in) {
    const int n = (int)d_in.size();
    std::vector<double> d = d_in, e(n, 0.0);
    for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 60; ++iter) {
            // look for a negligible off-diagonal element at or after l
            int m = l;
            for (; m + 1 < n; ++m) {
                const double scale = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * scale) break;
            }
            if (m == l) break;
            // Wilkinson shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    std::sort(d.begin(), d.end());
    return d;
}

// Number of eigenvalues of T below x: negative pivots of T - x I = L D L^T.
inline int tridiag_count_below(const std::vector<double> &d, const std::vector<double> &e, double x) {
    int neg = 0;
    double piv = 1.0;
    for (size_t k = 0; k < d.size(); ++k) {
        const double off = k ? e[k - 1] * e[k - 1] / piv : 0.0;
        piv = d[k] - x - off;
        if (piv == 0.0) piv = -1e-300;
        neg += piv < 0.0;
    }
    return neg;
}

// Lowest eigenvalue of T by bisection.  `hint` (a previous lowest Ritz
// value, an upper bound by interlacing) and `step` (its last change) narrow
// the starting bracket; the result is accurate to a few ulps.
inline double tridiag_lowest(const std::vector<double> &d, const std::vector<double> &e, double hint, double step) {
    const int n = (int)d.size();
    double glo = d[0], ghi = d[0];
    for (int i = 0; i < n; ++i) {
        const double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        glo = std::min(glo, d[i] - r);
        ghi = std::max(ghi, d[i] + r);
    }
    const double scale = std::max(std::fabs(glo), std::fabs(ghi)) + 1e-300;
    double hi = ghi + 1e-12 * scale, lo = glo - 1e-12 * scale;
    if (std::isfinite(hint) && hint < hi) {
        const double h = hint + 1e-13 * scale;
        if (tridiag_count_below(d, e, h) >= 1) {
            hi = h;
            double w = std::max(4.0 * std::fabs(step), 1e-10 * scale);
            while (hi - w > lo && tridiag_count_below(d, e, hi - w) >= 1) w *= 8.0;
            lo = std::max(lo, hi - w);
        }
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (tridiag_count_below(d, e, mid) >= 1) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Unit eigenvector of T for eigenvalue lam by inverse iteration:
// solve (T - sigma I) x = b with Gaussian elimination and partial pivoting
// (at most two super-diagonals of fill), three sweeps.
inline std::vector<double> tridiag_eigenvector(const std::vector<double> &d, const std::vector<double> &e, double lam) {
    const int n = (int)d.size();
    std::vector<double> x(n, 1.0);
    if (n == 1) return x;
    double norm = 0.0;
    for (int i = 0; i < n; ++i) norm = std::max(norm, std::fabs(d[i]) + (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0));
    const double sigma = lam - 1e-14 * std::max(norm, 1e-300);
    for (int it = 0; it < 3; ++it) {
        // rows: sub a[i] (below diag), diag b[i], super c1[i], c2[i]
        std::vector<double> a(n, 0.0), b(n), c1(n, 0.0), c2(n, 0.0), rhs = x;
        for (int i = 0; i < n; ++i) {
            b[i] = d[i] - sigma;
            if (i + 1 < n) { c1[i] = e[i]; a[i + 1] = e[i]; }
        }
        for (int i = 0; i + 1 < n; ++i) {
            // pivot between row i and row i+1 on column i
            if (std::fabs(a[i + 1]) > std::fabs(b[i])) {
                std::swap(b[i], a[i + 1]);
                std::swap(c1[i], b[i + 1]);
                std::swap(c2[i], c1[i + 1]);
                std::swap(rhs[i], rhs[i + 1]);
            }
            if (b[i] == 0.0) b[i] = 1e-300;
            const double f = a[i + 1] / b[i];
            a[i + 1] = 0.0;
            b[i + 1] -= f * c1[i];
            c1[i + 1] -= f * c2[i];
            rhs[i + 1] -= f * rhs[i];
        }
        if (b[n - 1] == 0.0) b[n - 1] = 1e-300;
        for (int i = n - 1; i >= 0; --i) {
            double v = rhs[i];
            if (i + 1 < n) v -= c1[i] * x[i + 1];
            if (i + 2 < n) v -= c2[i] * x[i + 2];
            x[i] = v / b[i];
        }
        double nx = 0.0;
        for (double v : x) nx += v * v;
        nx = std::sqrt(nx);
        for (double &v : x) v /= nx;
    }
    return x;
}

}  // namespace ecut
