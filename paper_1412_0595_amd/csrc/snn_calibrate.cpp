// Host-side calibration of the conductance scale (Section 5.1): the selection
// procedure of Fig. 1 over the per-run table of a conductance-scaling sweep,
// and the least-squares fit of the inverse law gScale = k1 / (k2 + nConn) + k3
// (Tables 1 and 2).  The table has one row per run and is tiny (hundreds of
// rows); the sweep that produces it runs on the GPU.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "../../include/snn.h"

namespace snn {
int set_error(int code, const char *msg);  // message for snn_last_error
}

namespace {

struct Line {
    double k1, k3, sse;
};

// For a fixed k2 the law is a straight line in u = 1 / (k2 + nConn): its
// least-squares slope (k1) and intercept (k3) from the centred sums.
Line line_fit(const std::vector<double> &x, const std::vector<double> &y, double k2)
{
    const size_t m = x.size();
    std::vector<double> u(m);
    double su = 0.0, sy = 0.0;
    for (size_t i = 0; i < m; ++i) {
        u[i] = 1.0 / (k2 + x[i]);
        su += u[i];
        sy += y[i];
    }
    const double mu = su / m, my = sy / m;
    double suu = 0.0, suy = 0.0;
    for (size_t i = 0; i < m; ++i) {
        suu += (u[i] - mu) * (u[i] - mu);
        suy += (u[i] - mu) * (y[i] - my);
    }
    Line L{0.0, my, 0.0};
    if (suu > 0.0) {
        L.k1 = suy / suu;
        L.k3 = my - L.k1 * mu;
    }
    for (size_t i = 0; i < m; ++i) {
        const double r = L.k1 * u[i] + L.k3 - y[i];
        L.sse += r * r;
    }
    return L;
}

double sse3(const std::vector<double> &x, const std::vector<double> &y, const double *k)
{
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) {
        const double r = k[0] / (k[1] + x[i]) + k[2] - y[i];
        s += r * r;
    }
    return s;
}

// Solve the 3x3 symmetric system A d = b by Gaussian elimination with partial
// pivoting; false when singular.
bool solve3(double A[3][3], double b[3], double d[3])
{
    int p[3] = {0, 1, 2};
    for (int c = 0; c < 3; ++c) {
        int best = c;
        for (int r = c + 1; r < 3; ++r)
            if (std::fabs(A[p[r]][c]) > std::fabs(A[p[best]][c])) best = r;
        std::swap(p[c], p[best]);
        const double piv = A[p[c]][c];
        if (!(std::fabs(piv) > 0.0)) return false;
        for (int r = c + 1; r < 3; ++r) {
            const double f = A[p[r]][c] / piv;
            for (int j = c; j < 3; ++j) A[p[r]][j] -= f * A[p[c]][j];
            b[p[r]] -= f * b[p[c]];
        }
    }
    for (int c = 2; c >= 0; --c) {
        double s = b[p[c]];
        for (int j = c + 1; j < 3; ++j) s -= A[p[c]][j] * d[j];
        d[c] = s / A[p[c]][c];
    }
    return std::isfinite(d[0]) && std::isfinite(d[1]) && std::isfinite(d[2]);
}

}  // namespace

extern "C" int snn_gscale_select(int64_t n_runs, const double *n_conn, const double *g_scale,
                                 const double *avg_spike, const int32_t *n_nans, int64_t ref_run,
                                 int64_t *n_groups, double *group_n_conn, int64_t *picked)
{
    if (n_runs < 1 || !n_conn || !g_scale || !avg_spike || !n_nans || !n_groups || !group_n_conn || !picked)
        return snn::set_error(SNN_EINVAL, "gscale_select: need n_runs >= 1 and non-NULL arrays");
    if (ref_run < 0 || ref_run >= n_runs)
        return snn::set_error(SNN_EINVAL, "gscale_select: reference run out of range");
    for (int64_t i = 0; i < n_runs; ++i)
        if (!std::isfinite(n_conn[i]) || !std::isfinite(g_scale[i]))
            return snn::set_error(SNN_EINVAL, "gscale_select: nConn and gScale must be finite");
    const double ref = avg_spike[ref_run];
    if (n_nans[ref_run] != 0 || !std::isfinite(ref))
        return snn::set_error(SNN_EINVAL, "gscale_select: the reference run has NaNs");

    std::vector<int64_t> ord(n_runs);
    std::iota(ord.begin(), ord.end(), int64_t(0));
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return n_conn[a] < n_conn[b]; });
    int64_t g = 0;
    for (int64_t s = 0; s < n_runs;) {
        int64_t e = s;
        int64_t best = -1;
        double best_d = 0.0;
        // runs of one nConn, in run order (the sort is stable)
        for (; e < n_runs && n_conn[ord[e]] == n_conn[ord[s]]; ++e) {
            const int64_t i = ord[e];
            if (n_nans[i] != 0 || !std::isfinite(avg_spike[i])) continue;
            const double d = std::fabs(avg_spike[i] - ref);
            if (best < 0 || d < best_d || (d == best_d && g_scale[i] < g_scale[best])) {
                best = i;
                best_d = d;
            }
        }
        group_n_conn[g] = n_conn[ord[s]];
        picked[g] = best;
        ++g;
        s = e;
    }
    *n_groups = g;
    return SNN_OK;
}

extern "C" int snn_gscale_fit(int64_t n_points, const double *n_conn, const double *g_scale, double *k,
                              double *mape_percent)
{
    if (n_points < 3 || !n_conn || !g_scale || !k)
        return snn::set_error(SNN_EINVAL, "gscale_fit: need at least three points and non-NULL arrays");
    std::vector<double> x(n_conn, n_conn + n_points), y(g_scale, g_scale + n_points);
    for (int64_t i = 0; i < n_points; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || y[i] <= 0.0)
            return snn::set_error(SNN_EINVAL, "gscale_fit: nConn must be finite and gScale finite and > 0");
    std::vector<double> xs(x);
    std::sort(xs.begin(), xs.end());
    if (std::unique(xs.begin(), xs.end()) - xs.begin() < 3)
        return snn::set_error(SNN_EINVAL, "gscale_fit: need at least three distinct nConn");
    const double lo = xs.front();
    const double L = std::max({xs.back() - lo, std::fabs(lo), 1.0});

    // k2 = t - min(nConn) with t > 0: scan log t over 16 decades either side
    // of the data's scale, then refine the best bracket by golden section.
    const int kPerDecade = 16, kDecades = 8, nGrid = 2 * kDecades * kPerDecade + 1;
    auto k2_of = [&](double s) { return std::exp(s) - lo; };
    const double s0 = std::log(L) - kDecades * std::log(10.0), ds = std::log(10.0) / kPerDecade;
    int jb = 0;
    double fb = INFINITY;
    for (int j = 0; j < nGrid; ++j) {
        const double f = line_fit(x, y, k2_of(s0 + j * ds)).sse;
        if (f < fb) {
            fb = f;
            jb = j;
        }
    }
    if (!std::isfinite(fb)) return snn::set_error(SNN_ERANGE, "gscale_fit: no finite fit");
    // As k2 grows the law tends to a straight line in nConn; when no k2 does
    // better than that line (beyond rounding) the best k2 is unbounded.
    double mx = 0.0, my = 0.0, sxx = 0.0, sxy = 0.0, syy = 0.0, yy = 0.0;
    for (size_t i = 0; i < x.size(); ++i) {
        mx += x[i];
        my += y[i];
        yy += y[i] * y[i];
    }
    mx /= x.size();
    my /= x.size();
    for (size_t i = 0; i < x.size(); ++i) {
        sxx += (x[i] - mx) * (x[i] - mx);
        sxy += (x[i] - mx) * (y[i] - my);
        syy += (y[i] - my) * (y[i] - my);
    }
    const double line_sse = std::max(0.0, syy - sxy * sxy / sxx);
    if (jb == nGrid - 1 || fb >= line_sse * (1.0 - 1e-9) - 1e-24 * yy)
        return snn::set_error(SNN_ERANGE, "gscale_fit: the best k2 runs to infinity (the points lie on a straight line)");
    if (jb == 0) return snn::set_error(SNN_ERANGE, "gscale_fit: the best k2 puts the pole on the smallest nConn");
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = s0 + (jb - 1) * ds, b = s0 + (jb + 1) * ds;
    double c = b - gr * (b - a), d = a + gr * (b - a);
    double fc = line_fit(x, y, k2_of(c)).sse, fd = line_fit(x, y, k2_of(d)).sse;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(1.0, std::fabs(a)); ++it) {
        if (fc <= fd) {
            b = d; d = c; fd = fc;
            c = b - gr * (b - a);
            fc = line_fit(x, y, k2_of(c)).sse;
        } else {
            a = c; c = d; fc = fd;
            d = a + gr * (b - a);
            fd = line_fit(x, y, k2_of(d)).sse;
        }
    }
    const double sb = fc <= fd ? c : d;
    const Line Lb = line_fit(x, y, k2_of(sb));
    double kk[3] = {Lb.k1, k2_of(sb), Lb.k3};
    double f = sse3(x, y, kk);

    // Gauss-Newton polish of all three coefficients (step halving keeps the
    // sum of squares decreasing and the pole left of the smallest nConn)
    for (int it = 0; it < 50; ++it) {
        double A[3][3] = {}, g[3] = {};
        for (size_t i = 0; i < x.size(); ++i) {
            const double u = 1.0 / (kk[1] + x[i]);
            const double r = kk[0] * u + kk[2] - y[i];
            const double J[3] = {u, -kk[0] * u * u, 1.0};
            for (int p = 0; p < 3; ++p) {
                g[p] -= J[p] * r;
                for (int q = 0; q < 3; ++q) A[p][q] += J[p] * J[q];
            }
        }
        double D[3], step[3];
        for (int p = 0; p < 3; ++p) D[p] = A[p][p] > 0.0 ? 1.0 / std::sqrt(A[p][p]) : 1.0;
        for (int p = 0; p < 3; ++p) {
            g[p] *= D[p];
            for (int q = 0; q < 3; ++q) A[p][q] *= D[p] * D[q];
        }
        if (!solve3(A, g, step)) break;
        for (int p = 0; p < 3; ++p) step[p] *= D[p];
        bool moved = false;
        for (double h = 1.0; h > 1e-10; h *= 0.5) {
            const double cand[3] = {kk[0] + h * step[0], kk[1] + h * step[1], kk[2] + h * step[2]};
            if (!(cand[1] + lo > 0.0)) continue;
            const double fn = sse3(x, y, cand);
            if (fn < f) {
                std::copy(cand, cand + 3, kk);
                moved = f - fn > 1e-15 * f;
                f = fn;
                break;
            }
        }
        if (!moved) break;
    }
    std::copy(kk, kk + 3, k);
    if (mape_percent) {
        double s = 0.0;
        for (size_t i = 0; i < x.size(); ++i) s += std::fabs(kk[0] / (kk[1] + x[i]) + kk[2] - y[i]) / std::fabs(y[i]);
        *mape_percent = 100.0 * s / x.size();
    }
    return SNN_OK;
}
