// Least-squares B-spline relocation of 2D interface markers (Section 4).
//
// Host FP64, compiled without floating-point contraction: every value is
// produced by + - * / and sqrt in the order written here, so a run is
// reproducible bit for bit on any IEEE binary64 machine.
//
// Steps: advance X* = X + dt U; chord-length parameters along the closed
// polyline from the first marker; periodic uniform knots with g = max(7,
// round(L / 1.5h)) spans (the knot spacing is the 1.5-cell progression of the
// paper adjusted to close the curve); cubic basis by the Cox-de Boor
// recursion (eq bspline); least squares for x(t) and y(t) separately (eq
// bspline_ls) through the normal equations and a Cholesky factorisation;
// new markers at constant arc spacing (8-point Gauss-Legendre arc length per
// span, 6 Newton steps per marker); curvature from unit tangents half-way
// between markers (eqs ten_f, b_tan).
//
// The normal matrix is cyclic banded; the factorisation visits only the
// envelope of each row (the entries outside it are exact zeros that stay
// zero), which gives the same floating-point result as a dense
// factorisation in row order.
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ibproj.h"

namespace ib {
int fail(int code, const std::string& msg);
}

namespace {

// 8-point Gauss-Legendre nodes and weights on [-1, 1] (Abramowitz & Stegun 25.4)
const double kGX[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                       -0.1834346424956498, 0.1834346424956498,  0.5255324099163290,
                       0.7966664774136267,  0.9602898564975363};
const double kGW[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                       0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                       0.2223810344533745, 0.1012285362903763};
const int kNewton = 6;

// Cox-de Boor on local knots kappa_j = j: cubic values b3[0..3] for basis
// offsets -3..0 and quadratic values b2[0..2] for offsets -2..0
void basis(double u, double b3[4], double b2[3]) {
    // value arrays indexed by offset + 3 (offsets -3..0), zero outside range
    double prev[5] = {0.0, 0.0, 0.0, 1.0, 0.0};  // degree 0: offset 0 -> 1
    double cur[5];
    for (int d = 1; d <= 3; ++d) {
        for (int q = 0; q < 5; ++q) cur[q] = 0.0;
        for (int i = -d; i <= 0; ++i) {
            double lo = prev[i + 3];
            double hi = prev[i + 4];
            double a = (u - (double)i) / ((double)(i + d) - (double)i);
            double b = ((double)(i + d + 1) - u) / ((double)(i + d + 1) - (double)(i + 1));
            cur[i + 3] = a * lo + b * hi;
        }
        if (d == 2) {
            b2[0] = cur[1];
            b2[1] = cur[2];
            b2[2] = cur[3];
        }
        for (int q = 0; q < 5; ++q) prev[q] = cur[q];
        prev[4] = 0.0;
    }
    b3[0] = prev[0];
    b3[1] = prev[1];
    b3[2] = prev[2];
    b3[3] = prev[3];
}

struct Curve {
    std::vector<double> cx, cy;
    int g;

    void point(int s, double u, double* x, double* y) const {
        double b3[4], b2[3];
        basis(u, b3, b2);
        double ax = 0.0, ay = 0.0;
        for (int r = 0; r < 4; ++r) {
            int i = ((s - 3 + r) % g + g) % g;
            ax = ax + cx[i] * b3[r];
            ay = ay + cy[i] * b3[r];
        }
        *x = ax;
        *y = ay;
    }

    void deriv(int s, double u, double* dx, double* dy) const {
        double b3[4], b2[3];
        basis(u, b3, b2);
        // quadratic values by offset -2..0, zero elsewhere
        double q[5] = {0.0, b2[0], b2[1], b2[2], 0.0};  // index offset + 3
        double ax = 0.0, ay = 0.0;
        for (int r = 0; r < 4; ++r) {
            int off = r - 3;
            double db = (3.0 / 3.0) * q[off + 3] - (3.0 / 3.0) * q[off + 4];
            int i = ((s - 3 + r) % g + g) % g;
            ax = ax + cx[i] * db;
            ay = ay + cy[i] * db;
        }
        *dx = ax;
        *dy = ay;
    }

    double speed(int s, double u) const {
        double dx, dy;
        deriv(s, u, &dx, &dy);
        return std::sqrt(dx * dx + dy * dy);
    }

    double arc(int s, double u) const {
        double half = 0.5 * u;
        double acc = 0.0;
        for (int q = 0; q < 8; ++q) acc = acc + kGW[q] * speed(s, half * (1.0 + kGX[q]));
        return half * acc;
    }
};

int span_of(double v, int g) {
    int s = (int)std::floor(v);
    if (s > g - 1) s = g - 1;
    if (s < 0) s = 0;
    return s;
}

// returns false when the normal matrix is not positive definite
bool fit(const std::vector<double>& X, int N, double h, Curve* out) {
    std::vector<double> t(N + 1);
    t[0] = 0.0;
    for (int k = 0; k < N; ++k) {
        int k1 = k + 1 == N ? 0 : k + 1;
        double dx = X[2 * k1] - X[2 * k];
        double dy = X[2 * k1 + 1] - X[2 * k + 1];
        t[k + 1] = t[k] + std::sqrt(dx * dx + dy * dy);
    }
    double L = t[N];
    int g = (int)std::floor(L / (1.5 * h) + 0.5);
    if (g < 7) g = 7;
    double tau = L / g;
    // normal matrix on the cyclic band: entry (i, j) with j = i + o (mod g),
    // o in -3..3, at B[7 i + o + 3] (the basis of a point spans four cyclic
    // neighbours, so no other entry is touched); accumulated in the order of a
    // dense assembly
    std::vector<double> B((size_t)7 * g, 0.0), bx(g, 0.0), by(g, 0.0);
    auto boff = [&](int i, int j) {
        int o = j - i;
        if (o > 3) o -= g;
        if (o < -3) o += g;
        return 7 * i + o + 3;
    };
    for (int k = 0; k < N; ++k) {
        double v = t[k] / tau;
        int s = span_of(v, g);
        double u = v - (double)s;
        double b3[4], b2[3];
        basis(u, b3, b2);
        int idx[4];
        for (int r = 0; r < 4; ++r) idx[r] = ((s - 3 + r) % g + g) % g;
        double xk = X[2 * k], yk = X[2 * k + 1];
        for (int a = 0; a < 4; ++a) {
            int ia = idx[a];
            bx[ia] = bx[ia] + b3[a] * xk;
            by[ia] = by[ia] + b3[a] * yk;
            for (int b = 0; b < 4; ++b) {
                int ib = idx[b];
                B[boff(ia, ib)] = B[boff(ia, ib)] + b3[a] * b3[b];
            }
        }
    }
    // value of the (dense) normal matrix at (i, j): zero off the cyclic band
    auto Mv = [&](int i, int j) {
        int o = j - i;
        if (o > 3) o -= g;
        if (o < -3) o += g;
        return (o >= -3 && o <= 3) ? B[7 * i + o + 3] : 0.0;
    };
    // envelope: first nonzero column of each row of the lower triangle
    // (only the band columns i - 3 .. i and, near the end, the wrapped columns
    // 0 .. i + 3 - g can be nonzero)
    std::vector<int> first(g);
    for (int i = 0; i < g; ++i) {
        int f = i;
        for (int j = 0; j <= i + 3 - g && j <= i; ++j)
            if (Mv(i, j) != 0.0) {
                f = j;
                break;
            }
        if (f == i)
            for (int j = i - 3 < 0 ? 0 : i - 3; j <= i; ++j)
                if (Mv(i, j) != 0.0) {
                    f = j;
                    break;
                }
        first[i] = f;
    }
    // Cholesky in row order over the envelope (fill-in stays inside it); row i
    // of the factor is stored from column first[i] on (profile storage)
    std::vector<size_t> rs(g + 1, 0);
    for (int i = 0; i < g; ++i) rs[i + 1] = rs[i] + (size_t)(i - first[i] + 1);
    std::vector<double> Lp(rs[g], 0.0);
    auto Lat = [&](int i, int k) -> double& { return Lp[rs[i] + (size_t)(k - first[i])]; };
    for (int i = 0; i < g; ++i) {
        for (int j = first[i]; j <= i; ++j) {
            double s_ = Mv(i, j);
            int k0 = first[i] > first[j] ? first[i] : first[j];
            for (int k = k0; k < j; ++k) s_ = s_ - Lat(i, k) * Lat(j, k);
            if (i == j) {
                if (!(s_ > 0.0)) return false;
                Lat(i, i) = std::sqrt(s_);
            } else {
                Lat(i, j) = s_ / Lat(j, j);
            }
        }
    }
    // rows whose envelope reaches back to column i, for the backward solve
    std::vector<std::vector<int>> below(g);
    for (int k = 0; k < g; ++k)
        for (int i = first[k]; i < k; ++i) below[i].push_back(k);
    auto solve = [&](const std::vector<double>& rhs, std::vector<double>& c) {
        std::vector<double> z(g);
        for (int i = 0; i < g; ++i) {
            double s_ = rhs[i];
            for (int k = first[i]; k < i; ++k) s_ = s_ - Lat(i, k) * z[k];
            z[i] = s_ / Lat(i, i);
        }
        c.assign(g, 0.0);
        for (int i = g - 1; i >= 0; --i) {
            double s_ = z[i];
            for (int k : below[i]) s_ = s_ - Lat(k, i) * c[k];
            c[i] = s_ / Lat(i, i);
        }
    };
    out->g = g;
    solve(bx, out->cx);
    solve(by, out->cy);
    return true;
}

void locate(const Curve& c, const std::vector<double>& S, const std::vector<double>& ell,
            double sigma, int* s_io, double* u_out) {
    int s = *s_io;
    while (s < c.g - 1 && S[s + 1] <= sigma) s = s + 1;
    double target = sigma - S[s];
    double u = target / ell[s];
    for (int it = 0; it < kNewton; ++it) u = u - (c.arc(s, u) - target) / c.speed(s, u);
    *s_io = s;
    *u_out = u;
}

}  // namespace

extern "C" int ib_relocate_bspline(int n, const double* X, const double* U, double dt, double h,
                                   double sigma, double* X_out, double* fs_out, double* ds_out,
                                   double* nrm_out) {
    if (n < 3 || !X || !U || !X_out || !fs_out || !ds_out || !(h > 0.0))
        return ib::fail(IB_EINVAL, "ib_relocate_bspline: bad argument");
    std::vector<double> Xs(2 * (size_t)n);
    for (int k = 0; k < n; ++k) {
        Xs[2 * k] = X[2 * k] + dt * U[2 * k];
        Xs[2 * k + 1] = X[2 * k + 1] + dt * U[2 * k + 1];
    }
    Curve c;
    if (!fit(Xs, n, h, &c))
        return ib::fail(IB_EGEOM, "ib_relocate_bspline: least-squares matrix not positive definite");
    int g = c.g;
    std::vector<double> ell(g), S(g + 1);
    // the markers are independent once the curve is fitted: spans, arc lengths and
    // the Newton inversions run in parallel, each with the arithmetic of the
    // sequential loop (the span search from 0 ends where a search from the
    // previous marker's span would)
#pragma omp parallel for schedule(static) if (g >= 64)
    for (int s = 0; s < g; ++s) ell[s] = c.arc(s, 1.0);
    S[0] = 0.0;
    for (int s = 0; s < g; ++s) S[s + 1] = S[s] + ell[s];
    double Lc = S[g];
    double ds = Lc / n;
#pragma omp parallel for schedule(static) if (n >= 64)
    for (int k = 0; k < n; ++k) {
        double u;
        int s = 0;
        locate(c, S, ell, (double)k * ds, &s, &u);
        c.point(s, u, &X_out[2 * k], &X_out[2 * k + 1]);
        double dx, dy;
        c.deriv(s, u, &dx, &dy);
        double sp = std::sqrt(dx * dx + dy * dy);
        if (nrm_out) {
            nrm_out[2 * k] = -dy / sp;
            nrm_out[2 * k + 1] = dx / sp;
        }
    }
    std::vector<double> T(2 * (size_t)n);
#pragma omp parallel for schedule(static) if (n >= 64)
    for (int k = 0; k < n; ++k) {
        double u;
        int s = 0;
        locate(c, S, ell, ((double)k + 0.5) * ds, &s, &u);
        double dx, dy;
        c.deriv(s, u, &dx, &dy);
        double sp = std::sqrt(dx * dx + dy * dy);
        T[2 * k] = dx / sp;
        T[2 * k + 1] = dy / sp;
    }
    for (int k = 0; k < n; ++k) {
        int km = k == 0 ? n - 1 : k - 1;
        double tmx = T[2 * km], tmy = T[2 * km + 1];
        double tpx = T[2 * k], tpy = T[2 * k + 1];
        double ddx = tpx - tmx, ddy = tpy - tmy;
        double kap = std::sqrt(ddx * ddx + ddy * ddy) / ds;
        if (tmx * tpy - tmy * tpx < 0.0) kap = -kap;
        fs_out[k] = sigma * kap;
        ds_out[k] = ds;
    }
    return IB_OK;
}
