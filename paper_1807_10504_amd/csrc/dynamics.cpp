// Enclosed area / volume of revolution, vertical centroid, and the mass
// correction of the interface markers (Section 2.1, conservation of mass;
// the non-inertial frame of the free-fall runs measures the drop's centre of
// mass the same way).
//
// Host FP64 on the markers, which the 2D and axisymmetric steps keep on the
// host for the B-spline relocation.
//   planar: signed shoelace area and centroid of the closed polygon;
//   axisymmetric (axis x = axis_x, the curve mirrored about it): Green's
//   theorem on the half x >= axis_x, V = pi sum int r^2 dz and
//   V z_c = pi sum int z r^2 dz, exact on straight segments.
// Mass correction: when |V - V0| > trigger V0, every marker moves by one
// distance delta along its unit normal toward the drop, delta found by
// bisection on [-h, h] until |V - V0| <= tol V0.
#include <cmath>
#include <string>
#include <vector>

#include "freefall.h"

namespace ib {
int fail(int code, const std::string& msg);
}

namespace {

void measure(int n, const double* X, double axis_x, double* vol, double* com) {
    if (std::isnan(axis_x)) {
        double A = 0.0, cy = 0.0;
        for (int k = 0; k < n; ++k) {
            const int q = k + 1 == n ? 0 : k + 1;
            const double x = X[2 * k], y = X[2 * k + 1], xn = X[2 * q], yn = X[2 * q + 1];
            const double cr = x * yn - xn * y;
            A += cr;
            cy += (y + yn) * cr;
        }
        A *= 0.5;
        *vol = A;
        *com = cy / (6.0 * A);
        return;
    }
    double v = 0.0, vz = 0.0;
    for (int k = 0; k < n; ++k) {
        const int q = k + 1 == n ? 0 : k + 1;
        const double r0 = X[2 * k] - axis_x, r1 = X[2 * q] - axis_x;
        if (r0 < -1e-12 || r1 < -1e-12) continue;  // the mirrored half
        const double a = std::fmax(r0, 0.0), b = std::fmax(r1, 0.0) - a;
        const double c = X[2 * k + 1], d = X[2 * q + 1] - c;
        const double m2 = a * a + a * b + b * b / 3.0;
        v += d * m2;
        vz += d * (c * m2 + d * (a * a / 2.0 + 2.0 * a * b / 3.0 + b * b / 4.0));
    }
    *vol = M_PI * v;
    *com = (M_PI * vz) / (M_PI * v);
}

// volume enclosed by a closed outward mesh and the y of its centroid (the
// divergence theorem over the tetrahedra origin, a, b, c)
void mesh_measure(int nv, const double* V, int nt, const int* T, double* vol, double* com) {
    (void)nv;
    double v = 0.0, vy = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double* a = V + 3 * T[3 * t];
        const double* b = V + 3 * T[3 * t + 1];
        const double* c = V + 3 * T[3 * t + 2];
        const double cx = b[1] * c[2] - b[2] * c[1], cy = b[2] * c[0] - b[0] * c[2], cz = b[0] * c[1] - b[1] * c[0];
        const double vt = (a[0] * cx + a[1] * cy + a[2] * cz) / 6.0;
        v += vt;
        vy += vt * (a[1] + b[1] + c[1]) / 4.0;
    }
    *vol = v;
    *com = vy / v;
}

}  // namespace

extern "C" int ib_mesh_measure(int nv, const double* V, int nt, const int* T, double* vol, double* com) {
    if (nv < 4 || nt < 4 || !V || !T || !vol || !com) return ib::fail(IB_EINVAL, "ib_mesh_measure: arguments");
    for (long i = 0; i < 3L * nt; ++i)
        if (T[i] < 0 || T[i] >= nv) return ib::fail(IB_EINVAL, "ib_mesh_measure: triangle index out of range");
    mesh_measure(nv, V, nt, T, vol, com);
    if (!std::isfinite(*vol) || !(*vol > 0.0)) return ib::fail(IB_EGEOM, "ib_mesh_measure: no enclosed volume");
    return IB_OK;
}

extern "C" int ib_mesh_mass_correct(int nv, double* V, const double* nrm, int nt, const int* T, double target,
                                    double h, double trigger, double tol, double* delta) {
    if (nv < 4 || nt < 4 || !V || !nrm || !T || !(target > 0.0) || !(h > 0.0))
        return ib::fail(IB_EINVAL, "ib_mesh_mass_correct: arguments");
    for (long i = 0; i < 3L * nt; ++i)
        if (T[i] < 0 || T[i] >= nv) return ib::fail(IB_EINVAL, "ib_mesh_mass_correct: triangle index out of range");
    double v, c;
    mesh_measure(nv, V, nt, T, &v, &c);
    if (delta) *delta = 0.0;
    if (std::fabs(v - target) <= trigger * target) return IB_OK;
    std::vector<double> Y(3 * (size_t)nv);
    double lo = -h, hi = h, mid = 0.0;
    for (int it = 0; it < 200; ++it) {
        mid = 0.5 * (lo + hi);
        for (size_t k = 0; k < 3 * (size_t)nv; ++k) Y[k] = V[k] + mid * nrm[k];
        mesh_measure(nv, Y.data(), nt, T, &v, &c);
        if (std::fabs(v - target) <= tol * target) break;
        if (v > target)
            lo = mid;
        else
            hi = mid;
    }
    for (size_t k = 0; k < 3 * (size_t)nv; ++k) V[k] = Y[k];
    if (delta) *delta = mid;
    return IB_OK;
}

extern "C" int ib_enclosed_measure(int n, const double* X, double axis_x, double* vol, double* com) {
    if (n < 3 || !X || !vol || !com) return ib::fail(IB_EINVAL, "ib_enclosed_measure: arguments");
    measure(n, X, axis_x, vol, com);
    if (!std::isfinite(*vol) || *vol == 0.0) return ib::fail(IB_EGEOM, "ib_enclosed_measure: empty curve");
    return IB_OK;
}

extern "C" int ib_mass_correct(int n, double* X, const double* nrm, double target, double axis_x,
                               double h, double trigger, double tol, double* delta) {
    if (n < 3 || !X || !nrm || !(target > 0.0) || !(h > 0.0))
        return ib::fail(IB_EINVAL, "ib_mass_correct: arguments");
    double v, c;
    measure(n, X, axis_x, &v, &c);
    if (delta) *delta = 0.0;
    if (std::fabs(v - target) <= trigger * target) return IB_OK;
    std::vector<double> Y(2 * (size_t)n);
    double lo = -h, hi = h, mid = 0.0;
    for (int it = 0; it < 200; ++it) {
        mid = 0.5 * (lo + hi);
        for (int k = 0; k < 2 * n; ++k) Y[k] = X[k] + mid * nrm[k];
        measure(n, Y.data(), axis_x, &v, &c);
        if (std::fabs(v - target) <= tol * target) break;
        if (v > target)
            lo = mid;
        else
            hi = mid;
    }
    for (int k = 0; k < 2 * n; ++k) X[k] = Y[k];
    if (delta) *delta = mid;
    return IB_OK;
}

namespace ib {

int freefall_begin(FreeFall* s, const ib_flow_params* fp, int n, const double* X, double axis_x,
                   double dt, ib_flow_stats* st, const double** mass_target, int nt, const int* T) {
    *mass_target = nullptr;
    st->frame_a = st->com = st->measure = st->mass_delta = 0.0;
    if (!fp->frame && fp->mass_every <= 0) return IB_OK;
    double v, com;
    const int rc = nt > 0 ? ib_mesh_measure(n, X, nt, T, &v, &com) : ib_enclosed_measure(n, X, axis_x, &v, &com);
    if (rc != IB_OK) return IB_EGEOM;
    if (!s->have) {
        s->com0 = s->com_prev = com;
        s->vol0 = v;
        s->nstep = 0;
        s->have = 1;
    }
    st->com = com;
    st->measure = v;
    if (fp->frame) st->frame_a = -fp->c1 * (com - s->com0) / dt - fp->c2 * (com - s->com_prev) / dt;
    s->com_prev = com;
    s->nstep += 1;
    if (fp->mass_every > 0 && s->nstep % fp->mass_every == 0)
        *mass_target = fp->mass_target > 0.0 ? &fp->mass_target : &s->vol0;
    return IB_OK;
}

}  // namespace ib

// Marker deletion and addition of the conventional front tracking (Section
// 2.2, after Singh et al.; the B-spline relocation replaces it): walk the
// closed curve from marker 0 deleting markers closer than lo h to the last kept
// one (and the last kept one when it ends closer than lo h to marker 0, while
// more than three remain), then put one marker at the midpoint of every kept
// gap longer than hi h.
extern "C" int ib_markers_add_delete(int n, const double* X, double h, double lo, double hi, int max_out,
                                     double* X_out, int* n_out) {
    if (n < 3 || !X || !X_out || !n_out || !(h > 0.0) || !(lo >= 0.0) || !(hi > lo) || max_out < 1)
        return ib::fail(IB_EINVAL, "ib_markers_add_delete: arguments");
    std::vector<double> kept;
    kept.reserve(2 * (size_t)n);
    kept.push_back(X[0]);
    kept.push_back(X[1]);
    for (int k = 1; k < n; ++k) {
        const double* last = &kept[kept.size() - 2];
        if (std::hypot(X[2 * k] - last[0], X[2 * k + 1] - last[1]) >= lo * h) {
            kept.push_back(X[2 * k]);
            kept.push_back(X[2 * k + 1]);
        }
    }
    size_t m = kept.size() / 2;
    if (m > 3 && std::hypot(kept[0] - kept[2 * m - 2], kept[1] - kept[2 * m - 1]) < lo * h) --m;
    int out = 0;
    for (size_t k = 0; k < m; ++k) {
        const size_t q = k + 1 == m ? 0 : k + 1;
        const double ax = kept[2 * k], ay = kept[2 * k + 1], bx = kept[2 * q], by = kept[2 * q + 1];
        if (out >= max_out) return ib::fail(IB_EINVAL, "ib_markers_add_delete: max_out too small");
        X_out[2 * out] = ax;
        X_out[2 * out + 1] = ay;
        ++out;
        if (std::hypot(bx - ax, by - ay) > hi * h) {
            if (out >= max_out) return ib::fail(IB_EINVAL, "ib_markers_add_delete: max_out too small");
            X_out[2 * out] = 0.5 * (ax + bx);
            X_out[2 * out + 1] = 0.5 * (ay + by);
            ++out;
        }
    }
    *n_out = out;
    return IB_OK;
}
