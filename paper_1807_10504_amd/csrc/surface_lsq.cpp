// Local least-squares reconstruction of a moving closed triangulated surface:
// the 3D counterpart of the least-squares B-spline of Section 4 (which the
// paper leaves to future work for surfaces). Host FP64.
//
// Per vertex v: frame (t1, t2, n), n the inward angle-weighted normal, t1 the
// tangent projection of the coordinate axis least aligned with n, t2 = n x t1;
// the vertex's two-ring (v included) in local coordinates scaled by L (the mean
// distance of the ring's other vertices from v); the least-squares quadric
// z = g + d x + e y + a x^2 + b xy + c y^2 by Householder QR. Then
//   X'_v = X_v + g L n,  n'_v = (n - d t1 - e t2)/sqrt(1 + d^2 + e^2),
//   kappa = [(1 + e^2) 2a - 2de b + (1 + d^2) 2c] / (L (1 + d^2 + e^2)^(3/2)),
// fs = sigma kappa, ds = a third of the adjacent triangles' areas of the moved
// mesh.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ibproj.h"

namespace ib {
int fail(int code, const std::string& msg);
}

namespace {

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 at(const double* V, int i) { return {V[3 * i], V[3 * i + 1], V[3 * i + 2]}; }

// inward unit angle-weighted vertex normals (triangles outward counter-clockwise)
void inward_normals(int nv, const double* V, int nt, const int* T, std::vector<V3>& out) {
    out.assign(nv, V3{0.0, 0.0, 0.0});
    for (int t = 0; t < nt; ++t) {
        const int* tr = T + 3 * t;
        V3 fn = cross(sub(at(V, tr[1]), at(V, tr[0])), sub(at(V, tr[2]), at(V, tr[0])));
        const double fl = norm(fn);
        fn = {fn.x / fl, fn.y / fl, fn.z / fl};
        for (int r = 0; r < 3; ++r) {
            const V3 a = at(V, tr[r]), b = at(V, tr[(r + 1) % 3]), c = at(V, tr[(r + 2) % 3]);
            const V3 e1 = sub(b, a), e2 = sub(c, a);
            const double ang = std::atan2(norm(cross(e1, e2)), dot(e1, e2));
            V3& o = out[tr[r]];
            o.x += ang * fn.x;
            o.y += ang * fn.y;
            o.z += ang * fn.z;
        }
    }
    for (V3& o : out) {
        const double l = norm(o);
        o = {-o.x / l, -o.y / l, -o.z / l};
    }
}

// least squares min ||A p - z|| for A (m x 6, row-major) by Householder QR
bool lsq6(int m, std::vector<double>& A, std::vector<double>& z, double p[6]) {
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
        for (int i = k; i < m; ++i) s += A[6 * i + k] * A[6 * i + k];
        const double nk = std::sqrt(s);
        if (!(nk > 0.0)) return false;
        const double alpha = A[6 * k + k] > 0.0 ? -nk : nk;
        // v = x - alpha e1, stored in column k below the diagonal
        A[6 * k + k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < m; ++i) vv += A[6 * i + k] * A[6 * i + k];
        for (int j = k + 1; j < 6; ++j) {
            double f = 0.0;
            for (int i = k; i < m; ++i) f += A[6 * i + k] * A[6 * i + j];
            f = 2.0 * f / vv;
            for (int i = k; i < m; ++i) A[6 * i + j] -= f * A[6 * i + k];
        }
        double f = 0.0;
        for (int i = k; i < m; ++i) f += A[6 * i + k] * z[i];
        f = 2.0 * f / vv;
        for (int i = k; i < m; ++i) z[i] -= f * A[6 * i + k];
        A[6 * k + k] = alpha;  // R's diagonal
    }
    for (int k = 5; k >= 0; --k) {
        double s = z[k];
        for (int j = k + 1; j < 6; ++j) s -= A[6 * k + j] * p[j];
        p[k] = s / A[6 * k + k];
    }
    return true;
}

}  // namespace

extern "C" int ib_surface_lsq_3d(int nv, const double* V, int nt, const int* T, double sigma, double* V_out,
                                 double* fs, double* ds, double* nrm) {
    if (nv < 4 || nt < 4 || !V || !T || !V_out || !fs || !ds || !nrm)
        return ib::fail(IB_EINVAL, "ib_surface_lsq_3d: arguments");
    for (int i = 0; i < 3 * nt; ++i)
        if (T[i] < 0 || T[i] >= nv) return ib::fail(IB_EINVAL, "ib_surface_lsq_3d: triangle index out of range");
    std::vector<V3> n0;
    inward_normals(nv, V, nt, T, n0);
    // one-ring adjacency
    std::vector<std::vector<int>> nb(nv);
    for (int t = 0; t < nt; ++t)
        for (int r = 0; r < 3; ++r) {
            nb[T[3 * t + r]].push_back(T[3 * t + (r + 1) % 3]);
            nb[T[3 * t + r]].push_back(T[3 * t + (r + 2) % 3]);
        }
    for (auto& l : nb) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    std::vector<int> ring;
    std::vector<double> A, z;
    for (int v = 0; v < nv; ++v) {
        ring.assign(nb[v].begin(), nb[v].end());
        for (int w : nb[v]) ring.insert(ring.end(), nb[w].begin(), nb[w].end());
        ring.push_back(v);
        std::sort(ring.begin(), ring.end());
        ring.erase(std::unique(ring.begin(), ring.end()), ring.end());
        const int m = (int)ring.size();
        if (m < 6) return ib::fail(IB_EGEOM, "ib_surface_lsq_3d: a vertex with fewer than 5 neighbours in its two-ring");
        const V3 n = n0[v];
        const double an[3] = {std::fabs(n.x), std::fabs(n.y), std::fabs(n.z)};
        const int axis = an[0] <= an[1] ? (an[0] <= an[2] ? 0 : 2) : (an[1] <= an[2] ? 1 : 2);
        V3 e{axis == 0 ? 1.0 : 0.0, axis == 1 ? 1.0 : 0.0, axis == 2 ? 1.0 : 0.0};
        const double en = dot(e, n);
        V3 t1{e.x - en * n.x, e.y - en * n.y, e.z - en * n.z};
        const double l1 = norm(t1);
        t1 = {t1.x / l1, t1.y / l1, t1.z / l1};
        const V3 t2 = cross(n, t1);
        const V3 xv = at(V, v);
        double L = 0.0;
        for (int w : ring) L += norm(sub(at(V, w), xv));
        L /= (double)(m - 1);
        A.resize(6 * (size_t)m);
        z.resize(m);
        for (int i = 0; i < m; ++i) {
            const V3 p = sub(at(V, ring[i]), xv);
            const double x = dot(p, t1) / L, y = dot(p, t2) / L;
            z[i] = dot(p, n) / L;
            double* row = &A[6 * (size_t)i];
            row[0] = 1.0;
            row[1] = x;
            row[2] = y;
            row[3] = x * x;
            row[4] = x * y;
            row[5] = y * y;
        }
        double q[6];
        if (!lsq6(m, A, z, q)) return ib::fail(IB_EGEOM, "ib_surface_lsq_3d: degenerate neighbourhood");
        const double g = q[0], d = q[1], ee = q[2], a = q[3], b = q[4], c = q[5];
        V_out[3 * v] = xv.x + g * L * n.x;
        V_out[3 * v + 1] = xv.y + g * L * n.y;
        V_out[3 * v + 2] = xv.z + g * L * n.z;
        const double w = 1.0 + d * d + ee * ee, sw = std::sqrt(w);
        nrm[3 * v] = (n.x - d * t1.x - ee * t2.x) / sw;
        nrm[3 * v + 1] = (n.y - d * t1.y - ee * t2.y) / sw;
        nrm[3 * v + 2] = (n.z - d * t1.z - ee * t2.z) / sw;
        fs[v] = sigma * ((1.0 + ee * ee) * 2.0 * a - 2.0 * d * ee * b + (1.0 + d * d) * 2.0 * c) / (L * w * sw);
    }
    for (int v = 0; v < nv; ++v) ds[v] = 0.0;
    for (int t = 0; t < nt; ++t) {
        const int* tr = T + 3 * t;
        const double ar = 0.5 * norm(cross(sub(at(V_out, tr[1]), at(V_out, tr[0])),
                                           sub(at(V_out, tr[2]), at(V_out, tr[0]))));
        for (int r = 0; r < 3; ++r) ds[tr[r]] += ar / 3.0;
    }
    return IB_OK;
}
