// Curvature force on a closed triangle mesh (host FP64). The paper
// reconstructs curves only and leaves closed surfaces in 3D to future work
// (Sections 4 and 6); this is the library's extension for static meshes.
//
// The force on vertex v is F_v = -sigma d(total area)/dX_v. For a triangle
// (a, b, c), counter-clockwise about its unit normal n, the area gradients
// are (1/2) n x (c - b), (1/2) n x (a - c), (1/2) n x (b - a) for a, b, c.
// The vertex area is one third of the adjacent triangle areas, the normal
// is the angle-weighted mean of the adjacent triangle normals, pointing into
// the enclosed volume. fs_v = (F_v . n_v) / A_v (sigma times the sum of the
// principal curvatures), ds_v = A_v.
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ibproj.h"

namespace ib {
int fail(int code, const std::string& msg);
}

namespace {
inline void cross(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
}  // namespace

extern "C" int ib_surface_geometry_3d(int nv, const double* X, int nt, const int32_t* tris,
                                      double sigma, double* fs_out, double* ds_out,
                                      double* nrm_out) {
    if (nv < 4 || nt < 4 || !X || !tris || !fs_out || !ds_out || !nrm_out)
        return ib::fail(IB_EINVAL, "ib_surface_geometry_3d: bad argument");
    std::vector<double> F(3 * (size_t)nv, 0.0), A(nv, 0.0), N(3 * (size_t)nv, 0.0);
    for (int t = 0; t < nt; ++t) {
        int v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
        for (int r = 0; r < 3; ++r)
            if (v[r] < 0 || v[r] >= nv)
                return ib::fail(IB_EINVAL, "ib_surface_geometry_3d: vertex index out of range");
        const double* p[3] = {X + 3 * v[0], X + 3 * v[1], X + 3 * v[2]};
        double e1[3], e2[3], n[3];
        for (int e = 0; e < 3; ++e) {
            e1[e] = p[1][e] - p[0][e];
            e2[e] = p[2][e] - p[0][e];
        }
        cross(e1, e2, n);
        double len = std::sqrt(dot(n, n));
        if (!(len > 0.0)) return ib::fail(IB_EGEOM, "ib_surface_geometry_3d: degenerate triangle");
        double un[3] = {n[0] / len, n[1] / len, n[2] / len};
        double area = 0.5 * len;
        for (int r = 0; r < 3; ++r) {
            const double* pn = p[(r + 1) % 3];
            const double* pp = p[(r + 2) % 3];
            // area gradient at vertex r: (1/2) n x (p_{r+2} - p_{r+1})
            double opp[3] = {pp[0] - pn[0], pp[1] - pn[1], pp[2] - pn[2]};
            double g[3];
            cross(un, opp, g);
            for (int e = 0; e < 3; ++e) F[3 * v[r] + e] -= sigma * 0.5 * g[e];
            A[v[r]] += area / 3.0;
            // angle at vertex r
            double a1[3] = {pn[0] - p[r][0], pn[1] - p[r][1], pn[2] - p[r][2]};
            double a2[3] = {pp[0] - p[r][0], pp[1] - p[r][1], pp[2] - p[r][2]};
            double cr[3];
            cross(a1, a2, cr);
            double ang = std::atan2(std::sqrt(dot(cr, cr)), dot(a1, a2));
            for (int e = 0; e < 3; ++e) N[3 * v[r] + e] -= ang * un[e];
        }
    }
    for (int v = 0; v < nv; ++v) {
        double* n = &N[3 * (size_t)v];
        double len = std::sqrt(dot(n, n));
        if (!(len > 0.0) || !(A[v] > 0.0))
            return ib::fail(IB_EGEOM, "ib_surface_geometry_3d: isolated vertex");
        for (int e = 0; e < 3; ++e) nrm_out[3 * v + e] = n[e] / len;
        fs_out[v] = dot(&F[3 * (size_t)v], &nrm_out[3 * v]) / A[v];
        ds_out[v] = A[v];
    }
    return IB_OK;
}
