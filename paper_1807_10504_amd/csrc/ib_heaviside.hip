// Discrete Heaviside from offset polygons / polyhedra (Section 3.2).
//
// H^(x) = sum_m dH_m 1[x in P_m], P_m = interface offset toward the drop by
// c_m in {-1.5h, -0.5h, 0.5h, 1.5h}; dH_m are the increments of the region
// values H(q) = 1/2 + q/4 + sin(pi q/2)/(2 pi) at q = -2..2 (eqs new_hea,
// new_hea2). The cell value is the overlap-weighted sum (caption of the
// three-polygon figure): H_c = sum_m dH_m |cell ∩ P_m| / h^dim.
//
// The overlap is computed from the boundary pieces, column by column: for a
// closed outward-oriented boundary, |P ∩ column ∩ {z > c}| is the sum over
// boundary pieces of (signed projected size) x integral of max(z - c, 0)
// (z = y in 2D). One thread owns one (offset m, element) pair, clips the
// element to every column it projects onto, and adds
//   * exact partial cell measures for the cells its height range crosses, and
//   * the full-height measure of every cell below, as one entry of a
//     per-column suffix sum.
// Both are accumulated as 64-bit fixed-point integers (2^-56 of a cell) with
// integer atomics, so the result does not depend on the order of the adds;
// a final pass per column converts to double and zeroes the accumulators.
#include "common.h"

namespace ib {

// region value increments, computed from the closed form on the host
struct Jumps {
    double dh[4];
    double c[4];  // offsets in units of h (positive toward the drop)
};

static Jumps make_jumps() {
    Jumps j;
    const double q[5] = {-2.0, -1.0, 0.0, 1.0, 2.0};
    double v[5];
    for (int r = 0; r < 5; ++r) {
        if (q[r] <= -2.0) v[r] = 0.0;
        else if (q[r] >= 2.0) v[r] = 1.0;
        else v[r] = 0.5 + 0.25 * q[r] + sin(0.5 * M_PI * q[r]) / (2.0 * M_PI);
    }
    for (int m = 0; m < 4; ++m) j.dh[m] = v[m + 1] - v[m];
    j.c[0] = -1.5;
    j.c[1] = -0.5;
    j.c[2] = 0.5;
    j.c[3] = 1.5;
    return j;
}

__device__ __forceinline__ long long to_fix(double v) {
    return (long long)rint(v * kFixScale);
}

// ---------------------------------------------------------------------------
// offset vertices; also checks that they keep 4h away from the box faces
__global__ void k_offsets_2d(const double* __restrict__ X, int n, Jumps J, Dims d,
                             double* __restrict__ off, int* __restrict__ flags) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * n) return;
    int m = t / n, k = t - m * n;
    int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
    double x = X[2 * k], y = X[2 * k + 1];
    double ax = x - X[2 * km], ay = y - X[2 * km + 1];
    double bx = X[2 * kp] - x, by = X[2 * kp + 1] - y;
    double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
    // unit left normals of the two adjacent segments
    double nax = -ay / la, nay = ax / la, nbx = -by / lb, nby = bx / lb;
    double den = 1.0 + (nax * nbx + nay * nby);
    double c = J.c[m] * d.h;
    double ox = x + c * ((nax + nbx) / den), oy = y + c * ((nay + nby) / den);
    off[2 * t] = ox;
    off[2 * t + 1] = oy;
    double lo = 4.0 * d.h;
    if (!(ox > lo && ox < d.nx * d.h - lo && oy > lo && oy < d.ny * d.h - lo)) atomicOr(flags, 1);
}

__global__ void k_offsets_3d(const double* __restrict__ X, const double* __restrict__ nrm, int n,
                             Jumps J, Dims d, double* __restrict__ off, int* __restrict__ flags) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * n) return;
    int m = t / n, v = t - m * n;
    double c = J.c[m] * d.h;
    double lo = 4.0 * d.h;
    double L[3] = {d.nx * d.h, d.ny * d.h, d.nz * d.h};
    bool ok = true;
    for (int e = 0; e < 3; ++e) {
        double p = X[3 * v + e] + c * nrm[3 * v + e];
        off[3 * (long)t + e] = p;
        ok = ok && (p > lo && p < L[e] - lo);
    }
    if (!ok) atomicOr(flags, 1);
}

// ---------------------------------------------------------------------------
// 2D: one thread per (m, segment)
// G(c) = -(integral over the piece of max(y - c, 0) dx), signed by dx
__device__ __forceinline__ double g_seg(double xa, double ya, double xb, double yb, double c) {
    double dx = xb - xa;
    if (ya >= c && yb >= c) return -dx * (0.5 * (ya + yb) - c);
    if (ya >= c) {  // yb < c
        double t = (ya - c) / (ya - yb);
        return -(t * dx) * (0.5 * (ya - c));
    }
    if (yb >= c) {  // ya < c
        double t = (yb - c) / (yb - ya);
        return -(t * dx) * (0.5 * (yb - c));
    }
    return 0.0;
}

__global__ void k_heaviside_2d(const double* __restrict__ off, int n, Jumps J, Dims d,
                               long long* __restrict__ A, long long* __restrict__ S) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * n) return;
    int m = t / n, k = t - m * n;
    int kp = k + 1 == n ? 0 : k + 1;
    const double* P = off + 2 * (long)m * n;
    double xa = P[2 * k], ya = P[2 * k + 1], xb = P[2 * kp], yb = P[2 * kp + 1];
    if (xa == xb) return;
    double h = d.h;
    double scale = J.dh[m] / (h * h);
    int i0 = (int)floor(fmin(xa, xb) / h), i1 = (int)floor(fmax(xa, xb) / h);
    for (int i = i0; i <= i1; ++i) {
        if (i < 0 || i >= d.nx) continue;
        double x0 = i * h, x1 = (i + 1) * h;
        double t0 = (x0 - xa) / (xb - xa), t1 = (x1 - xa) / (xb - xa);
        double ta = fmax(0.0, fmin(t0, t1)), tb = fmin(1.0, fmax(t0, t1));
        if (!(tb > ta)) continue;
        double pxa = xa + ta * (xb - xa), pya = ya + ta * (yb - ya);
        double pxb = xa + tb * (xb - xa), pyb = ya + tb * (yb - ya);
        if (pxa == pxb) continue;
        int j0 = (int)floor(fmin(pya, pyb) / h), j1 = (int)floor(fmax(pya, pyb) / h);
        for (int j = j0; j <= j1; ++j) {
            if (j < 0 || j >= d.ny) continue;
            double v = g_seg(pxa, pya, pxb, pyb, j * h) - g_seg(pxa, pya, pxb, pyb, (j + 1) * h);
            atomicAdd((unsigned long long*)&A[(long)j * d.nx + i], (unsigned long long)to_fix(v * scale));
        }
        if (j0 >= 1 && j0 <= d.ny) {
            double full = -(pxb - pxa) * h;
            atomicAdd((unsigned long long*)&S[(long)(j0 - 1) * d.nx + i],
                      (unsigned long long)to_fix(full * scale));
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: one thread per (m, triangle)
// vertices in vector registers: a variable index into a vector is a register
// select, where one into an array would put the polygons in scratch memory.
// Eight vertices suffice: each cut of a convex polygon by a half-plane adds at
// most one vertex, and a piece is the triangle cut five times (four column
// walls, then the plane z = c).
typedef double Coord8 __attribute__((ext_vector_type(8)));
struct Poly {
    Coord8 x, y, z;
    int n;
};

template <int AXIS>
__device__ __forceinline__ double coord(const Poly& p, int r) {
    if constexpr (AXIS == 0)
        return p.x[r];
    else if constexpr (AXIS == 1)
        return p.y[r];
    else
        return p.z[r];
}

// keep the part with coordinate AXIS >= v (GE) or <= v (!GE)
template <int AXIS, bool GE>
__device__ __forceinline__ void clip(const Poly& in, Poly& out, double v) {
    out.n = 0;
    for (int r = 0; r < in.n; ++r) {
        int q = r + 1 == in.n ? 0 : r + 1;
        double pr = coord<AXIS>(in, r);
        double pq = coord<AXIS>(in, q);
        double sr = GE ? pr - v : v - pr;
        double sq = GE ? pq - v : v - pq;
        if (sr >= 0.0 && out.n < 8) {
            out.x[out.n] = in.x[r];
            out.y[out.n] = in.y[r];
            out.z[out.n] = in.z[r];
            ++out.n;
        }
        if ((sr >= 0.0) != (sq >= 0.0) && out.n < 8) {
            double tt = sr / (sr - sq);
            out.x[out.n] = in.x[r] + tt * (in.x[q] - in.x[r]);
            out.y[out.n] = in.y[r] + tt * (in.y[q] - in.y[r]);
            out.z[out.n] = in.z[r] + tt * (in.z[q] - in.z[r]);
            ++out.n;
        }
    }
}

// signed projected area and integral of max(z - c, 0) over the projection
__device__ __forceinline__ double g_poly(const Poly& p, double c, Poly& tmp) {
    clip<2, true>(p, tmp, c);
    if (tmp.n < 3) return 0.0;
    double s = 0.0;
    for (int r = 1; r + 1 < tmp.n; ++r) {
        double ax = tmp.x[r] - tmp.x[0], ay = tmp.y[r] - tmp.y[0];
        double bx = tmp.x[r + 1] - tmp.x[0], by = tmp.y[r + 1] - tmp.y[0];
        double area = 0.5 * (ax * by - ay * bx);
        s += area * ((tmp.z[0] + tmp.z[r] + tmp.z[r + 1]) * (1.0 / 3.0) - c);
    }
    return s;
}

__global__ __launch_bounds__(256) void k_heaviside_3d(const double* __restrict__ off, int nv,
                                                      const int32_t* __restrict__ T, int nt, Jumps J, Dims d,
                                                      long long* __restrict__ A, long long* __restrict__ S,
                                                      int* __restrict__ flags) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * nt) return;
    int m = t / nt, e = t - m * nt;
    const double* P = off + 3 * (long)m * nv;
    Poly tri;
    tri.n = 3;
    for (int r = 0; r < 3; ++r) {
        int v = T[3 * e + r];
        if (v < 0 || v >= nv) {
            atomicOr(flags + 2, 1);
            return;
        }
        tri.x[r] = P[3 * v];
        tri.y[r] = P[3 * v + 1];
        tri.z[r] = P[3 * v + 2];
    }
    double h = d.h;
    double scale = J.dh[m] / (h * h * h);
    double xmn = fmin(tri.x[0], fmin(tri.x[1], tri.x[2])), xmx = fmax(tri.x[0], fmax(tri.x[1], tri.x[2]));
    double ymn = fmin(tri.y[0], fmin(tri.y[1], tri.y[2])), ymx = fmax(tri.y[0], fmax(tri.y[1], tri.y[2]));
    int i0 = (int)floor(xmn / h), i1 = (int)floor(xmx / h);
    int j0 = (int)floor(ymn / h), j1 = (int)floor(ymx / h);
    Poly a, b;
    for (int j = j0; j <= j1; ++j) {
        if (j < 0 || j >= d.ny) continue;
        for (int i = i0; i <= i1; ++i) {
            if (i < 0 || i >= d.nx) continue;
            clip<0, true>(tri, a, i * h);
            if (a.n < 3) continue;
            clip<0, false>(a, b, (i + 1) * h);
            if (b.n < 3) continue;
            clip<1, true>(b, a, j * h);
            if (a.n < 3) continue;
            clip<1, false>(a, b, (j + 1) * h);
            if (b.n < 3) continue;
            // b = the piece over column (i, j)
            double area = 0.0, zmn = b.z[0], zmx = b.z[0];
            for (int r = 1; r + 1 < b.n; ++r) {
                double ax = b.x[r] - b.x[0], ay = b.y[r] - b.y[0];
                double bx = b.x[r + 1] - b.x[0], by = b.y[r + 1] - b.y[0];
                area += 0.5 * (ax * by - ay * bx);
            }
            for (int r = 1; r < b.n; ++r) {
                zmn = fmin(zmn, b.z[r]);
                zmx = fmax(zmx, b.z[r]);
            }
            if (area == 0.0) continue;
            int k0 = (int)floor(zmn / h), k1 = (int)floor(zmx / h);
            long col = (long)j * d.nx + i;
            long plane = (long)d.nx * d.ny;
            double gprev = g_poly(b, k0 * h, a);
            for (int k = k0; k <= k1; ++k) {
                double gnext = g_poly(b, (k + 1) * h, a);
                if (k >= 0 && k < d.nz)
                    atomicAdd((unsigned long long*)&A[(long)k * plane + col],
                              (unsigned long long)to_fix((gprev - gnext) * scale));
                gprev = gnext;
            }
            if (k0 >= 1 && k0 <= d.nz)
                atomicAdd((unsigned long long*)&S[(long)(k0 - 1) * plane + col],
                          (unsigned long long)to_fix(area * h * scale));
        }
    }
}

// ---------------------------------------------------------------------------
// per column: suffix sum from the top, convert, and zero the accumulators
__global__ void k_heaviside_finish(Dims d, long long* __restrict__ A, long long* __restrict__ S,
                                   double* __restrict__ H) {
    long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long plane, ncol;
    int len;
    if (d.dim == 2) {
        ncol = d.nx;
        plane = d.nx;
        len = d.ny;
    } else {
        ncol = (long)d.nx * d.ny;
        plane = ncol;
        len = d.nz;
    }
    if (col >= ncol) return;
    long long run = 0;
    for (int k = len - 1; k >= 0; --k) {
        long idx = (long)k * plane + col;
        run += S[idx];
        long long v = A[idx] + run;
        H[idx] = (double)v * kFixInv;
        A[idx] = 0;
        S[idx] = 0;
    }
}

// the same with eight segments per column in parallel: a workgroup
// holds 64 columns x 8 segments; each lane sums S over its segment, the
// segment sums above it give the suffix it starts from (integer sums, so the
// result is bit for bit the one-lane-per-column pass), then it runs down its
// segment. Needs a column length divisible by 8 and a column count by 64.
constexpr int kFinCols = 64, kFinSegs = 8;
__global__ __launch_bounds__(kFinCols* kFinSegs) void k_heaviside_finish_seg(Dims d, long long* __restrict__ A,
                                                                            long long* __restrict__ S,
                                                                            double* __restrict__ H) {
    __shared__ long long segsum[kFinSegs][kFinCols];
    const long plane = d.dim == 2 ? (long)d.nx : (long)d.nx * d.ny;
    const int sl = (d.dim == 2 ? d.ny : d.nz) / kFinSegs;
    const long col = (long)blockIdx.x * kFinCols + threadIdx.x;
    const int sg = threadIdx.y;
    const int k0 = sg * sl;
    long long acc = 0;
    for (int k = k0; k < k0 + sl; ++k) acc += S[(long)k * plane + col];
    segsum[sg][threadIdx.x] = acc;
    __syncthreads();
    long long run = 0;
    for (int q = kFinSegs - 1; q > sg; --q) run += segsum[q][threadIdx.x];
    for (int k = k0 + sl - 1; k >= k0; --k) {
        const long idx = (long)k * plane + col;
        run += S[idx];
        long long v = A[idx] + run;
        H[idx] = (double)v * kFixInv;
        A[idx] = 0;
        S[idx] = 0;
    }
}

int launch_heaviside(Ctx* c, const ib_surface* s, double* H, hipStream_t st) {
    Jumps J = make_jumps();
    int n = s->n_markers;
    IB_CHECK(n >= 3, IB_EINVAL, "ib_spread: fewer than 3 markers");
    if (c->d.dim == 2) {
        hipLaunchKernelGGL(k_offsets_2d, dim3(grid_for(4L * n)), dim3(kBlock), 0, st, s->X, n, J,
                           c->d, c->offv, c->flags);
        hipLaunchKernelGGL(k_heaviside_2d, dim3(grid_for(4L * n)), dim3(kBlock), 0, st, c->offv,
                           n, J, c->d, c->accA, c->accS);
        if (c->d.ny % kFinSegs == 0 && c->d.nx % kFinCols == 0)
            hipLaunchKernelGGL(k_heaviside_finish_seg, dim3((unsigned)(c->d.nx / kFinCols)),
                               dim3(kFinCols, kFinSegs), 0, st, c->d, c->accA, c->accS, H);
        else
            hipLaunchKernelGGL(k_heaviside_finish, dim3(grid_for(c->d.nx)), dim3(kBlock), 0, st, c->d,
                               c->accA, c->accS, H);
    } else {
        IB_CHECK(s->nrm && s->elems && s->n_elems > 0, IB_EINVAL,
                 "ib_spread: 3D surfaces need elems and nrm");
        hipLaunchKernelGGL(k_offsets_3d, dim3(grid_for(4L * n)), dim3(kBlock), 0, st, s->X,
                           s->nrm, n, J, c->d, c->offv, c->flags);
        int nt = s->n_elems;
        hipLaunchKernelGGL(k_heaviside_3d, dim3(grid_for(4L * nt)), dim3(kBlock), 0, st, c->offv,
                           n, s->elems, nt, J, c->d, c->accA, c->accS, c->flags);
        const long ncol = (long)c->d.nx * c->d.ny;
        if (c->d.nz % kFinSegs == 0 && ncol % kFinCols == 0)
            hipLaunchKernelGGL(k_heaviside_finish_seg, dim3((unsigned)(ncol / kFinCols)), dim3(kFinCols, kFinSegs),
                               0, st, c->d, c->accA, c->accS, H);
        else
            hipLaunchKernelGGL(k_heaviside_finish, dim3(grid_for(ncol)), dim3(kBlock), 0, st, c->d, c->accA,
                               c->accS, H);
    }
    IB_HIP(hipGetLastError());
    return IB_OK;
}

}  // namespace ib
