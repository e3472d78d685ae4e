// Local least-squares reconstruction of a moving triangulated surface on the
// GPU: the same fit as the host ib_surface_lsq_3d (one thread per vertex), so
// that a 3D flow step keeps its vertices on the device. The connectivity is
// fixed between steps: the two-rings and the vertex-triangle incidence are
// built once on the host (CSR) and uploaded.
//
// Per vertex: inward angle-weighted normal n (incident triangles in ascending
// order); frame t1 (tangent projection of the coordinate axis least aligned
// with n), t2 = n x t1; the two-ring (itself included) scaled by L, its mean
// distance; the quadric z = g + dx + ey + ax^2 + bxy + cy^2 from the 6 x 6
// normal equations (Cholesky); X' = X + g L n, n' = (n - d t1 - e t2)/|.|,
// fs = sigma kappa; ds = a third of the adjacent triangles' areas of X'.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "surface_gpu.h"

namespace ib {

namespace {

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 ld3(const double* V, int i) { return {V[3 * i], V[3 * i + 1], V[3 * i + 2]}; }
__device__ __forceinline__ D3 dsub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 dcross(D3 a, D3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

}  // namespace

// Xa = X + dt U
__global__ void k_surf_advance(const double* __restrict__ X, const double* __restrict__ U, double dt, int n3,
                               double* __restrict__ Xa) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) Xa[i] = X[i] + dt * U[i];
}

// inward unit angle-weighted vertex normals; vt holds 3 t + corner
__global__ void k_surf_normals(const double* __restrict__ V, const int32_t* __restrict__ T,
                               const int32_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt, int nv,
                               double* __restrict__ nrm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    D3 acc{0.0, 0.0, 0.0};
    for (int k = vt_ptr[v]; k < vt_ptr[v + 1]; ++k) {
        const int t = vt[k] / 3, r = vt[k] - 3 * t;
        const int i0 = T[3 * t], i1 = T[3 * t + 1], i2 = T[3 * t + 2];
        const D3 p0 = ld3(V, i0), p1 = ld3(V, i1), p2 = ld3(V, i2);
        D3 fn = dcross(dsub(p1, p0), dsub(p2, p0));
        const double fl = sqrt(ddot(fn, fn));
        fn = {fn.x / fl, fn.y / fl, fn.z / fl};
        const D3 a = r == 0 ? p0 : (r == 1 ? p1 : p2);
        const D3 b = r == 0 ? p1 : (r == 1 ? p2 : p0);
        const D3 c = r == 0 ? p2 : (r == 1 ? p0 : p1);
        const D3 e1 = dsub(b, a), e2 = dsub(c, a);
        const D3 cr = dcross(e1, e2);
        const double ang = atan2(sqrt(ddot(cr, cr)), ddot(e1, e2));
        acc.x += ang * fn.x;
        acc.y += ang * fn.y;
        acc.z += ang * fn.z;
    }
    const double l = sqrt(ddot(acc, acc));
    nrm[3 * v] = -acc.x / l;
    nrm[3 * v + 1] = -acc.y / l;
    nrm[3 * v + 2] = -acc.z / l;
}

// the quadric fit per vertex
__global__ void k_surf_fit(const double* __restrict__ Xa, const double* __restrict__ n0,
                           const int32_t* __restrict__ ring_ptr, const int32_t* __restrict__ ring, int nv,
                           double sigma, double* __restrict__ Xo, double* __restrict__ fs,
                           double* __restrict__ nrm, int* __restrict__ flag) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const D3 n = ld3(n0, v);
    const double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
    const int axis = ax <= ay ? (ax <= az ? 0 : 2) : (ay <= az ? 1 : 2);
    const D3 e{axis == 0 ? 1.0 : 0.0, axis == 1 ? 1.0 : 0.0, axis == 2 ? 1.0 : 0.0};
    const double en = ddot(e, n);
    D3 t1{e.x - en * n.x, e.y - en * n.y, e.z - en * n.z};
    const double l1 = sqrt(ddot(t1, t1));
    t1 = {t1.x / l1, t1.y / l1, t1.z / l1};
    const D3 t2 = dcross(n, t1);
    const D3 xv = ld3(Xa, v);
    const int r0 = ring_ptr[v], r1 = ring_ptr[v + 1], m = r1 - r0;
    double L = 0.0;
    for (int k = r0; k < r1; ++k) {
        const D3 p = dsub(ld3(Xa, ring[k]), xv);
        L += sqrt(ddot(p, p));
    }
    L /= (double)(m - 1);
    const double iL = 1.0 / L;
    // normal equations: M (6 x 6 symmetric, lower triangle) and rhs
    double M[21], q[6];
#pragma unroll
    for (int i = 0; i < 21; ++i) M[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) q[i] = 0.0;
    for (int k = r0; k < r1; ++k) {
        const D3 p = dsub(ld3(Xa, ring[k]), xv);
        const double x = ddot(p, t1) * iL, y = ddot(p, t2) * iL, z = ddot(p, n) * iL;
        const double ph[6] = {1.0, x, y, x * x, x * y, y * y};
        int o = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            q[i] += ph[i] * z;
#pragma unroll
            for (int j = 0; j <= i; ++j) M[o++] += ph[i] * ph[j];
        }
    }
    // Cholesky M = R R^T in place (lower), then two triangular solves
    double Lc[21];
    bool ok = true;
    {
        int o = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double s = M[o];
#pragma unroll
                for (int k = 0; k < j; ++k) s -= Lc[i * (i + 1) / 2 + k] * Lc[j * (j + 1) / 2 + k];
                if (i == j) {
                    ok = ok && s > 0.0;
                    Lc[o] = sqrt(s > 0.0 ? s : 1.0);
                } else {
                    Lc[o] = s / Lc[j * (j + 1) / 2 + j];
                }
                ++o;
            }
        }
    }
    if (!ok) {
        atomicOr(flag, 1);
        return;
    }
    double w[6], c[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = q[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= Lc[i * (i + 1) / 2 + k] * w[k];
        w[i] = s / Lc[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = w[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= Lc[k * (k + 1) / 2 + i] * c[k];
        c[i] = s / Lc[i * (i + 1) / 2 + i];
    }
    const double g = c[0], d = c[1], ee = c[2], a = c[3], b = c[4], cc = c[5];
    Xo[3 * v] = xv.x + g * L * n.x;
    Xo[3 * v + 1] = xv.y + g * L * n.y;
    Xo[3 * v + 2] = xv.z + g * L * n.z;
    const double wq = 1.0 + d * d + ee * ee, sw = sqrt(wq);
    nrm[3 * v] = (n.x - d * t1.x - ee * t2.x) / sw;
    nrm[3 * v + 1] = (n.y - d * t1.y - ee * t2.y) / sw;
    nrm[3 * v + 2] = (n.z - d * t1.z - ee * t2.z) / sw;
    fs[v] = sigma * ((1.0 + ee * ee) * 2.0 * a - 2.0 * d * ee * b + (1.0 + d * d) * 2.0 * cc) / (L * wq * sw);
}

// vertex areas of the moved surface
__global__ void k_surf_areas(const double* __restrict__ V, const int32_t* __restrict__ T,
                             const int32_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt, int nv,
                             double* __restrict__ ds) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double acc = 0.0;
    for (int k = vt_ptr[v]; k < vt_ptr[v + 1]; ++k) {
        const int t = vt[k] / 3;
        const D3 p0 = ld3(V, T[3 * t]), p1 = ld3(V, T[3 * t + 1]), p2 = ld3(V, T[3 * t + 2]);
        const D3 cr = dcross(dsub(p1, p0), dsub(p2, p0));
        acc += 0.5 * sqrt(ddot(cr, cr)) / 3.0;
    }
    ds[v] = acc;
}

void SurfMesh::release() {
    for (int32_t* p : {ring_ptr, ring, vt_ptr, vt, tri})
        if (p) hipFree(p);
    for (double* p : {Xa, n0})
        if (p) hipFree(p);
    if (flag) hipFree(flag);
    *this = SurfMesh();
}

int SurfMesh::prepare(int nv_, int ne_, const int32_t* T) {
    // FNV-1a over the triangles: rebuild when the connectivity changes
    uint64_t hs = 1469598103934665603ull;
    for (long i = 0; i < 3L * ne_; ++i) {
        hs ^= (uint64_t)(uint32_t)T[i];
        hs *= 1099511628211ull;
    }
    if (nv == nv_ && ne == ne_ && hash == hs) return IB_OK;
    release();
    for (long i = 0; i < 3L * ne_; ++i)
        IB_CHECK(T[i] >= 0 && T[i] < nv_, IB_EINVAL, "flow_step: triangle index out of range");
    std::vector<std::vector<int32_t>> nb(nv_);
    std::vector<int32_t> vtp(nv_ + 1, 0), vti(3L * ne_);
    for (int t = 0; t < ne_; ++t)
        for (int r = 0; r < 3; ++r) {
            nb[T[3 * t + r]].push_back(T[3 * t + (r + 1) % 3]);
            nb[T[3 * t + r]].push_back(T[3 * t + (r + 2) % 3]);
            ++vtp[T[3 * t + r] + 1];
        }
    for (int v = 0; v < nv_; ++v) vtp[v + 1] += vtp[v];
    {
        std::vector<int32_t> fill(vtp.begin(), vtp.end() - 1);
        for (int t = 0; t < ne_; ++t)
            for (int r = 0; r < 3; ++r) vti[fill[T[3 * t + r]]++] = 3 * t + r;
    }
    for (auto& l : nb) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    std::vector<int32_t> rp(nv_ + 1, 0), ri;
    std::vector<int32_t> tmp;
    for (int v = 0; v < nv_; ++v) {
        tmp.assign(nb[v].begin(), nb[v].end());
        for (int w : nb[v]) tmp.insert(tmp.end(), nb[w].begin(), nb[w].end());
        tmp.push_back(v);
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        IB_CHECK(tmp.size() >= 6, IB_EGEOM, "flow_step: a vertex with fewer than 5 neighbours in its two-ring");
        ri.insert(ri.end(), tmp.begin(), tmp.end());
        rp[v + 1] = (int32_t)ri.size();
    }
    bool okm = true;
    auto up = [&](int32_t** d, const std::vector<int32_t>& h) {
        if (okm && hipMalloc((void**)d, sizeof(int32_t) * h.size()) != hipSuccess) okm = false;
        if (okm && hipMemcpy(*d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice) != hipSuccess)
            okm = false;
    };
    up(&ring_ptr, rp);
    up(&ring, ri);
    up(&vt_ptr, vtp);
    up(&vt, vti);
    up(&tri, std::vector<int32_t>(T, T + 3L * ne_));
    okm = okm && hipMalloc((void**)&Xa, sizeof(double) * 3 * nv_) == hipSuccess;
    okm = okm && hipMalloc((void**)&n0, sizeof(double) * 3 * nv_) == hipSuccess;
    okm = okm && hipMalloc((void**)&flag, sizeof(int)) == hipSuccess;
    if (!okm) {
        release();
        return fail(IB_ENOMEM, "flow_step: out of memory for the surface connectivity");
    }
    nv = nv_;
    ne = ne_;
    hash = hs;
    return IB_OK;
}

int SurfMesh::reconstruct(const double* X, const double* U, double dt, double sigma, double* Xo, double* fs,
                          double* ds, double* nrm, hipStream_t st) {
    const int32_t* T = tri;
    const dim3 blk(kBlock);
    hipLaunchKernelGGL(k_surf_advance, dim3(grid_for(3L * nv)), blk, 0, st, X, U, dt, 3 * nv, Xa);
    hipLaunchKernelGGL(k_surf_normals, dim3(grid_for(nv)), blk, 0, st, Xa, T, vt_ptr, vt, nv, n0);
    IB_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_surf_fit, dim3(grid_for(nv)), blk, 0, st, Xa, n0, ring_ptr, ring, nv, sigma, Xo, fs,
                       nrm, flag);
    hipLaunchKernelGGL(k_surf_areas, dim3(grid_for(nv)), blk, 0, st, Xo, T, vt_ptr, vt, nv, ds);
    IB_HIP(hipGetLastError());
    int hf = 0;
    IB_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    IB_CHECK(hf == 0, IB_EGEOM, "flow_step: a degenerate vertex neighbourhood in the surface fit");
    return IB_OK;
}

}  // namespace ib
