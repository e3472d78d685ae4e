// Irrotational face force, coefficients, right side, velocity update,
// diagnostics and deterministic reductions.
//
// Irrotational delta vector (eq delta_hea_xy): on the face between cells
// c - e_d and c, F_d = f (H_c - H_{c-e_d}) / h, where f is sigma*kappa at the
// foot point on the nearest interface element (linear along a segment,
// barycentric on a triangle; ties to the lower element index). The nearest
// element is found by a scatter from every element to the faces within 3h
// of it (every face with a nonzero Heaviside difference lies within 2.9h of
// the interface): each candidate writes atomicMin of a 64-bit key made of
// the quantised squared distance (2^-36 h^2 steps) and the element index, so
// the winner does not depend on execution order. The face pass reads the
// winner, evaluates f in FP64 and resets the key.
//
// Away from the interface H is 0 or 1 up to the rounding of the overlap sums
// (~1e-16); a face is an interface face when |dH| > kDhEps = 1e-13, and
// carries F = 0 otherwise.
#include "common.h"

namespace ib {

constexpr int kElemBits = 23;
constexpr unsigned long long kElemMask = (1ull << kElemBits) - 1;
constexpr double kDistScale = 68719476736.0;  // 2^36
constexpr double kReach = 3.0;                // search radius in h
constexpr double kDhEps = 1e-13;

__device__ __forceinline__ long cell_index(const Dims& d, int i, int j, int k) {
    return ((long)k * d.ny + j) * d.nx + i;
}

// closest point on segment a-b to p: returns squared distance, t in [0, 1]
__device__ __forceinline__ double seg_closest(double px, double py, double ax, double ay, double bx,
                                              double by, double* t_out) {
    double ex = bx - ax, ey = by - ay;
    double t = ((px - ax) * ex + (py - ay) * ey) / (ex * ex + ey * ey);
    t = fmin(1.0, fmax(0.0, t));
    double qx = ax + t * ex - px, qy = ay + t * ey - py;
    *t_out = t;
    return qx * qx + qy * qy;
}

// closest point on triangle abc to p by Voronoi regions of the vertices,
// edges and face; returns squared distance and barycentric weights of a, b, c
__device__ double tri_closest(const double* p, const double* a, const double* b, const double* c,
                              double* w) {
    double ab[3], ac[3], ap[3];
    for (int e = 0; e < 3; ++e) {
        ab[e] = b[e] - a[e];
        ac[e] = c[e] - a[e];
        ap[e] = p[e] - a[e];
    }
    double d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
    double d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
    double u, v, ww;
    if (d1 <= 0.0 && d2 <= 0.0) {
        u = 1.0; v = 0.0; ww = 0.0;
    } else {
        double bp[3];
        for (int e = 0; e < 3; ++e) bp[e] = p[e] - b[e];
        double d3 = ab[0] * bp[0] + ab[1] * bp[1] + ab[2] * bp[2];
        double d4 = ac[0] * bp[0] + ac[1] * bp[1] + ac[2] * bp[2];
        double cp[3];
        for (int e = 0; e < 3; ++e) cp[e] = p[e] - c[e];
        double d5 = ab[0] * cp[0] + ab[1] * cp[1] + ab[2] * cp[2];
        double d6 = ac[0] * cp[0] + ac[1] * cp[1] + ac[2] * cp[2];
        double vc = d1 * d4 - d3 * d2;
        double vb = d5 * d2 - d1 * d6;
        double va = d3 * d6 - d5 * d4;
        if (d3 >= 0.0 && d4 <= d3) {
            u = 0.0; v = 1.0; ww = 0.0;
        } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
            double s = d1 / (d1 - d3);
            u = 1.0 - s; v = s; ww = 0.0;
        } else if (d6 >= 0.0 && d5 <= d6) {
            u = 0.0; v = 0.0; ww = 1.0;
        } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
            double s = d2 / (d2 - d6);
            u = 1.0 - s; v = 0.0; ww = s;
        } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
            double s = (d4 - d3) / ((d4 - d3) + (d5 - d6));
            u = 0.0; v = 1.0 - s; ww = s;
        } else {
            double den = 1.0 / (va + vb + vc);
            v = vb * den;
            ww = vc * den;
            u = 1.0 - v - ww;
        }
    }
    w[0] = u;
    w[1] = v;
    w[2] = ww;
    double q2 = 0.0;
    for (int e = 0; e < 3; ++e) {
        double q = u * a[e] + v * b[e] + ww * c[e] - p[e];
        q2 += q * q;
    }
    return q2;
}

__device__ __forceinline__ unsigned long long make_key(double d2, double inv_h2, int elem) {
    double q = d2 * inv_h2 * kDistScale;
    return ((unsigned long long)q << kElemBits) | (unsigned long long)elem;
}

// 2D scatter: one thread per (segment, orientation)
__global__ void k_nearest_2d(const double* __restrict__ X, int n, const double* __restrict__ H,
                             Dims d, unsigned long long* __restrict__ best) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * n) return;
    int comp = t / n, k = t - comp * n;
    int kp = k + 1 == n ? 0 : k + 1;
    double ax = X[2 * k], ay = X[2 * k + 1], bx = X[2 * kp], by = X[2 * kp + 1];
    double h = d.h, R = kReach * h, R2 = R * R, inv_h2 = 1.0 / (h * h);
    double offx = comp == 0 ? 0.0 : 0.5, offy = comp == 1 ? 0.0 : 0.5;
    int i0 = (int)ceil((fmin(ax, bx) - R) / h - offx), i1 = (int)floor((fmax(ax, bx) + R) / h - offx);
    int j0 = (int)ceil((fmin(ay, by) - R) / h - offy), j1 = (int)floor((fmax(ay, by) + R) / h - offy);
    i0 = max(i0, 0); j0 = max(j0, 0);
    i1 = min(i1, d.nx - 1); j1 = min(j1, d.ny - 1);
    unsigned long long* B = best + (long)comp * d.cells();
    for (int j = j0; j <= j1; ++j) {
        for (int i = i0; i <= i1; ++i) {
            long c = (long)j * d.nx + i;
            long cm = comp == 0 ? (long)j * d.nx + (i == 0 ? d.nx - 1 : i - 1)
                                : (long)(j == 0 ? d.ny - 1 : j - 1) * d.nx + i;
            if (fabs(H[c] - H[cm]) <= kDhEps) continue;
            double tt;
            double d2 = seg_closest((i + offx) * h, (j + offy) * h, ax, ay, bx, by, &tt);
            if (d2 >= R2) continue;
            atomicMin(&B[c], make_key(d2, inv_h2, k));
        }
    }
}

// 3D scatter: one wavefront per (triangle, orientation); its 64 lanes split
// the faces of the triangle's reach box (about 8 each), so the loads of H
// that decide each face are independent across lanes instead of a chain of
// several hundred dependent loads in one thread
constexpr int kNearLanes = 64;

__global__ __launch_bounds__(256) void k_nearest_3d(const double* __restrict__ X, int nv,
                                                    const int32_t* __restrict__ T, int nt,
                                                    const double* __restrict__ H, Dims d,
                                                    unsigned long long* __restrict__ best) {
    const long task = ((long)blockIdx.x * blockDim.x + threadIdx.x) / kNearLanes;
    const int lane = threadIdx.x % kNearLanes;
    if (task >= 3L * nt) return;
    int comp = (int)(task / nt), e = (int)(task - (long)comp * nt);
    for (int r = 0; r < 3; ++r) {
        int v = T[3 * e + r];
        if (v < 0 || v >= nv) return;  // reported by the Heaviside pass
    }
    double a[3], b[3], c[3];
    for (int r = 0; r < 3; ++r) {
        a[r] = X[3 * T[3 * e] + r];
        b[r] = X[3 * T[3 * e + 1] + r];
        c[r] = X[3 * T[3 * e + 2] + r];
    }
    double h = d.h, R = kReach * h, R2 = R * R, inv_h2 = 1.0 / (h * h);
    int lo[3], hi[3];
    int nn[3] = {d.nx, d.ny, d.nz};
    for (int r = 0; r < 3; ++r) {
        double off = r == comp ? 0.0 : 0.5;
        double mn = fmin(a[r], fmin(b[r], c[r])), mx = fmax(a[r], fmax(b[r], c[r]));
        lo[r] = max((int)ceil((mn - R) / h - off), 0);
        hi[r] = min((int)floor((mx + R) / h - off), nn[r] - 1);
    }
    unsigned long long* B = best + (long)comp * d.cells();
    long stride = comp == 0 ? 1 : (comp == 1 ? (long)d.nx : (long)d.nx * d.ny);
    // faces farther from the centroid than R plus the circumradius cannot be
    // within R of the triangle: skipped before any load (the bound is widened
    // by a relative 1e-9 so that rounding never rejects a face within reach)
    double g[3], rad2 = 0.0;
    for (int r = 0; r < 3; ++r) g[r] = (a[r] + b[r] + c[r]) * (1.0 / 3.0);
    for (const double* v : {a, b, c}) {
        double s2 = 0.0;
        for (int r = 0; r < 3; ++r) s2 += (v[r] - g[r]) * (v[r] - g[r]);
        rad2 = fmax(rad2, s2);
    }
    const double reach = R + sqrt(rad2);
    const double bound = reach * reach * (1.0 + 1e-9);
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    if (ex <= 0 || ey <= 0 || ez <= 0) return;
    const int nbox = ex * ey * ez;
    for (int f = lane; f < nbox; f += kNearLanes) {
        const int i = lo[0] + f % ex;
        const int rr = f / ex;
        const int j = lo[1] + rr % ey;
        const int k = lo[2] + rr / ey;
        double p[3] = {(i + (comp == 0 ? 0.0 : 0.5)) * h, (j + (comp == 1 ? 0.0 : 0.5)) * h,
                       (k + (comp == 2 ? 0.0 : 0.5)) * h};
        const double gx = p[0] - g[0], gy = p[1] - g[1], gz = p[2] - g[2];
        if (gx * gx + gy * gy + gz * gz > bound) continue;
        long cc = cell_index(d, i, j, k);
        int ic = comp == 0 ? i : (comp == 1 ? j : k);
        long cm = ic == 0 ? cc + (long)(nn[comp] - 1) * stride : cc - stride;
        if (fabs(H[cc] - H[cm]) <= kDhEps) continue;
        double w[3];
        double d2 = tri_closest(p, a, b, c, w);
        if (d2 >= R2) continue;
        atomicMin(&B[cc], make_key(d2, inv_h2, e));
    }
}

// face pass: F = f dH / h, reset keys
template <int DIM>
__global__ void k_irrot_force(const double* __restrict__ X, const int32_t* __restrict__ T,
                              const double* __restrict__ fs, const double* __restrict__ H, Dims d,
                              int comp, int n, unsigned long long* __restrict__ best,
                              double* __restrict__ F, int* __restrict__ flags) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    int i, j, k;
    cell_ijk(c, d.nx, d.ny, i, j, k);
    int ic = comp == 0 ? i : (comp == 1 ? j : k);
    int nn = comp == 0 ? d.nx : (comp == 1 ? d.ny : d.nz);
    long stride = comp == 0 ? 1 : (comp == 1 ? (long)d.nx : (long)d.nx * d.ny);
    long cm = ic == 0 ? c + (long)(nn - 1) * stride : c - stride;
    double dH = H[c] - H[cm];
    double out = 0.0;
    if (fabs(dH) > kDhEps) {
        unsigned long long* B = best + (long)comp * d.cells();
        unsigned long long key = B[c];
        if (key == ~0ull) {
            atomicOr(flags + 1, 1);
        } else {
            int e = (int)(key & kElemMask);
            double h = d.h;
            double f;
            if (DIM == 2) {
                int kp = e + 1 == n ? 0 : e + 1;
                double tt;
                seg_closest((i + (comp == 0 ? 0.0 : 0.5)) * h, (j + (comp == 1 ? 0.0 : 0.5)) * h,
                            X[2 * e], X[2 * e + 1], X[2 * kp], X[2 * kp + 1], &tt);
                f = (1.0 - tt) * fs[e] + tt * fs[kp];
            } else {
                int va = T[3 * e], vb = T[3 * e + 1], vc = T[3 * e + 2];
                double p[3] = {(i + (comp == 0 ? 0.0 : 0.5)) * h, (j + (comp == 1 ? 0.0 : 0.5)) * h,
                               (k + (comp == 2 ? 0.0 : 0.5)) * h};
                double w[3];
                tri_closest(p, X + 3 * (long)va, X + 3 * (long)vb, X + 3 * (long)vc, w);
                f = w[0] * fs[va] + w[1] * fs[vb] + w[2] * fs[vc];
            }
            out = f * dH / h;
            B[c] = ~0ull;
        }
    }
    F[c] = out;
}

int launch_irrot_force(Ctx* c, const ib_surface* s, const double* H, double* const F[3],
                       hipStream_t st) {
    int dim = c->d.dim;
    int n = s->n_markers;
    if (dim == 2) {
        hipLaunchKernelGGL(k_nearest_2d, dim3(grid_for(2L * n)), dim3(kBlock), 0, st, s->X, n, H,
                           c->d, c->best);
        for (int comp = 0; comp < 2; ++comp)
            hipLaunchKernelGGL(k_irrot_force<2>, dim3(grid_for(c->d.cells())), dim3(kBlock), 0, st,
                               s->X, s->elems, s->fs, H, c->d, comp, n, c->best, F[comp], c->flags);
    } else {
        int nt = s->n_elems;
        IB_CHECK(nt < (1 << kElemBits), IB_EINVAL, "ib_spread: too many triangles");
        hipLaunchKernelGGL(k_nearest_3d, dim3(grid_for(3L * nt * kNearLanes)), dim3(kBlock), 0, st, s->X, n,
                           s->elems, nt, H, c->d, c->best);
        for (int comp = 0; comp < 3; ++comp)
            hipLaunchKernelGGL(k_irrot_force<3>, dim3(grid_for(c->d.cells())), dim3(kBlock), 0, st,
                               s->X, s->elems, s->fs, H, c->d, comp, n, c->best, F[comp], c->flags);
    }
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// a6 coefficients
// rho = rho_out + (rho_in - rho_out) H, multiply and add rounded separately
// (no fused multiply-add), as the formula reads
__device__ __forceinline__ double cell_density(double rout, double drho, double H) {
#pragma clang fp contract(off)
    return rout + drho * H;
}

template <int DIM>
__global__ void k_coefficients(const double* __restrict__ H, Dims d, double rin, double rout,
                               double* __restrict__ b0, double* __restrict__ b1,
                               double* __restrict__ b2, double* __restrict__ rho) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    int i, j, k;
    cell_ijk(c, d.nx, d.ny, i, j, k);
    double drho = rin - rout;
    double rc = cell_density(rout, drho, H[c]);
    if (rho) rho[c] = rc;
    if (!b0) return;
    long cx = i == 0 ? c + d.nx - 1 : c - 1;
    long cy = j == 0 ? c + (long)(d.ny - 1) * d.nx : c - d.nx;
    b0[c] = 2.0 / (rc + cell_density(rout, drho, H[cx]));
    b1[c] = 2.0 / (rc + cell_density(rout, drho, H[cy]));
    if (DIM == 3) {
        long pl = (long)d.nx * d.ny;
        long cz = k == 0 ? c + (long)(d.nz - 1) * pl : c - pl;
        b2[c] = 2.0 / (rc + cell_density(rout, drho, H[cz]));
    }
}

int launch_coefficients(Ctx* c, const double* H, double rin, double rout, double* const beta[3],
                        double* rho, hipStream_t st) {
    double* b0 = beta ? beta[0] : nullptr;
    double* b1 = beta ? beta[1] : nullptr;
    double* b2 = beta ? beta[c->d.dim == 3 ? 2 : 1] : nullptr;
    if (c->d.dim == 2)
        hipLaunchKernelGGL(k_coefficients<2>, dim3(grid_for(c->d.cells())), dim3(kBlock), 0, st, H,
                           c->d, rin, rout, b0, b1, b1, rho);
    else
        hipLaunchKernelGGL(k_coefficients<3>, dim3(grid_for(c->d.cells())), dim3(kBlock), 0, st, H,
                           c->d, rin, rout, b0, b1, b2, rho);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// deterministic sums: fixed number of blocks, fixed tree inside a block
constexpr int kRedBlocks = 1024;

// One workgroup of 1024 threads per sum; each thread keeps 8 accumulators so
// that its loads are independent (one memory latency per 8192 partials instead
// of one per load), then a fixed butterfly inside each wave and a fixed serial
// sum over the 16 wave totals. Workgroup 1 (when launched) makes a second,
// independent sum of as many partials the same way.
constexpr int kSumThreads = 1024;

__global__ __launch_bounds__(kSumThreads) void k_sum_final(const double* __restrict__ in0, int n,
                                                           double* __restrict__ out0,
                                                           const double* __restrict__ in1,
                                                           double* __restrict__ out1) {
    __shared__ double sh[kSumThreads / 64];
    const double* __restrict__ in = blockIdx.x ? in1 : in0;
    double* __restrict__ out = blockIdx.x ? out1 : out0;
    const int t = threadIdx.x;
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    int q = t;
    for (; q + 7 * kSumThreads < n; q += 8 * kSumThreads) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += in[q + u * kSumThreads];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (q + u * kSumThreads < n) a[u] += in[q + u * kSumThreads];
    double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        double r = 0.0;
        for (int w = 0; w < kSumThreads / 64; ++w) r += sh[w];
        *out = r;
    }
}

int device_sum(const double* partials, int n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kSumThreads), 0, st, partials, n, out, partials, out);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

int device_sum2(const double* partials0, const double* partials1, int n, double* out0, double* out1,
                hipStream_t st) {
    hipLaunchKernelGGL(k_sum_final, dim3(2), dim3(kSumThreads), 0, st, partials0, n, out0, partials1, out1);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// a7 right side with partial sums for the mean
// face coefficient of the d-face of cell c: stored, or 2 / (rho_c + rho_{c-e_d})
// (the stored value bit for bit)
template <bool RHO>
__device__ __forceinline__ double face_beta(const double* __restrict__ b, const double* __restrict__ rho, long c,
                                           long cm) {
    if constexpr (RHO)
        return 2.0 / (rho[c] + rho[cm]);
    else
        return b[c];
}

template <int DIM, bool RHO>
__global__ void k_rhs(const double* __restrict__ u0, const double* __restrict__ u1,
                      const double* __restrict__ u2, const double* __restrict__ F0,
                      const double* __restrict__ F1, const double* __restrict__ F2,
                      const double* __restrict__ b0, const double* __restrict__ b1,
                      const double* __restrict__ b2, const double* __restrict__ rho, Dims d, double inv_dt,
                      double* __restrict__ b, double* __restrict__ partial) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    long N = d.cells();
    double inv_h = 1.0 / d.h;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_ijk(c, d.nx, d.ny, i, j, k);
        long cx = i == d.nx - 1 ? c - (d.nx - 1) : c + 1;
        long cy = j == d.ny - 1 ? c - (long)(d.ny - 1) * d.nx : c + d.nx;
        long mx = 0, my = 0;
        if constexpr (RHO) {
            mx = i == 0 ? c + d.nx - 1 : c - 1;
            my = j == 0 ? c + (long)(d.ny - 1) * d.nx : c - d.nx;
        }
        double s = ((u0[cx] * inv_dt + face_beta<RHO>(b0, rho, cx, c) * F0[cx]) -
                    (u0[c] * inv_dt + face_beta<RHO>(b0, rho, c, mx) * F0[c]));
        s += ((u1[cy] * inv_dt + face_beta<RHO>(b1, rho, cy, c) * F1[cy]) -
              (u1[c] * inv_dt + face_beta<RHO>(b1, rho, c, my) * F1[c]));
        if (DIM == 3) {
            long pl = (long)d.nx * d.ny;
            long cz = k == d.nz - 1 ? c - (long)(d.nz - 1) * pl : c + pl;
            long mz = 0;
            if constexpr (RHO) mz = k == 0 ? c + (long)(d.nz - 1) * pl : c - pl;
            s += ((u2[cz] * inv_dt + face_beta<RHO>(b2, rho, cz, c) * F2[cz]) -
                  (u2[c] * inv_dt + face_beta<RHO>(b2, rho, c, mz) * F2[c]));
        }
        double v = s * inv_h;
        b[c] = v;
        acc += v;
    }
    double tot = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_sub_mean(double* __restrict__ x, long N, const double* __restrict__ sum) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    x[c] -= *sum / (double)N;
}

int launch_rhs(Ctx* c, const double* const us[3], const double* const F[3],
               const double* const beta[3], double dt, double* b, hipStream_t st, const double* rho) {
    long N = c->d.cells();
    int blocks = (int)std::min<long>(kRedBlocks, (long)grid_for(N));
    const double* b0 = rho ? nullptr : beta[0];
    const double* b1 = rho ? nullptr : beta[1];
    const double* b2 = rho ? nullptr : beta[c->d.dim == 3 ? 2 : 1];
    if (c->d.dim == 2) {
        if (rho)
            hipLaunchKernelGGL((k_rhs<2, true>), dim3(blocks), dim3(kBlock), 0, st, us[0], us[1], us[1], F[0],
                               F[1], F[1], b0, b1, b1, rho, c->d, 1.0 / dt, b, c->red);
        else
            hipLaunchKernelGGL((k_rhs<2, false>), dim3(blocks), dim3(kBlock), 0, st, us[0], us[1], us[1], F[0],
                               F[1], F[1], b0, b1, b1, rho, c->d, 1.0 / dt, b, c->red);
    } else {
        if (rho)
            hipLaunchKernelGGL((k_rhs<3, true>), dim3(blocks), dim3(kBlock), 0, st, us[0], us[1], us[2], F[0],
                               F[1], F[2], b0, b1, b2, rho, c->d, 1.0 / dt, b, c->red);
        else
            hipLaunchKernelGGL((k_rhs<3, false>), dim3(blocks), dim3(kBlock), 0, st, us[0], us[1], us[2], F[0],
                               F[1], F[2], b0, b1, b2, rho, c->d, 1.0 / dt, b, c->red);
    }
    IB_TRY(device_sum(c->red, blocks, c->red + kRedBlocks, st));
    hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(N)), dim3(kBlock), 0, st, b, N, c->red + kRedBlocks);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// a11 velocity update
template <int DIM, bool RHO>
__global__ void k_update(const double* __restrict__ u0, const double* __restrict__ u1,
                         const double* __restrict__ u2, const double* __restrict__ F0,
                         const double* __restrict__ F1, const double* __restrict__ F2,
                         const double* __restrict__ b0, const double* __restrict__ b1,
                         const double* __restrict__ b2, const double* __restrict__ rho,
                         const double* __restrict__ p, Dims d,
                         double dt, double* __restrict__ o0, double* __restrict__ o1,
                         double* __restrict__ o2) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    int i, j, k;
    cell_ijk(c, d.nx, d.ny, i, j, k);
    double inv_h = 1.0 / d.h;
    double pc = p[c];
    long cx = i == 0 ? c + d.nx - 1 : c - 1;
    long cy = j == 0 ? c + (long)(d.ny - 1) * d.nx : c - d.nx;
    double gx = (pc - p[cx]) * inv_h, gy = (pc - p[cy]) * inv_h;
    double v0 = u0[c] + dt * face_beta<RHO>(b0, rho, c, cx) * (F0[c] - gx);
    double v1 = u1[c] + dt * face_beta<RHO>(b1, rho, c, cy) * (F1[c] - gy);
    double v2 = 0.0;
    if (DIM == 3) {
        long pl = (long)d.nx * d.ny;
        long cz = k == 0 ? c + (long)(d.nz - 1) * pl : c - pl;
        double gz = (pc - p[cz]) * inv_h;
        v2 = u2[c] + dt * face_beta<RHO>(b2, rho, c, cz) * (F2[c] - gz);
    }
    o0[c] = v0;
    o1[c] = v1;
    if (DIM == 3) o2[c] = v2;
}

int launch_update(Ctx* c, const double* const us[3], const double* const F[3],
                  const double* const beta[3], const double* p, double dt, double* const un[3],
                  hipStream_t st, const double* rho) {
    const dim3 g(grid_for(c->d.cells())), blk(kBlock);
    const double* b0 = rho ? nullptr : beta[0];
    const double* b1 = rho ? nullptr : beta[1];
    const double* b2 = rho ? nullptr : beta[c->d.dim == 3 ? 2 : 1];
    if (c->d.dim == 2) {
        if (rho)
            hipLaunchKernelGGL((k_update<2, true>), g, blk, 0, st, us[0], us[1], us[1], F[0], F[1], F[1], b0, b1,
                               b1, rho, p, c->d, dt, un[0], un[1], un[1]);
        else
            hipLaunchKernelGGL((k_update<2, false>), g, blk, 0, st, us[0], us[1], us[1], F[0], F[1], F[1], b0,
                               b1, b1, rho, p, c->d, dt, un[0], un[1], un[1]);
    } else {
        if (rho)
            hipLaunchKernelGGL((k_update<3, true>), g, blk, 0, st, us[0], us[1], us[2], F[0], F[1], F[2], b0, b1,
                               b2, rho, p, c->d, dt, un[0], un[1], un[2]);
        else
            hipLaunchKernelGGL((k_update<3, false>), g, blk, 0, st, us[0], us[1], us[2], F[0], F[1], F[2], b0,
                               b1, b2, rho, p, c->d, dt, un[0], un[1], un[2]);
    }
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// a12 diagnostics: per-block partials of 9 quantities + 2 maxima, summed on
// the host in block order
constexpr int kDiagQ = 11;

template <int DIM>
__global__ void k_diag(const double* __restrict__ p, const double* __restrict__ H,
                       const double* __restrict__ u0, const double* __restrict__ u1,
                       const double* __restrict__ u2, const double* __restrict__ F0,
                       const double* __restrict__ F1, const double* __restrict__ F2, Dims d,
                       double* __restrict__ partial) {
    __shared__ double sh[kBlock];
    double q[kDiagQ];
    for (int a = 0; a < kDiagQ; ++a) q[a] = 0.0;
    long N = d.cells();
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        if (p && H) {
            double hv = H[c];
            if (hv >= 1.0 - 1e-12) { q[0] += p[c]; q[1] += 1.0; }
            if (hv <= 1e-12) { q[2] += p[c]; q[3] += 1.0; }
        }
        if (u0) {
            double s = u0[c] * u0[c] + u1[c] * u1[c];
            if (DIM == 3) s += u2[c] * u2[c];
            q[4] += s;
        }
        if (F0) {
            q[5] += F0[c];
            q[6] += F1[c];
            if (DIM == 3) q[7] += F2[c];
            int i, j, k;
            cell_ijk(c, d.nx, d.ny, i, j, k);
            long cx = i == 0 ? c + d.nx - 1 : c - 1;
            long cy = j == 0 ? c + (long)(d.ny - 1) * d.nx : c - d.nx;
            // index-form curl, (x, y) plane
            double cur = (F1[c] - F1[cx]) - (F0[c] - F0[cy]);
            double m = fabs(cur);
            double fm = fmax(fabs(F0[c]), fabs(F1[c]));
            if (DIM == 3) {
                long pl = (long)d.nx * d.ny;
                long cz = k == 0 ? c + (long)(d.nz - 1) * pl : c - pl;
                double cyz = (F2[c] - F2[cy]) - (F1[c] - F1[cz]);
                double czx = (F0[c] - F0[cz]) - (F2[c] - F2[cx]);
                m = fmax(m, fmax(fabs(cyz), fabs(czx)));
                fm = fmax(fm, fabs(F2[c]));
            }
            q[9] = fmax(q[9], m);
            q[10] = fmax(q[10], fm);
        }
    }
    for (int a = 0; a < 9; ++a) {
        double r = block_reduce_sum(q[a], sh);
        if (threadIdx.x == 0) partial[(long)blockIdx.x * kDiagQ + a] = r;
    }
    for (int a = 9; a < kDiagQ; ++a) {
        sh[threadIdx.x] = q[a];
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(long)blockIdx.x * kDiagQ + a] = sh[0];
        __syncthreads();
    }
}

int launch_diagnostics(Ctx* c, const double* p, const double* H, const double* const u[3],
                       const double* const F[3], ib_diag* out, hipStream_t st) {
    int blocks = 256;
    const double* u0 = u ? u[0] : nullptr;
    const double* u1 = u ? u[1] : nullptr;
    const double* u2 = u ? u[c->d.dim == 3 ? 2 : 1] : nullptr;
    const double* F0 = F ? F[0] : nullptr;
    const double* F1 = F ? F[1] : nullptr;
    const double* F2 = F ? F[c->d.dim == 3 ? 2 : 1] : nullptr;
    if (c->d.dim == 2)
        hipLaunchKernelGGL(k_diag<2>, dim3(blocks), dim3(kBlock), 0, st, p, H, u0, u1, u2, F0, F1,
                           F2, c->d, c->red);
    else
        hipLaunchKernelGGL(k_diag<3>, dim3(blocks), dim3(kBlock), 0, st, p, H, u0, u1, u2, F0, F1,
                           F2, c->d, c->red);
    IB_HIP(hipGetLastError());
    IB_HIP(hipMemcpyAsync(c->host_red, c->red, sizeof(double) * blocks * kDiagQ,
                          hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    double q[kDiagQ] = {0};
    for (int b = 0; b < blocks; ++b) {
        for (int a = 0; a < 9; ++a) q[a] += c->host_red[b * kDiagQ + a];
        for (int a = 9; a < kDiagQ; ++a) q[a] = std::max(q[a], c->host_red[b * kDiagQ + a]);
    }
    double hd = c->d.dim == 3 ? c->d.h * c->d.h * c->d.h : c->d.h * c->d.h;
    out->dP = (q[1] > 0 && q[3] > 0) ? q[0] / q[1] - q[2] / q[3] : 0.0;
    out->tke = q[4] * hd;
    out->force_sum[0] = q[5] * hd;
    out->force_sum[1] = q[6] * hd;
    out->force_sum[2] = q[7] * hd;
    out->curl_max = q[9];
    out->f_max = q[10];
    return IB_OK;
}

}  // namespace ib
