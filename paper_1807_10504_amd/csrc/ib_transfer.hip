// Marker binning, velocity interpolation and conventional delta spreading.
//
// Interpolation: eq jump_condu, U(X_s) = sum_f u(x_f) delta_h(x_f - X_s) h^dim,
// delta_h = prod_d phi(dx_d/h)/h, phi(q) = (1 + cos(pi q/2))/4 for |q| < 2
// (eqs delta, cherby in grid units). One thread per (marker, component)
// gathers its 4^dim faces.
//
// Conventional spreading: eq delta_vec, F(x_f) = sum_s F_s delta_h(x_f - X_s).
// Markers are counting-sorted into tiles of 4^dim cells (stable radix sort on
// the tile key); every face gathers the markers of the <= 2^dim tiles that
// cover its kernel support, in tile order then marker order, so the sum has
// a fixed order and the result is bitwise reproducible (no float atomics).
#include <hipcub/hipcub.hpp>

#include "common.h"

namespace ib {

__device__ __forceinline__ double phi_dev(double q) {
    return fabs(q) < 2.0 ? 0.25 * (1.0 + cospi(0.5 * q)) : 0.0;
}

// ---------------------------------------------------------------------------
// a1: binning
__global__ void k_tile_keys(const double* __restrict__ X, int n, Dims d, int tnx, int tny,
                            int32_t* __restrict__ key, int32_t* __restrict__ idx) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int dim = d.dim;
    int c[3] = {0, 0, 0};
    int nn[3] = {d.nx, d.ny, d.nz};
    for (int e = 0; e < dim; ++e) {
        double v = X[(long)s * dim + e] / d.h;
        c[e] = wrap((int)floor(v), nn[e]) / kTile;
    }
    key[s] = (c[2] * tny + c[1]) * tnx + c[0];
    idx[s] = s;
}

__global__ void k_tile_start(const int32_t* __restrict__ sorted_key, int n, int n_tiles,
                             int32_t* __restrict__ start) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_tiles) return;
    // first position with key >= t
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (sorted_key[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    start[t] = lo;
}

int launch_bin_markers(Ctx* c, const ib_surface* s, hipStream_t st) {
    int n = s->n_markers;
    if (n == 0) {
        IB_HIP(hipMemsetAsync(c->tile_start, 0, sizeof(int32_t) * (c->n_tiles + 1), st));
        return IB_OK;
    }
    hipLaunchKernelGGL(k_tile_keys, dim3(grid_for(n)), dim3(kBlock), 0, st, s->X, n, c->d, c->tnx,
                       c->tny, c->bin_key, c->bin_idx);
    int end_bit = 1;
    while ((1 << end_bit) <= c->n_tiles) ++end_bit;
    size_t need = 0;
    IB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, need, c->bin_key, c->bin_key_sorted,
                                               c->bin_idx, c->bin_order, n, 0, end_bit, st));
    IB_CHECK(need <= c->sort_tmp_bytes, IB_ENOMEM, "ib_bin_markers: sort workspace too small");
    size_t bytes = c->sort_tmp_bytes;
    IB_HIP(hipcub::DeviceRadixSort::SortPairs(c->sort_tmp, bytes, c->bin_key, c->bin_key_sorted,
                                               c->bin_idx, c->bin_order, n, 0, end_bit, st));
    hipLaunchKernelGGL(k_tile_start, dim3(grid_for(c->n_tiles + 1)), dim3(kBlock), 0, st,
                       c->bin_key_sorted, n, c->n_tiles, c->tile_start);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// a2: interpolation
template <int DIM>
__global__ void k_interp(const double* __restrict__ u0, const double* __restrict__ u1,
                         const double* __restrict__ u2, const double* __restrict__ X, int n,
                         Dims d, double* __restrict__ U) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * DIM) return;
    int s = t / DIM, comp = t - s * DIM;
    const double* u = comp == 0 ? u0 : (comp == 1 ? u1 : u2);
    int nn[3] = {d.nx, d.ny, d.nz};
    int id[3][4];
    double w[3][4];
    for (int e = 0; e < DIM; ++e) {
        double off = (e == comp) ? 0.0 : 0.5;
        double sv = X[(long)s * DIM + e] / d.h - off;
        int base = (int)floor(sv) - 1;
        for (int q = 0; q < 4; ++q) {
            id[e][q] = wrap(base + q, nn[e]);
            w[e][q] = phi_dev((double)(base + q) - sv);
        }
    }
    double acc = 0.0;
    if (DIM == 2) {
        for (int b = 0; b < 4; ++b) {
            double ab = 0.0;
            const double* row = u + (long)id[1][b] * d.nx;
            for (int a = 0; a < 4; ++a) ab += w[0][a] * row[id[0][a]];
            acc += w[1][b] * ab;
        }
    } else {
        for (int k = 0; k < 4; ++k) {
            double ak = 0.0;
            for (int b = 0; b < 4; ++b) {
                double ab = 0.0;
                const double* row = u + ((long)id[2][k] * d.ny + id[1][b]) * d.nx;
                for (int a = 0; a < 4; ++a) ab += w[0][a] * row[id[0][a]];
                ak += w[1][b] * ab;
            }
            acc += w[2][k] * ak;
        }
    }
    U[t] = acc;
}

int launch_interp(Ctx* c, const double* const u[3], const ib_surface* s, double* U,
                  hipStream_t st) {
    int n = s->n_markers;
    if (n == 0) return IB_OK;
    if (c->d.dim == 2)
        hipLaunchKernelGGL(k_interp<2>, dim3(grid_for((long)n * 2)), dim3(kBlock), 0, st, u[0],
                           u[1], u[1], s->X, n, c->d, U);
    else
        hipLaunchKernelGGL(k_interp<3>, dim3(grid_for((long)n * 3)), dim3(kBlock), 0, st, u[0],
                           u[1], u[2], s->X, n, c->d, U);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// conventional spreading
// marker force vectors F_s = fs * ds * n (2D default normal: left
// perpendicular of the chord X_{k+1} - X_{k-1})
__global__ void k_marker_force(const double* __restrict__ X, const double* __restrict__ nrm,
                               const double* __restrict__ fs, const double* __restrict__ ds, int n,
                               int dim, double* __restrict__ Fs) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double a = fs[s] * ds[s];
    if (nrm) {
        for (int e = 0; e < dim; ++e) Fs[(long)s * dim + e] = a * nrm[(long)s * dim + e];
    } else {
        int sp = s + 1 == n ? 0 : s + 1, sm = s == 0 ? n - 1 : s - 1;
        double tx = X[2 * sp] - X[2 * sm], ty = X[2 * sp + 1] - X[2 * sm + 1];
        double inv = 1.0 / sqrt(tx * tx + ty * ty);
        Fs[2 * s] = a * (-ty * inv);
        Fs[2 * s + 1] = a * (tx * inv);
    }
}

template <int DIM>
__global__ void k_spread_delta(const double* __restrict__ X, const double* __restrict__ Fs,
                               const int32_t* __restrict__ order, const int32_t* __restrict__ start,
                               Dims d, int tnx, int tny, int tnz, int comp, double* __restrict__ F) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    int i = (int)(c % d.nx);
    long r = c / d.nx;
    int j = (int)(r % d.ny);
    int k = (int)(r / d.ny);
    int ci[3] = {i, j, k};
    int nn[3] = {d.nx, d.ny, d.nz};
    int tn[3] = {tnx, tny, tnz};
    double L[3] = {d.nx * d.h, d.ny * d.h, d.nz * d.h};
    double xf[3];
    int t0[3], tc[3];
    for (int e = 0; e < DIM; ++e) {
        double off = (e == comp) ? 0.0 : 0.5;
        xf[e] = (ci[e] + off) * d.h;
        // cells whose markers can reach this face: |x_f - X| < 2h
        int lo = (int)floor((ci[e] + off) - 2.0);
        int hi = (int)floor((ci[e] + off) + 2.0);
        int tlo = (int)floor((double)lo / kTile);
        int thi = (int)floor((double)hi / kTile);
        t0[e] = tlo;
        tc[e] = thi - tlo + 1;  // 1 or 2
    }
    const double inv = 1.0 / (DIM == 2 ? d.h * d.h : d.h * d.h * d.h);
    double acc = 0.0;
    int tzc = DIM == 3 ? tc[2] : 1;
    for (int a2 = 0; a2 < tzc; ++a2) {
        int tz = DIM == 3 ? wrap(t0[2] + a2, tn[2]) : 0;
        for (int a1 = 0; a1 < tc[1]; ++a1) {
            int ty = wrap(t0[1] + a1, tn[1]);
            for (int a0 = 0; a0 < tc[0]; ++a0) {
                int tx = wrap(t0[0] + a0, tn[0]);
                int t = (tz * tny + ty) * tnx + tx;
                int b = start[t], e_ = start[t + 1];
                for (int q = b; q < e_; ++q) {
                    int s = order[q];
                    double w = 1.0;
                    for (int e = 0; e < DIM; ++e) {
                        double dx = xf[e] - X[(long)s * DIM + e];
                        dx -= L[e] * rint(dx / L[e]);
                        w *= phi_dev(dx / d.h);
                    }
                    acc += w * (Fs[(long)s * DIM + comp] * inv);
                }
            }
        }
    }
    (void)nn;
    F[c] = acc;
}

int launch_spread_delta(Ctx* c, const ib_surface* s, double* const F[3], hipStream_t st) {
    int n = s->n_markers;
    int dim = c->d.dim;
    IB_TRY(launch_bin_markers(c, s, st));
    if (n > 0)
        hipLaunchKernelGGL(k_marker_force, dim3(grid_for(n)), dim3(kBlock), 0, st, s->X, s->nrm,
                           s->fs, s->ds, n, dim, c->offv);
    for (int comp = 0; comp < dim; ++comp) {
        if (dim == 2)
            hipLaunchKernelGGL(k_spread_delta<2>, dim3(grid_for(c->d.cells())), dim3(kBlock), 0,
                               st, s->X, c->offv, c->bin_order, c->tile_start, c->d, c->tnx,
                               c->tny, c->tnz, comp, F[comp]);
        else
            hipLaunchKernelGGL(k_spread_delta<3>, dim3(grid_for(c->d.cells())), dim3(kBlock), 0,
                               st, s->X, c->offv, c->bin_order, c->tile_start, c->d, c->tnx,
                               c->tny, c->tnz, comp, F[comp]);
    }
    IB_HIP(hipGetLastError());
    return IB_OK;
}

}  // namespace ib
