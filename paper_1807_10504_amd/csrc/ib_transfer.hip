// Marker binning, velocity interpolation and conventional delta spreading.
//
// Interpolation: eq jump_condu, U(X_s) = sum_f u(x_f) delta_h(x_f - X_s) h^dim,
// delta_h = prod_d phi(dx_d/h)/h, phi(q) = (1 + cos(pi q/2))/4 for |q| < 2
// (eqs delta, cherby in grid units). One thread per (marker, component)
// gathers its 4^dim faces.
//
// Conventional spreading: eq delta_vec, F(x_f) = sum_s F_s delta_h(x_f - X_s).
// Markers are counting-sorted into tiles of 4^dim cells (histogram of the
// tile keys, exclusive scan, scatter, marker order restored within each
// tile); every face gathers the markers of the <= 2^dim tiles that cover its
// kernel support, in tile order then marker order, so the sum has a fixed
// order and the result is bitwise reproducible (no float atomics).
#include "common.h"

namespace ib {

__device__ __forceinline__ double phi_dev(double q) {
    return fabs(q) < 2.0 ? 0.25 * (1.0 + cospi(0.5 * q)) : 0.0;
}

// ---------------------------------------------------------------------------
// a1: binning
__global__ void k_tile_keys(const double* __restrict__ X, int n, Dims d, int tnx, int tny,
                            int32_t* __restrict__ key) {
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
}

__global__ void k_fill_i32(int32_t* __restrict__ x, int n, int32_t v) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

// histogram of the tile keys (integer atomics: the counts do not depend on
// the order the adds land in)
__global__ void k_tile_count(const int32_t* __restrict__ key, int n, int32_t* __restrict__ count) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) atomicAdd(&count[key[s]], 1);
}

// Exclusive scan of in[0, n) into out in blocks of kScanTile items (each
// thread four consecutive items; lane prefixes by shuffles, wave totals
// through LDS); the block's total goes to part[blockIdx.x].
__global__ __launch_bounds__(kScanThreads) void k_scan_block(const int32_t* __restrict__ in, int n,
                                                             int32_t* __restrict__ out,
                                                             int32_t* __restrict__ part) {
    __shared__ int32_t wsum[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const long base = (long)blockIdx.x * kScanTile + (long)t * kScanItems;
    int32_t v[kScanItems];
    int32_t own = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < n ? in[base + q] : 0;
        own += v[q];
    }
    // inclusive scan of the thread totals across the wave
    int32_t inc = own;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (t == 0) {
        int32_t acc = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            const int32_t x = wsum[w];
            wsum[w] = acc;
            acc += x;
        }
        part[blockIdx.x] = acc;
    }
    __syncthreads();
    int32_t run = wsum[wave] + inc - own;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
}

__global__ void k_scan_add(int32_t* __restrict__ out, int n, const int32_t* __restrict__ part) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += part[i / kScanTile];
}

// slot of each marker in its tile (the order the atomics land in) ...
__global__ void k_tile_scatter(const int32_t* __restrict__ key, int n, const int32_t* __restrict__ start,
                               int32_t* __restrict__ cursor, int32_t* __restrict__ order) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int k = key[s];
    order[start[k] + atomicAdd(&cursor[k], 1)] = s;
}

// ... then each tile's markers back into ascending index (a stable sort's
// order); tiles hold a handful of markers, so one thread sorts one tile
__global__ void k_tile_order(const int32_t* __restrict__ start, int n_tiles, int32_t* __restrict__ order) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const int a = start[t], b = start[t + 1];
    for (int i = a + 1; i < b; ++i) {
        const int32_t v = order[i];
        int j = i - 1;
        while (j >= a && order[j] > v) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
}

// tile_start = exclusive scan of the n_tiles + 1 counts (the last is 0, so
// tile_start[n_tiles] = n)
static int scan_tiles(Ctx* c, hipStream_t st) {
    const int n = c->n_tiles + 1;
    const int blocks = (int)((n + kScanTile - 1) / kScanTile);
    IB_CHECK(blocks <= kScanTile, IB_EINVAL, "ib_bin_markers: too many tiles for the scan");
    hipLaunchKernelGGL(k_scan_block, dim3(blocks), dim3(kScanThreads), 0, st, c->bin_count, n, c->tile_start,
                       c->scan_part);
    if (blocks > 1) {
        // the block totals, scanned in place by one block (its own total is not needed)
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(kScanThreads), 0, st, c->scan_part, blocks,
                           c->scan_part, c->scan_part + blocks);
        hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n)), dim3(kBlock), 0, st, c->tile_start, n, c->scan_part);
    }
    return IB_OK;
}

int launch_bin_markers(Ctx* c, const ib_surface* s, hipStream_t st) {
    int n = s->n_markers;
    const int nt1 = c->n_tiles + 1;
    if (n == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nt1)), dim3(kBlock), 0, st, c->tile_start, nt1, 0);
        IB_HIP(hipGetLastError());
        return IB_OK;
    }
    hipLaunchKernelGGL(k_tile_keys, dim3(grid_for(n)), dim3(kBlock), 0, st, s->X, n, c->d, c->tnx,
                       c->tny, c->bin_key);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nt1)), dim3(kBlock), 0, st, c->bin_count, nt1, 0);
    hipLaunchKernelGGL(k_tile_count, dim3(grid_for(n)), dim3(kBlock), 0, st, c->bin_key, n, c->bin_count);
    IB_TRY(scan_tiles(c, st));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nt1)), dim3(kBlock), 0, st, c->bin_count, nt1, 0);
    hipLaunchKernelGGL(k_tile_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, c->bin_key, n, c->tile_start,
                       c->bin_count, c->bin_order);
    hipLaunchKernelGGL(k_tile_order, dim3(grid_for(c->n_tiles)), dim3(kBlock), 0, st, c->tile_start,
                       c->n_tiles, c->bin_order);
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
