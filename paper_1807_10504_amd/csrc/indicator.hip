// Indicator function of the conventional scheme (Section 2.2, eqs indicator,
// ind_psn): div grad I = div delta_vec, delta_vec the unit normals times the
// arc elements spread by the discrete delta function (eq delta_vec). The
// periodic solution is fixed by the integral of I equalling the enclosed area.
//
// Path: conventional spreading of n ds (the a5 kernels with fs = 1) ->
// divergence, mean removed -> flexible-CG multigrid with unit coefficients
// (density 1 everywhere, so beta = 1 bitwise) -> I = P + A / |Omega| with A the
// shoelace area of the markers.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ib {

constexpr int kIndRed = 256;

// b = div F (faces at the low side of each cell), block partials of sum b
__global__ void k_ind_div(const double* __restrict__ Fx, const double* __restrict__ Fy, Dims d,
                          double* __restrict__ b, double* __restrict__ part) {
    __shared__ double sh[kBlock];
    const long N = d.cells();
    const double inv_h = 1.0 / d.h;
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        const int i = (int)(c % d.nx), j = (int)(c / d.nx);
        const long cx = i + 1 == d.nx ? c - (d.nx - 1) : c + 1;
        const long cy = j + 1 == d.ny ? c - (long)(d.ny - 1) * d.nx : c + d.nx;
        const double v = ((Fx[cx] - Fx[c]) + (Fy[cy] - Fy[c])) * inv_h;
        b[c] = v;
        acc += v;
    }
    const double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_ind_sub_mean(double* __restrict__ b, long N, const double* __restrict__ sum) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) b[c] -= *sum / (double)N;
}

// block partials of the shoelace sum x_k y_{k+1} - x_{k+1} y_k
__global__ void k_ind_shoelace(const double* __restrict__ X, int n, double* __restrict__ part) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int q = k + 1 == n ? 0 : k + 1;
        acc += X[2 * k] * X[2 * q + 1] - X[2 * q] * X[2 * k + 1];
    }
    const double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// I = P + (shoelace sum / 2) / |Omega|
__global__ void k_ind_shift(double* __restrict__ I, long N, double inv_vol, const double* __restrict__ s2) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) I[c] += 0.5 * *s2 * inv_vol;
}

__global__ void k_ind_fill(double* __restrict__ a, long n, double v) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) a[c] = v;
}

}  // namespace ib

using namespace ib;

struct ib_indicator {
    Dims d;
    int max_markers = 0;
    mg_handle* mg = nullptr;
    double* ones_cells = nullptr;    // density 1 for the unit-coefficient hierarchy
    double* ones_markers = nullptr;  // fs = 1
    double* F[2] = {nullptr, nullptr};
    double* b = nullptr;
    double* red = nullptr;           // kIndRed partials + 2 sums
};

static void free_indicator(ib_indicator* a) {
    if (!a) return;
    if (a->mg) mg_destroy(a->mg);
    for (double* p : {a->ones_cells, a->ones_markers, a->F[0], a->F[1], a->b, a->red})
        if (p) hipFree(p);
    delete a;
}

extern "C" int ib_indicator_create(const ib_grid* g, int max_markers, ib_indicator** out) {
    IB_CHECK(g && out, IB_EINVAL, "ib_indicator_create: null argument");
    IB_CHECK(g->dim == 2, IB_EINVAL, "ib_indicator_create: the conventional indicator is 2D");
    IB_CHECK(max_markers >= 3, IB_EINVAL, "ib_indicator_create: max_markers");
    ib_indicator* a = new ib_indicator();
    a->d = make_dims(*g);
    a->max_markers = max_markers;
    mg_opts o{MG_FP64, 2, 2, 4, 1, 0};
    int rc = mg_setup(g, &o, &a->mg);
    if (rc != IB_OK) {
        a->mg = nullptr;
        free_indicator(a);
        return rc;
    }
    const long N = a->d.cells();
    bool ok = true;
    ok = ok && hipMalloc((void**)&a->ones_cells, sizeof(double) * N) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->ones_markers, sizeof(double) * max_markers) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->F[0], sizeof(double) * N) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->F[1], sizeof(double) * N) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->b, sizeof(double) * N) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->red, sizeof(double) * (kIndRed + 2)) == hipSuccess;
    if (!ok) {
        free_indicator(a);
        return fail(IB_ENOMEM, "ib_indicator_create: out of memory");
    }
    hipLaunchKernelGGL(k_ind_fill, dim3(grid_for(N)), dim3(kBlock), 0, 0, a->ones_cells, N, 1.0);
    hipLaunchKernelGGL(k_ind_fill, dim3(grid_for(max_markers)), dim3(kBlock), 0, 0, a->ones_markers,
                       (long)max_markers, 1.0);
    rc = mg_update_density(a->mg, a->ones_cells, nullptr);
    if (rc == IB_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(IB_EHIP, "ib_indicator_create: set-up");
    if (rc != IB_OK) {
        free_indicator(a);
        return rc;
    }
    *out = a;
    return IB_OK;
}

extern "C" void ib_indicator_destroy(ib_indicator* a) { free_indicator(a); }

extern "C" int ib_indicator_solve(ib_ctx* ctx, ib_indicator* a, const ib_surface* s, double rtol,
                                  int max_cycles, double* I, mg_stats* stats, void* stream) {
    IB_CHECK(ctx && a && s && I, IB_EINVAL, "ib_indicator_solve: null argument");
    Ctx* c = ctx;
    IB_CHECK(c->d.dim == 2 && c->d.nx == a->d.nx && c->d.ny == a->d.ny && c->d.h == a->d.h, IB_EINVAL,
             "ib_indicator_solve: the handle belongs to another grid");
    const int n = s->n_markers;
    IB_CHECK(n >= 3 && n <= a->max_markers && n <= c->max_markers, IB_EINVAL,
             "ib_indicator_solve: marker count");
    IB_CHECK(s->X && s->nrm && s->ds, IB_EINVAL, "ib_indicator_solve: X, nrm and ds are required");
    IB_CHECK(rtol > 0 && max_cycles > 0, IB_EINVAL, "ib_indicator_solve: rtol, max_cycles");
    hipStream_t st = (hipStream_t)stream;
    const long N = c->d.cells();
    ib_surface sc = *s;
    sc.fs = a->ones_markers;
    double* F[3] = {a->F[0], a->F[1], a->F[1]};
    IB_TRY(launch_spread_delta(c, &sc, F, st));
    const int nb = (int)std::min<long>(kIndRed, (long)grid_for(N));
    hipLaunchKernelGGL(k_ind_div, dim3(nb), dim3(kBlock), 0, st, a->F[0], a->F[1], c->d, a->b, a->red);
    IB_TRY(device_sum(a->red, nb, a->red + kIndRed, st));
    hipLaunchKernelGGL(k_ind_sub_mean, dim3(grid_for(N)), dim3(kBlock), 0, st, a->b, N, a->red + kIndRed);
    const int ns = (int)std::min<long>(kIndRed, (long)grid_for(n));
    hipLaunchKernelGGL(k_ind_shoelace, dim3(ns), dim3(kBlock), 0, st, s->X, n, a->red);
    IB_TRY(device_sum(a->red, ns, a->red + kIndRed + 1, st));
    hipLaunchKernelGGL(k_ind_fill, dim3(grid_for(N)), dim3(kBlock), 0, st, I, N, 0.0);
    IB_HIP(hipGetLastError());
    int rc = mg_solve(a->mg, a->b, I, rtol, max_cycles, 0, stats, stream);
    if (rc != IB_OK && rc != IB_ENOTCONV) return rc;
    hipLaunchKernelGGL(k_ind_shift, dim3(grid_for(N)), dim3(kBlock), 0, st, I, N,
                       1.0 / ((double)N * c->d.h * c->d.h), a->red + kIndRed + 1);
    IB_HIP(hipGetLastError());
    return rc;
}
