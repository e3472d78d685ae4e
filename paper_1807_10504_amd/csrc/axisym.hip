// Axisymmetric projection step (Section 2.1 in cylindrical coordinates,
// eq curv_ax, the static drop of Section 5.1).
//
// Half plane r in [0, nr h], z in [0, nz h], arrays nz x nr with r fastest,
// periodic in z. u_r lives on the face at r = i h: face column 0 is the axis
// and, one period on, the outer wall; it carries no flux and holds u_r = 0.
// Annular finite volumes multiplied by the cell radius give a symmetric
// pressure operator with face coefficients r_i beta_r and r_c beta_z; it
// vanishes on face column 0, which also cuts the periodic wrap in r, so the
// plane multigrid solves it unchanged.
//
// The interface is the meridian curve mirrored about the axis, closed, in a
// doubled plane (2 nr x nz, axis at x = nr h): H and the irrotational face
// force come from the planar kernels there (symmetric about the axis, so the
// axis faces get no force) and are copied to the half plane.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ib {

constexpr int kAxiRed = 1024;

// doubled-plane velocity from the half plane: u_r odd, u_z even about the axis
__global__ void k_axi_mirror(const double* __restrict__ ur, const double* __restrict__ uz, int nr,
                             int nz, double* __restrict__ dr, double* __restrict__ dz) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = 2 * nr;
    if (t >= (long)w * nz) return;
    const int k = (int)(t / w), j = (int)(t - (long)k * w);
    const long row = (long)k * nr;
    if (j >= nr) {
        dr[t] = ur[row + (j - nr)];
        dz[t] = uz[row + (j - nr)];
    } else {
        dr[t] = j == 0 ? 0.0 : -ur[row + (nr - j)];
        dz[t] = uz[row + (nr - 1 - j)];
    }
}

// face column 0: no coefficient, no force; r-weighted coefficients of the
// symmetric operator: r_i beta_r, r_c beta_z
__global__ void k_axi_prepare(double* __restrict__ br, const double* __restrict__ bz,
                              double* __restrict__ Fr, int nr, long N, double h,
                              double* __restrict__ wr, double* __restrict__ wz) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const int i = (int)(c % nr);
    if (i == 0) {
        br[c] = 0.0;
        Fr[c] = 0.0;
    }
    wr[c] = ((double)i * h) * br[c];
    wz[c] = (((double)i + 0.5) * h) * bz[c];
}

// b = r_c div(u*/dt + beta F) of the annular cells, with block partials of its sum
__global__ void k_axi_rhs(const double* __restrict__ ur, const double* __restrict__ uz,
                          const double* __restrict__ Fr, const double* __restrict__ Fz,
                          const double* __restrict__ br, const double* __restrict__ bz, int nr,
                          int nz, double h, double inv_dt, double* __restrict__ b,
                          double* __restrict__ part) {
    __shared__ double sh[kBlock];
    const long N = (long)nr * nz;
    const double inv_h = 1.0 / h;
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        const int i = (int)(c % nr), k = (int)(c / nr);
        const double wr_lo = i == 0 ? 0.0 : ur[c] * inv_dt + br[c] * Fr[c];
        const double wr_hi = i + 1 == nr ? 0.0 : ur[c + 1] * inv_dt + br[c + 1] * Fr[c + 1];
        const long cz = k + 1 == nz ? c - (long)(nz - 1) * nr : c + nr;
        const double wz_lo = uz[c] * inv_dt + bz[c] * Fz[c];
        const double wz_hi = uz[cz] * inv_dt + bz[cz] * Fz[cz];
        const double ri = (double)i * h, rip = ri + h, rc = ((double)i + 0.5) * h;
        const double v = (rip * wr_hi - ri * wr_lo) * inv_h + rc * (wz_hi - wz_lo) * inv_h;
        b[c] = v;
        acc += v;
    }
    const double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_axi_sub_mean(double* __restrict__ b, long N, const double* __restrict__ sum) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) b[c] -= *sum / (double)N;
}

__global__ void k_axi_zero_axis(double* __restrict__ ur, int nr, int nz) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nz) ur[(long)k * nr] = 0.0;
}

}  // namespace ib

using namespace ib;

struct ib_axi {
    ib_ctx* full = nullptr;   // doubled plane, 2 nr x nz
    ib_ctx* half = nullptr;   // half plane, nr x nz
    int nr = 0, nz = 0;
    double h = 0.0;
    double* ud[2] = {nullptr, nullptr};   // mirrored velocity
    double* wb[2] = {nullptr, nullptr};   // r-weighted coefficients
    double* red = nullptr;                // partials + sum
};

static void free_axi(ib_axi* a) {
    if (!a) return;
    if (a->full) ib_destroy(a->full);
    if (a->half) ib_destroy(a->half);
    for (double* p : {a->ud[0], a->ud[1], a->wb[0], a->wb[1], a->red})
        if (p) hipFree(p);
    delete a;
}

extern "C" int ib_axi_create(const ib_grid* g, int max_markers, ib_axi** out) {
    IB_CHECK(g && out, IB_EINVAL, "ib_axi_create: null argument");
    IB_CHECK(g->dim == 2, IB_EINVAL, "ib_axi_create: the meridian plane is 2D (dim = 2)");
    ib_axi* a = new ib_axi();
    a->nr = g->n[0];
    a->nz = g->n[1];
    a->h = g->h;
    ib_grid gf = *g;
    gf.n[0] = 2 * g->n[0];
    int rc = ib_create(g, max_markers, 0, &a->half);
    if (rc == IB_OK) rc = ib_create(&gf, max_markers, 0, &a->full);
    if (rc != IB_OK) {
        free_axi(a);
        return rc;
    }
    const size_t half = sizeof(double) * (size_t)a->nr * a->nz;
    bool ok = true;
    for (int q = 0; q < 2; ++q) {
        ok = ok && hipMalloc((void**)&a->ud[q], 2 * half) == hipSuccess;
        ok = ok && hipMalloc((void**)&a->wb[q], half) == hipSuccess;
    }
    ok = ok && hipMalloc((void**)&a->red, sizeof(double) * (kAxiRed + 1)) == hipSuccess;
    if (!ok) {
        free_axi(a);
        return fail(IB_ENOMEM, "ib_axi_create: out of memory");
    }
    *out = a;
    return IB_OK;
}

extern "C" void ib_axi_destroy(ib_axi* a) { free_axi(a); }

extern "C" int axi_project_step(ib_axi* a, mg_handle* m, const ib_params* prm, ib_state* stt,
                                ib_outputs* out, void* stream) {
    IB_CHECK(a && m && prm && stt && out, IB_EINVAL, "axi_project_step: null argument");
    IB_CHECK(out->p && out->U && out->u[0] && out->u[1], IB_EINVAL,
             "axi_project_step: p, u and U outputs are required");
    IB_CHECK(stt->u_star[0] && stt->u_star[1] && stt->X_host, IB_EINVAL,
             "axi_project_step: u_star and X_host are required");
    IB_CHECK(prm->dt > 0 && prm->rho_in > 0 && prm->rho_out > 0, IB_EINVAL,
             "axi_project_step: dt and densities must be positive");
    IB_CHECK(prm->spread_mode == IB_SPREAD_IRROT, IB_EINVAL,
             "axi_project_step: only the irrotational spreading is provided");
    IB_CHECK(prm->warm_start == WS_ZERO || prm->warm_start == WS_PREV, IB_EINVAL,
             "axi_project_step: warm start must be WS_ZERO or WS_PREV");
    hipStream_t st = (hipStream_t)stream;
    Ctx* F = a->full;
    Ctx* Hc = a->half;
    const int nr = a->nr, nz = a->nz;
    const long N = (long)nr * nz;
    ib_surface s = stt->surf;
    const int n = s.n_markers;
    IB_CHECK(n >= 3 && n <= F->max_markers, IB_EINVAL, "axi_project_step: marker count");
    IB_HIP(hipMemcpyAsync(F->mX, stt->X_host, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
    s.X = F->mX;
    s.elems = nullptr;
    s.n_elems = 0;
    // marker velocities from the mirrored field, advance and relocation with
    // the azimuthal curvature added
    hipLaunchKernelGGL(k_axi_mirror, dim3(grid_for(2 * N)), dim3(kBlock), 0, st, stt->u_star[0],
                       stt->u_star[1], nr, nz, a->ud[0], a->ud[1]);
    const double* udc[3] = {a->ud[0], a->ud[1], a->ud[1]};
    IB_TRY(launch_interp(F, udc, &s, out->U, st));
    IB_TRY(relocate_2d(F, prm, stt, out->U, out->fs_host, &s, st, (double)nr * a->h));
    // H and the face force on the doubled plane, right half copied out
    double* Ff[3] = {F->F[0], F->F[1], F->F[1]};
    IB_TRY(spread_impl(F, &s, IB_SPREAD_IRROT, Ff, F->H, st));
    const size_t row = sizeof(double) * nr, frow = 2 * row;
    double* H = out->H ? out->H : Hc->H;
    double* Fh[2] = {out->F[0] ? out->F[0] : Hc->F[0], out->F[1] ? out->F[1] : Hc->F[1]};
    IB_HIP(hipMemcpy2DAsync(H, row, F->H + nr, frow, row, nz, hipMemcpyDeviceToDevice, st));
    for (int q = 0; q < 2; ++q)
        IB_HIP(hipMemcpy2DAsync(Fh[q], row, F->F[q] + nr, frow, row, nz, hipMemcpyDeviceToDevice, st));
    // coefficients, axis column, r weights, hierarchy
    IB_TRY(launch_coefficients(Hc, H, prm->rho_in, prm->rho_out, Hc->beta, Hc->rho, st));
    hipLaunchKernelGGL(k_axi_prepare, dim3(grid_for(N)), dim3(kBlock), 0, st, Hc->beta[0], Hc->beta[1],
                       Fh[0], nr, N, a->h, a->wb[0], a->wb[1]);
    const double* wb[3] = {a->wb[0], a->wb[1], a->wb[1]};
    IB_TRY(mg_update_coeffs(m, wb, st));
    // right side
    const int nb = (int)std::min<long>(kAxiRed, (long)grid_for(N));
    hipLaunchKernelGGL(k_axi_rhs, dim3(nb), dim3(kBlock), 0, st, stt->u_star[0], stt->u_star[1], Fh[0],
                       Fh[1], Hc->beta[0], Hc->beta[1], nr, nz, a->h, 1.0 / prm->dt, Hc->b, a->red);
    IB_TRY(device_sum(a->red, nb, a->red + kAxiRed, st));
    hipLaunchKernelGGL(k_axi_sub_mean, dim3(grid_for(N)), dim3(kBlock), 0, st, Hc->b, N, a->red + kAxiRed);
    if (out->b) IB_HIP(hipMemcpyAsync(out->b, Hc->b, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    // warm start and solve
    if (prm->warm_start == WS_PREV && stt->p_prev) {
        if (stt->p_prev != out->p)
            IB_HIP(hipMemcpyAsync(out->p, stt->p_prev, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    } else {
        IB_HIP(hipMemsetAsync(out->p, 0, sizeof(double) * N, st));
    }
    int rc = mg_solve(m, Hc->b, out->p, prm->rtol, prm->max_cycles, prm->fixed_cycles, &out->stats, st);
    if (rc != IB_OK && rc != IB_ENOTCONV) return rc;
    // update (beta_r and F_r vanish on the axis column), u_r = 0 there
    const double* us[3] = {stt->u_star[0], stt->u_star[1], stt->u_star[1]};
    const double* Fc[3] = {Fh[0], Fh[1], Fh[1]};
    const double* bc[3] = {Hc->beta[0], Hc->beta[1], Hc->beta[1]};
    double* un[3] = {out->u[0], out->u[1], out->u[1]};
    IB_TRY(launch_update(Hc, us, Fc, bc, out->p, prm->dt, un, st));
    hipLaunchKernelGGL(k_axi_zero_axis, dim3(grid_for(nz)), dim3(kBlock), 0, st, out->u[0], nr, nz);
    IB_HIP(hipGetLastError());
    return rc;
}
