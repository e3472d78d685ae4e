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

// ---------------------------------------------------------------------------
// momentum predictor on the meridian plane (annular control volumes; u_r on
// face column 0 is zero and is neither read as an unknown nor written)
struct AxiIdx {
    int i, k, nr, nz;
    long c;
    __device__ AxiIdx(long c_, int nr_, int nz_) : nr(nr_), nz(nz_), c(c_) {
        i = (int)(c % nr);
        k = (int)(c / nr);
    }
    // cell (i + di, k + dk): r wraps periodically (the callers never use the
    // wrapped value except where it multiplies zero), z is periodic
    __device__ long at(int di, int dk) const {
        int ii = i + di, kk = k + dk;
        ii = ii < 0 ? ii + nr : (ii >= nr ? ii - nr : ii);
        kk = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);
        return (long)kk * nr + ii;
    }
};

// u_z u_r on the top edge of the u_r face (i, k + dk): cells i-1, i at k+dk, k+dk+1
__device__ __forceinline__ double axi_ftop(const AxiIdx& X, int dk, const double* ur, const double* uz) {
    const double uze = 0.5 * (uz[X.at(0, dk + 1)] + uz[X.at(-1, dk + 1)]);
    const double ure = 0.5 * (ur[X.at(0, dk)] + ur[X.at(0, dk + 1)]);
    return uze * ure;
}

// r_{i+1+di} u_r u_z on the right edge of the u_z face (i + di, k)
__device__ __forceinline__ double axi_fright(const AxiIdx& X, int di, double h, const double* ur,
                                             const double* uz) {
    const double ure = 0.5 * (ur[X.at(di + 1, 0)] + ur[X.at(di + 1, -1)]);
    const double uze = 0.5 * (uz[X.at(di, 0)] + uz[X.at(di + 1, 0)]);
    return ((double)(X.i + di + 1) * h) * ure * uze;
}

// C_r and C_z: the face density times the annular surface sum of u u . ds
// over the control volume (the density outside the divergence, as in the
// planar predictor)
__device__ double axi_adv_r(const AxiIdx& X, double h, const double* ur, const double* uz,
                            const double* rho) {
    const double ri = (double)X.i * h;
    const double u0 = 0.5 * (ur[X.c] + ur[X.at(1, 0)]);
    const double um = 0.5 * (ur[X.at(-1, 0)] + ur[X.c]);
    const double fc = (((double)X.i + 0.5) * h) * u0 * u0;
    const double fm = (((double)X.i - 0.5) * h) * um * um;
    const double radial = (fc - fm) / ri;
    const double rf = 0.5 * (rho[X.c] + rho[X.at(-1, 0)]);
    return rf * (radial + (axi_ftop(X, 0, ur, uz) - axi_ftop(X, -1, ur, uz))) / h;
}

__device__ double axi_adv_z(const AxiIdx& X, double h, const double* ur, const double* uz,
                            const double* rho) {
    const double rc = ((double)X.i + 0.5) * h;
    const double fr = axi_fright(X, 0, h, ur, uz);
    const double fl = X.i > 0 ? axi_fright(X, -1, h, ur, uz) : 0.0;
    const double c0 = 0.5 * (uz[X.c] + uz[X.at(0, 1)]);
    const double cm = 0.5 * (uz[X.at(0, -1)] + uz[X.c]);
    const double fz = c0 * c0 - cm * cm;
    const double rf = 0.5 * (rho[X.c] + rho[X.at(0, -1)]);
    return rf * ((fr - fl) / rc + fz) / h;
}

// viscous coefficients: D x = c[1] (x_r+ - x) - c[0] (x - x_r-) + c[3] (x_z+ - x)
//                              - c[2] (x - x_z-) - c[4] x
__device__ void axi_visc_r(const AxiIdx& X, double h, const double* mu, double* c) {
    const double h2 = h * h, ri = (double)X.i * h;
    const double mi = mu[X.c], mm = mu[X.at(-1, 0)];
    c[1] = (((double)X.i + 0.5) * h) * mi / (ri * h2);
    c[0] = (((double)X.i - 0.5) * h) * mm / (ri * h2);
    const double et = 0.25 * (((mi + mm) + mu[X.at(0, 1)]) + mu[X.at(-1, 1)]);
    const double eb = 0.25 * (((mu[X.at(0, -1)] + mu[X.at(-1, -1)]) + mi) + mm);
    c[3] = et / h2;
    c[2] = eb / h2;
    c[4] = (0.5 * (mi + mm)) / (ri * ri);
}

__device__ void axi_visc_z(const AxiIdx& X, double h, const double* mu, double* c) {
    const double h2 = h * h, rc = ((double)X.i + 0.5) * h;
    const double mi = mu[X.c];
    if (X.i + 1 < X.nr) {
        const double er = 0.25 * (((mi + mu[X.at(1, 0)]) + mu[X.at(0, -1)]) + mu[X.at(1, -1)]);
        c[1] = ((double)(X.i + 1) * h) * er / (rc * h2);
    } else {
        c[1] = 0.0;
    }
    if (X.i > 0) {
        const double el = 0.25 * (((mu[X.at(-1, 0)] + mi) + mu[X.at(-1, -1)]) + mu[X.at(0, -1)]);
        c[0] = ((double)X.i * h) * el / (rc * h2);
    } else {
        c[0] = 0.0;
    }
    c[3] = mi / h2;
    c[2] = mu[X.at(0, -1)] / h2;
    c[4] = 0.0;
}

__device__ __forceinline__ double axi_apply(const AxiIdx& X, const double* x, const double* c) {
    const double v = x[X.c];
    return c[1] * (x[X.at(1, 0)] - v) - c[0] * (v - x[X.at(-1, 0)]) + c[3] * (x[X.at(0, 1)] - v) -
           c[2] * (v - x[X.at(0, -1)]) - c[4] * v;
}

__global__ void k_axi_pred_rhs(const double* __restrict__ ur, const double* __restrict__ uz,
                               const double* __restrict__ rho_n, const double* __restrict__ rho1,
                               const double* __restrict__ mu, const double* __restrict__ Ar_prev,
                               const double* __restrict__ Az_prev, int first, int nr, int nz, double h,
                               double inv_dt, double* __restrict__ Ar, double* __restrict__ Az,
                               double* __restrict__ gr, double* __restrict__ gz, Body B, int body_on) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (long)nr * nz) return;
    const AxiIdx X(c, nr, nz);
    double co[5];
    if (X.i > 0) {
        const double a = axi_adv_r(X, h, ur, uz, rho_n);
        Ar[c] = a;
        const double ab = first ? a : 1.5 * a - 0.5 * Ar_prev[c];
        axi_visc_r(X, h, mu, co);
        const double rf = 0.5 * (rho1[c] + rho1[X.at(-1, 0)]);
        gr[c] = rf * inv_dt * ur[c] - ab + 0.5 * axi_apply(X, ur, co);
    } else {
        Ar[c] = 0.0;
        gr[c] = 0.0;
    }
    const double a = axi_adv_z(X, h, ur, uz, rho_n);
    Az[c] = a;
    const double ab = first ? a : 1.5 * a - 0.5 * Az_prev[c];
    axi_visc_z(X, h, mu, co);
    const double rf = 0.5 * (rho1[c] + rho1[X.at(0, -1)]);
    double gv = rf * inv_dt * uz[c] - ab + 0.5 * axi_apply(X, uz, co);
    if (body_on) gv += B.at(rf);
    gz[c] = gv;
}

__global__ void k_axi_helm_sweep(double* __restrict__ xr, double* __restrict__ xz,
                                 const double* __restrict__ gr, const double* __restrict__ gz,
                                 const double* __restrict__ rho1, const double* __restrict__ mu, int nr,
                                 int nz, double h, double inv_dt, int colour) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int hr = nr >> 1;
    if (t >= (long)hr * nz) return;
    const int k = (int)(t / hr);
    const int i = 2 * (int)(t - (long)k * hr) + ((k + colour) & 1);
    const AxiIdx X((long)k * nr + i, nr, nz);
    double co[5];
    if (i > 0) {
        axi_visc_r(X, h, mu, co);
        const double rf = 0.5 * (rho1[X.c] + rho1[X.at(-1, 0)]);
        const double nb = co[1] * xr[X.at(1, 0)] + co[0] * xr[X.at(-1, 0)] + co[3] * xr[X.at(0, 1)] +
                          co[2] * xr[X.at(0, -1)];
        const double dg = ((co[1] + co[0]) + (co[3] + co[2])) + co[4];
        xr[X.c] = (gr[X.c] + 0.5 * nb) / (rf * inv_dt + 0.5 * dg);
    }
    axi_visc_z(X, h, mu, co);
    const double rf = 0.5 * (rho1[X.c] + rho1[X.at(0, -1)]);
    const double nb = co[1] * xz[X.at(1, 0)] + co[0] * xz[X.at(-1, 0)] + co[3] * xz[X.at(0, 1)] +
                      co[2] * xz[X.at(0, -1)];
    const double dg = ((co[1] + co[0]) + (co[3] + co[2])) + co[4];
    xz[X.c] = (gz[X.c] + 0.5 * nb) / (rf * inv_dt + 0.5 * dg);
}

__global__ void k_axi_helm_resid(const double* __restrict__ xr, const double* __restrict__ xz,
                                 const double* __restrict__ gr, const double* __restrict__ gz,
                                 const double* __restrict__ rho1, const double* __restrict__ mu, int nr,
                                 int nz, double h, double inv_dt, double* __restrict__ part) {
    __shared__ double sh[kBlock];
    const long N = (long)nr * nz;
    double rr = 0.0, gg = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        const AxiIdx X(c, nr, nz);
        double co[5];
        if (X.i > 0) {
            axi_visc_r(X, h, mu, co);
            const double rf = 0.5 * (rho1[c] + rho1[X.at(-1, 0)]);
            const double r = gr[c] - (rf * inv_dt * xr[c] - 0.5 * axi_apply(X, xr, co));
            rr += r * r;
            gg += gr[c] * gr[c];
        }
        axi_visc_z(X, h, mu, co);
        const double rf = 0.5 * (rho1[c] + rho1[X.at(0, -1)]);
        const double r = gz[c] - (rf * inv_dt * xz[c] - 0.5 * axi_apply(X, xz, co));
        rr += r * r;
        gg += gz[c] * gz[c];
    }
    double s = block_reduce_sum(rr, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    s = block_reduce_sum(gg, sh);
    if (threadIdx.x == 0) part[kAxiRed + blockIdx.x] = s;
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
    double* red = nullptr;                // partials (2 kAxiRed) + sums (2)
    double* host = nullptr;               // pinned: two sums
    // predictor state (axi_predict, axi_flow_step)
    double* adv[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int cur = 0, have_adv = 0, have_H = 0;
    int last_sweeps = 0;                  // sweeps of the previous predictor call
    double* g[2] = {nullptr, nullptr};
    double* ustar[2] = {nullptr, nullptr};
    double* Hn = nullptr;
    double* rho_n = nullptr;
    double* mu = nullptr;
    double* mred = nullptr;   // density-sum partials (kMeanParts) + the sum
    FreeFall ff;
};

static void free_axi(ib_axi* a) {
    if (!a) return;
    if (a->full) ib_destroy(a->full);
    if (a->half) ib_destroy(a->half);
    for (double* p : {a->ud[0], a->ud[1], a->wb[0], a->wb[1], a->red, a->adv[0][0], a->adv[0][1],
                      a->adv[1][0], a->adv[1][1], a->g[0], a->g[1], a->ustar[0], a->ustar[1], a->Hn,
                      a->rho_n, a->mu, a->mred})
        if (p) hipFree(p);
    if (a->host) hipHostFree(a->host);
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
        ok = ok && hipMalloc((void**)&a->adv[0][q], half) == hipSuccess;
        ok = ok && hipMalloc((void**)&a->adv[1][q], half) == hipSuccess;
        ok = ok && hipMalloc((void**)&a->g[q], half) == hipSuccess;
        ok = ok && hipMalloc((void**)&a->ustar[q], half) == hipSuccess;
    }
    for (double** p : {&a->Hn, &a->rho_n, &a->mu}) ok = ok && hipMalloc((void**)p, half) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->red, sizeof(double) * (2 * kAxiRed + 2)) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->mred, sizeof(double) * (kMeanParts + 1)) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&a->host, 2 * sizeof(double)) == hipSuccess;
    if (!ok) {
        free_axi(a);
        return fail(IB_ENOMEM, "ib_axi_create: out of memory");
    }
    *out = a;
    return IB_OK;
}

extern "C" void ib_axi_destroy(ib_axi* a) { free_axi(a); }

// coefficients of level n+1 (rho, beta with the axis column zeroed), the face
// force's axis column zeroed, r-weighted coefficients into the hierarchy
static int axi_coefficients(ib_axi* a, mg_handle* m, const ib_params* prm, const double* H,
                            double* Fr, hipStream_t st) {
    Ctx* Hc = a->half;
    const long N = (long)a->nr * a->nz;
    IB_TRY(launch_coefficients(Hc, H, prm->rho_in, prm->rho_out, Hc->beta, Hc->rho, st));
    hipLaunchKernelGGL(k_axi_prepare, dim3(grid_for(N)), dim3(kBlock), 0, st, Hc->beta[0], Hc->beta[1],
                       Fr, a->nr, N, a->h, a->wb[0], a->wb[1]);
    const double* wb[3] = {a->wb[0], a->wb[1], a->wb[1]};
    IB_TRY(mg_update_coeffs(m, wb, st));
    return IB_OK;
}

// right side from u_star and F, warm start, solve, update, u_r = 0 on the axis column
static int axi_solve_update(ib_axi* a, mg_handle* m, const ib_params* prm, ib_state* stt,
                            ib_outputs* out, const double* const us[2], double* const Fh[2],
                            const double* H, hipStream_t st) {
    Ctx* Hc = a->half;
    const int nr = a->nr, nz = a->nz;
    const long N = (long)nr * nz;
    const int nb = (int)std::min<long>(kAxiRed, (long)grid_for(N));
    hipLaunchKernelGGL(k_axi_rhs, dim3(nb), dim3(kBlock), 0, st, us[0], us[1], Fh[0], Fh[1], Hc->beta[0],
                       Hc->beta[1], nr, nz, a->h, 1.0 / prm->dt, Hc->b, a->red);
    IB_TRY(device_sum(a->red, nb, a->red + 2 * kAxiRed, st));
    hipLaunchKernelGGL(k_axi_sub_mean, dim3(grid_for(N)), dim3(kBlock), 0, st, Hc->b, N,
                       a->red + 2 * kAxiRed);
    if (out->b) IB_HIP(hipMemcpyAsync(out->b, Hc->b, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    out->guess_accepted = 0;
    out->guess_rel_res = out->prev_rel_res = 0.0;
    out->guess_energy = out->prev_energy = 0.0;
    if (prm->warm_start == WS_NN) {
        // the network sees the r-weighted right side of the meridian plane
        IB_TRY(nn_warm_start(m, stt, out, prm->rho_in, prm->rho_out, Hc->b, H, N, st));
    } else if (prm->warm_start == WS_PREV && stt->p_prev) {
        if (stt->p_prev != out->p)
            IB_HIP(hipMemcpyAsync(out->p, stt->p_prev, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    } else {
        IB_HIP(hipMemsetAsync(out->p, 0, sizeof(double) * N, st));
        mg_hint_zero_guess(m);
    }
    int rc = mg_solve(m, Hc->b, out->p, prm->rtol, prm->max_cycles, prm->fixed_cycles, &out->stats, st);
    if (rc != IB_OK && rc != IB_ENOTCONV) return rc;
    const double* u3[3] = {us[0], us[1], us[1]};
    const double* Fc[3] = {Fh[0], Fh[1], Fh[1]};
    const double* bc[3] = {Hc->beta[0], Hc->beta[1], Hc->beta[1]};
    double* un[3] = {out->u[0], out->u[1], out->u[1]};
    IB_TRY(launch_update(Hc, u3, Fc, bc, out->p, prm->dt, un, st));
    hipLaunchKernelGGL(k_axi_zero_axis, dim3(grid_for(nz)), dim3(kBlock), 0, st, out->u[0], nr, nz);
    IB_HIP(hipGetLastError());
    return rc;
}

// markers of stt->X_host to the device, mirrored velocity interpolated to
// them, advance and relocation with the azimuthal curvature, H and F of the
// doubled plane copied to the half plane (H, Fh)
static int axi_interface(ib_axi* a, const ib_params* prm, ib_state* stt, ib_outputs* out,
                         ib_surface* s, double* H, double* const Fh[2], hipStream_t st,
                         const double* mass_target = nullptr, double* mass_delta = nullptr) {
    Ctx* F = a->full;
    const int nr = a->nr, nz = a->nz;
    const long N = (long)nr * nz;
    hipLaunchKernelGGL(k_axi_mirror, dim3(grid_for(2 * N)), dim3(kBlock), 0, st, stt->u_star[0],
                       stt->u_star[1], nr, nz, a->ud[0], a->ud[1]);
    const double* udc[3] = {a->ud[0], a->ud[1], a->ud[1]};
    IB_TRY(launch_interp(F, udc, s, out->U, st));
    IB_TRY(relocate_2d(F, prm, stt, out->U, out->fs_host, s, st, (double)nr * a->h, mass_target, mass_delta));
    double* Ff[3] = {F->F[0], F->F[1], F->F[1]};
    // irrotational, or the conventional delta-function spreading of fs ds n on the
    // doubled plane (an axisymmetric surface's delta restricted to the meridian
    // plane is the curve's delta); H is formed either way
    IB_TRY(spread_impl(F, s, prm->spread_mode, Ff, F->H, st));
    const size_t row = sizeof(double) * nr, frow = 2 * row;
    IB_HIP(hipMemcpy2DAsync(H, row, F->H + nr, frow, row, nz, hipMemcpyDeviceToDevice, st));
    for (int q = 0; q < 2; ++q)
        IB_HIP(hipMemcpy2DAsync(Fh[q], row, F->F[q] + nr, frow, row, nz, hipMemcpyDeviceToDevice, st));
    return IB_OK;
}

static int axi_check(ib_axi* a, mg_handle* m, const ib_params* prm, ib_state* stt, ib_outputs* out,
                     const char* who) {
    IB_CHECK(a && m && prm && stt && out, IB_EINVAL, std::string(who) + ": null argument");
    IB_CHECK(out->p && out->U && out->u[0] && out->u[1], IB_EINVAL,
             std::string(who) + ": p, u and U outputs are required");
    IB_CHECK(stt->u_star[0] && stt->u_star[1] && stt->X_host, IB_EINVAL,
             std::string(who) + ": u_star and X_host are required");
    IB_CHECK(prm->dt > 0 && prm->rho_in > 0 && prm->rho_out > 0, IB_EINVAL,
             std::string(who) + ": dt and densities must be positive");
    IB_CHECK(prm->spread_mode == IB_SPREAD_IRROT || prm->spread_mode == IB_SPREAD_DELTA, IB_EINVAL,
             std::string(who) + ": spread mode");
    IB_CHECK(prm->warm_start == WS_ZERO || prm->warm_start == WS_PREV ||
                 (prm->warm_start == WS_NN && stt->nn),
             IB_EINVAL, std::string(who) + ": warm start must be WS_ZERO, WS_PREV or WS_NN with a network");
    IB_CHECK(stt->surf.n_markers >= 3 && stt->surf.n_markers <= a->full->max_markers, IB_EINVAL,
             std::string(who) + ": marker count");
    return IB_OK;
}

extern "C" int axi_project_step(ib_axi* a, mg_handle* m, const ib_params* prm, ib_state* stt,
                                ib_outputs* out, void* stream) {
    IB_TRY(axi_check(a, m, prm, stt, out, "axi_project_step"));
    hipStream_t st = (hipStream_t)stream;
    Ctx* F = a->full;
    Ctx* Hc = a->half;
    ib_surface s = stt->surf;
    const int n = s.n_markers;
    IB_HIP(hipMemcpyAsync(F->mX, stt->X_host, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
    s.X = F->mX;
    s.elems = nullptr;
    s.n_elems = 0;
    double* H = out->H ? out->H : Hc->H;
    double* Fh[2] = {out->F[0] ? out->F[0] : Hc->F[0], out->F[1] ? out->F[1] : Hc->F[1]};
    IB_TRY(axi_interface(a, prm, stt, out, &s, H, Fh, st));
    IB_TRY(axi_coefficients(a, m, prm, H, Fh[0], st));
    const double* us[2] = {stt->u_star[0], stt->u_star[1]};
    return axi_solve_update(a, m, prm, stt, out, us, Fh, H, st);
}

static int axi_predict_impl(ib_axi* a, const double* const u[2], const double* rho_n,
                            const double* rho1, const double* mu, double dt, double rtol, int max_sweeps,
                            double* const ustar[2], ib_flow_stats* S, const Body& B, hipStream_t st) {
    const int nr = a->nr, nz = a->nz;
    const long N = (long)nr * nz;
    const double inv_dt = 1.0 / dt, h = a->h;
    const int first = a->have_adv ? 0 : 1;
    double* Ac[2] = {a->adv[a->cur][0], a->adv[a->cur][1]};
    const double* Ap[2] = {a->adv[a->cur ^ 1][0], a->adv[a->cur ^ 1][1]};
    for (int q = 0; q < 2; ++q)
        IB_HIP(hipMemcpyAsync(ustar[q], u[q], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_axi_pred_rhs, dim3(grid_for(N)), dim3(kBlock), 0, st, u[0], u[1], rho_n, rho1, mu,
                       Ap[0], Ap[1], first, nr, nz, h, inv_dt, Ac[0], Ac[1], a->g[0], a->g[1], B,
                       B.on() ? 1 : 0);
    IB_HIP(hipGetLastError());
    a->cur ^= 1;
    a->have_adv = 1;
    hipLaunchKernelGGL(k_axi_zero_axis, dim3(grid_for(nz)), dim3(kBlock), 0, st, ustar[0], nr, nz);
    const int nb = (int)std::min<long>(kAxiRed, (long)grid_for(N));
    int sweeps = 0;
    double rel = 0.0;
    S->first_step = first;
    S->checks = 0;
    while (true) {
        for (int colour = 0; colour < 2; ++colour)
            hipLaunchKernelGGL(k_axi_helm_sweep, dim3(grid_for(N / 2)), dim3(kBlock), 0, st, ustar[0],
                               ustar[1], a->g[0], a->g[1], rho1, mu, nr, nz, h, inv_dt, colour);
        ++sweeps;
        // the residual is read from one sweep before the previous call's count on
        if (sweeps < a->last_sweeps - 1 && sweeps < max_sweeps) continue;
        ++S->checks;
        hipLaunchKernelGGL(k_axi_helm_resid, dim3(nb), dim3(kBlock), 0, st, ustar[0], ustar[1], a->g[0],
                           a->g[1], rho1, mu, nr, nz, h, inv_dt, a->red);
        IB_TRY(device_sum(a->red, nb, a->red + 2 * kAxiRed, st));
        IB_TRY(device_sum(a->red + kAxiRed, nb, a->red + 2 * kAxiRed + 1, st));
        IB_HIP(hipMemcpyAsync(a->host, a->red + 2 * kAxiRed, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        IB_HIP(hipStreamSynchronize(st));
        const double rr = a->host[0], gg = a->host[1];
        S->sweeps = sweeps;
        if (!std::isfinite(rr) || !std::isfinite(gg)) {
            S->rel_res = rr;
            return fail(IB_ENAN, "axi_predict: residual is not finite");
        }
        if (gg == 0.0) {
            for (int q = 0; q < 2; ++q) IB_HIP(hipMemsetAsync(ustar[q], 0, sizeof(double) * N, st));
            rel = 0.0;
            break;
        }
        rel = std::sqrt(rr / gg);
        S->rel_res = rel;
        if (rel <= rtol) break;
        if (sweeps >= max_sweeps)
            return fail(IB_ENOTCONV, "axi_predict: the implicit viscous system did not converge");
    }
    S->rel_res = rel;
    a->last_sweeps = sweeps;
    return IB_OK;
}

extern "C" int ib_axi_reset(ib_axi* a) {
    IB_CHECK(a, IB_EINVAL, "ib_axi_reset: null handle");
    a->have_adv = 0;
    a->have_H = 0;
    a->last_sweeps = 0;
    a->ff = FreeFall();
    return IB_OK;
}

extern "C" int axi_predict(ib_axi* a, const double* const u[2], const double* rho_n,
                           const double* rho_np1, const double* mu, double dt, double rtol, int max_sweeps,
                           double* const u_star[2], ib_flow_stats* stats, void* stream) {
    IB_CHECK(a && u && rho_n && rho_np1 && mu && u_star, IB_EINVAL, "axi_predict: null argument");
    IB_CHECK(dt > 0 && rtol > 0 && max_sweeps > 0, IB_EINVAL, "axi_predict: dt, rtol, max_sweeps");
    for (int q = 0; q < 2; ++q) {
        IB_CHECK(u[q] && u_star[q], IB_EINVAL, "axi_predict: null velocity array");
        IB_CHECK(u[q] != u_star[q], IB_EINVAL, "axi_predict: u_star may not alias u");
    }
    ib_flow_stats loc{};
    const Body none{0.0, 0.0, 0.0, nullptr};
    return axi_predict_impl(a, u, rho_n, rho_np1, mu, dt, rtol, max_sweeps, u_star, stats ? stats : &loc, none,
                            (hipStream_t)stream);
}

extern "C" int axi_flow_step(ib_axi* a, mg_handle* m, const ib_params* prm, const ib_flow_params* fp,
                             ib_state* stt, ib_outputs* out, ib_flow_stats* fstats, void* stream) {
    IB_TRY(axi_check(a, m, prm, stt, out, "axi_flow_step"));
    IB_CHECK(fp && fp->mu_in >= 0 && fp->mu_out >= 0 && fp->rtol > 0 && fp->max_sweeps > 0, IB_EINVAL,
             "axi_flow_step: viscosities, rtol, max_sweeps");
    IB_TRY(check_freefall(fp, "axi_flow_step"));
    IB_CHECK(fp->indicator_density == 0, IB_EINVAL, "axi_flow_step: the indicator density is planar only");
    hipStream_t st = (hipStream_t)stream;
    Ctx* F = a->full;
    Ctx* Hc = a->half;
    const int nr = a->nr, nz = a->nz;
    const long N = (long)nr * nz;
    ib_surface s = stt->surf;
    const int n = s.n_markers;
    IB_HIP(hipMemcpyAsync(F->mX, stt->X_host, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
    s.X = F->mX;
    s.elems = nullptr;
    s.n_elems = 0;
    const size_t row = sizeof(double) * nr, frow = 2 * row;
    if (!a->have_H) {
        IB_TRY(launch_heaviside(F, &s, F->H, st));
        int fl[3];
        IB_TRY(read_flags(F, fl, st));
        IB_CHECK(fl[0] == 0, IB_EGEOM, "axi_flow_step: an offset curve comes within 4h of the box sides");
        IB_HIP(hipMemcpy2DAsync(a->Hn, row, F->H + nr, frow, row, nz, hipMemcpyDeviceToDevice, st));
        a->have_H = 1;
    }
    double* H = out->H ? out->H : Hc->H;
    double* Fh[2] = {out->F[0] ? out->F[0] : Hc->F[0], out->F[1] ? out->F[1] : Hc->F[1]};
    ib_flow_stats loc{};
    ib_flow_stats* FS = fstats ? fstats : &loc;
    const double* mass_target = nullptr;
    const double axis_x = (double)nr * a->h;
    IB_CHECK(freefall_begin(&a->ff, fp, n, stt->X_host, axis_x, prm->dt, FS, &mass_target) == IB_OK, IB_EGEOM,
             "axi_flow_step: the markers enclose no volume");
    IB_TRY(axi_interface(a, prm, stt, out, &s, H, Fh, st, mass_target, &FS->mass_delta));
    IB_TRY(launch_coefficients(Hc, a->Hn, prm->rho_in, prm->rho_out, nullptr, a->rho_n, st));
    IB_TRY(launch_coefficients(Hc, H, fp->mu_in, fp->mu_out, nullptr, a->mu, st));
    IB_TRY(axi_coefficients(a, m, prm, H, Fh[0], st));
    // body force with rho_mean the r-weighted volume mean of rho^{n+1}
    // (sum over columns of (i + 1/2) h is h nr^2 / 2)
    Body B{fp->gravity, FS->frame_a, 1.0 / ((double)nz * (0.5 * a->h * (double)nr * (double)nr)), nullptr};
    if (fp->gravity != 0.0) {
        IB_TRY(density_sum(Hc->rho, N, nr, a->h, 1, a->mred, a->mred + kMeanParts, st));
        B.rsum = a->mred + kMeanParts;
    }
    const double* un[2] = {stt->u_star[0], stt->u_star[1]};
    IB_TRY(axi_predict_impl(a, un, a->rho_n, Hc->rho, a->mu, prm->dt, fp->rtol, fp->max_sweeps, a->ustar,
                            FS, B, st));
    const double* us[2] = {a->ustar[0], a->ustar[1]};
    int rc = axi_solve_update(a, m, prm, stt, out, us, Fh, H, st);
    if (rc != IB_OK && rc != IB_ENOTCONV) return rc;
    IB_HIP(hipMemcpyAsync(a->Hn, H, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    return rc;
}
