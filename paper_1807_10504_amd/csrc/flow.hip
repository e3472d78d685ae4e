// Momentum predictor (Section 2.1, eq ns1_new): Adams-Bashforth advection in
// the flux form of eq ad_bf, Crank-Nicolson viscous stress of eq cr_ni, the
// implicit system solved by red-black Gauss-Seidel on the faces; and the
// full 2D step that runs it between the marker update and the projection.
//
// One thread per cell handles the faces of every component at that cell
// (face d of cell c is its low side along d). The stencil reaches one cell
// along each axis and, for the edge means, one more along d; periodic
// neighbours are formed once per thread.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "surface_gpu.h"

namespace ib {

constexpr int kFlowRed = 1024;  // reduction blocks

template <int DIM>
struct Sten {
    int ii[3], jj[3], kk[3];
    int nx, ny;
    __device__ Sten(const Dims& d, int i, int j, int k) : nx(d.nx), ny(d.ny) {
        ii[0] = wrap_near(i - 1, d.nx);
        ii[1] = i;
        ii[2] = wrap_near(i + 1, d.nx);
        jj[0] = wrap_near(j - 1, d.ny);
        jj[1] = j;
        jj[2] = wrap_near(j + 1, d.ny);
        if (DIM == 3) {
            kk[0] = wrap_near(k - 1, d.nz);
            kk[1] = k;
            kk[2] = wrap_near(k + 1, d.nz);
        } else {
            kk[0] = kk[1] = kk[2] = 0;
        }
    }
    // index of c + s e_a + t e_b (each offset component stays in -1..1)
    __device__ long at(int a, int s, int b = 0, int t = 0) const {
        int o[3] = {0, 0, 0};
        o[a] += s;
        o[b] += t;
        return ((long)kk[o[2] + 1] * ny + jj[o[1] + 1]) * nx + ii[o[0] + 1];
    }
};

template <int DIM>
__device__ __forceinline__ Sten<DIM> sten_of(const Dims& d, long c) {
    int i = (int)(c % d.nx);
    long r = c / d.nx;
    int j = (int)(r % d.ny);
    int k = (int)(r / d.ny);
    return Sten<DIM>(d, i, j, k);
}

// surface sum of u u . ds over the control volume of the d-face of cell c
// (eq ad_bf without the density), over h^(DIM-1); C_d is the face density
// times this over h (eq ns_1 has rho outside the divergence)
template <int DIM>
__device__ double adv_flux_sum(const Sten<DIM>& S, long c, const double* const* u, int d) {
    const double* ud = u[d];
    const long cmd = S.at(d, -1);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        if (e == d) {
            const double up = 0.5 * (ud[S.at(d, 1)] + ud[c]);
            const double um = 0.5 * (ud[c] + ud[cmd]);
            acc += up * up - um * um;
        } else {
            const double* ue = u[e];
            const long cp = S.at(e, 1), cpd = S.at(e, 1, d, -1);
            const long cm = S.at(e, -1), cmm = S.at(e, -1, d, -1);
            const double vep = 0.5 * (ue[cp] + ue[cpd]);
            const double udp = 0.5 * (ud[c] + ud[cp]);
            const double vem = 0.5 * (ue[c] + ue[cmd]);
            const double udm = 0.5 * (ud[c] + ud[cm]);
            acc += vep * udp - vem * udm;
        }
    }
    return acc;
}

// viscosities on the high (mp) and low (mm) side of the face of cell c along
// each axis: the cells c, c - e_d along d, the 4-cell edge means across
template <int DIM>
__device__ void visc_coefs(const Sten<DIM>& S, long c, const double* __restrict__ mu, int d,
                           double* mp, double* mm) {
    const long cmd = S.at(d, -1);
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        if (e == d) {
            mp[e] = mu[c];
            mm[e] = mu[cmd];
        } else {
            const double base = mu[c] + mu[cmd];
            mp[e] = 0.25 * ((base + mu[S.at(e, 1)]) + mu[S.at(e, 1, d, -1)]);
            mm[e] = 0.25 * ((base + mu[S.at(e, -1)]) + mu[S.at(e, -1, d, -1)]);
        }
    }
}

// D_d at the face of cell c (eq cr_ni), times h^2
template <int DIM>
__device__ double visc_sum(const Sten<DIM>& S, long c, const double* __restrict__ ud,
                           const double* mp, const double* mm) {
    const double uc = ud[c];
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e)
        acc += mp[e] * (ud[S.at(e, 1)] - uc) - mm[e] * (uc - ud[S.at(e, -1)]);
    return acc;
}

struct Vec3 {
    const double* p[3];
};
struct Out3 {
    double* p[3];
};

template <int DIM>
__global__ void k_advection(Vec3 u, const double* __restrict__ rho, Dims d, Out3 A) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    const Sten<DIM> S = sten_of<DIM>(d, c);
    const double inv_h = 1.0 / d.h;
#pragma unroll
    for (int q = 0; q < DIM; ++q)
        A.p[q][c] = 0.5 * (rho[c] + rho[S.at(q, -1)]) * adv_flux_sum<DIM>(S, c, u.p, q) * inv_h;
}

template <int DIM>
__global__ void k_viscous(Vec3 u, const double* __restrict__ mu, Dims d, Out3 V) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    const Sten<DIM> S = sten_of<DIM>(d, c);
    const double inv_h2 = 1.0 / (d.h * d.h);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        double mp[3], mm[3];
        visc_coefs<DIM>(S, c, mu, q, mp, mm);
        V.p[q][c] = visc_sum<DIM>(S, c, u.p[q], mp, mm) * inv_h2;
    }
}

// right side of the implicit system and the advection history:
//   A = C(u^n);  g = rho_f/dt u^n - (A or 3/2 A - 1/2 A_prev) + D u^n / 2
// (+ the body force on the y faces when body_on)
template <int DIM>
__global__ void k_pred_rhs(Vec3 u, const double* __restrict__ rho_n,
                           const double* __restrict__ rho1, const double* __restrict__ mu,
                           Vec3 Aprev, int first, Dims d, double inv_dt, Out3 A, Out3 g, Body B,
                           int body_on) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    const Sten<DIM> S = sten_of<DIM>(d, c);
    const double inv_h = 1.0 / d.h, inv_h2 = inv_h * inv_h;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        const double a = 0.5 * (rho_n[c] + rho_n[S.at(q, -1)]) * adv_flux_sum<DIM>(S, c, u.p, q) * inv_h;
        A.p[q][c] = a;
        const double ab = first ? a : 1.5 * a - 0.5 * Aprev.p[q][c];
        double mp[3], mm[3];
        visc_coefs<DIM>(S, c, mu, q, mp, mm);
        const double vis = visc_sum<DIM>(S, c, u.p[q], mp, mm) * inv_h2;
        const double rf = 0.5 * (rho1[c] + rho1[S.at(q, -1)]);
        double gv = rf * inv_dt * u.p[q][c] - ab + 0.5 * vis;
        if (q == 1 && body_on) gv += B.at(rf);
        g.p[q][c] = gv;
    }
}

// block partials of sum rho (weighted: sum rho (i + 1/2) h, i the column of
// an nr-wide plane)
__global__ void k_density_sum(const double* __restrict__ rho, long N, int nr, double h, int weighted,
                              double* __restrict__ part) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x)
        acc += weighted ? rho[c] * (((double)(c % nr) + 0.5) * h) : rho[c];
    const double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// one colour of a Gauss-Seidel sweep of (rho_f/dt - D/2) x = g, every component
template <int DIM>
__global__ void k_helm_sweep(Out3 x, Vec3 g, const double* __restrict__ rho1,
                             const double* __restrict__ mu, Dims d, double inv_dt, int colour) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int hx = d.nx >> 1;
    if (t >= d.cells() / 2) return;
    const long r = t / hx;
    const int j = (int)(r % d.ny), k = (int)(r / d.ny);
    const int i = 2 * (int)(t - r * hx) + ((j + k + colour) & 1);
    const long c = r * d.nx + i;
    const Sten<DIM> S(d, i, j, k);
    const double half_h2 = 0.5 / (d.h * d.h);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        double mp[3], mm[3];
        visc_coefs<DIM>(S, c, mu, q, mp, mm);
        const double rf = 0.5 * (rho1[c] + rho1[S.at(q, -1)]);
        double sdiag = 0.0, nb = 0.0;
        const double* xq = x.p[q];
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            sdiag += mp[e] + mm[e];
            nb += mp[e] * xq[S.at(e, 1)] + mm[e] * xq[S.at(e, -1)];
        }
        x.p[q][c] = (g.p[q][c] + half_h2 * nb) / (rf * inv_dt + half_h2 * sdiag);
    }
}

// block partials of ||g - M x||^2 and ||g||^2
template <int DIM>
__global__ void k_helm_resid(Vec3 x, Vec3 g, const double* __restrict__ rho1,
                             const double* __restrict__ mu, Dims d, double inv_dt,
                             double* __restrict__ part) {
    __shared__ double sh[kBlock];
    const long N = d.cells();
    const double inv_h2 = 1.0 / (d.h * d.h);
    double rr = 0.0, gg = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        const Sten<DIM> S = sten_of<DIM>(d, c);
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
            double mp[3], mm[3];
            visc_coefs<DIM>(S, c, mu, q, mp, mm);
            const double rf = 0.5 * (rho1[c] + rho1[S.at(q, -1)]);
            const double Mx = rf * inv_dt * x.p[q][c] - 0.5 * visc_sum<DIM>(S, c, x.p[q], mp, mm) * inv_h2;
            const double gv = g.p[q][c];
            rr += (gv - Mx) * (gv - Mx);
            gg += gv * gv;
        }
    }
    double s = block_reduce_sum(rr, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    s = block_reduce_sum(gg, sh);
    if (threadIdx.x == 0) part[kFlowRed + blockIdx.x] = s;
}

static Vec3 vec3(const double* const a[3], int dim) {
    Vec3 v{{a[0], a[1], dim == 3 ? a[2] : a[1]}};
    return v;
}
static Out3 out3(double* const a[3], int dim) {
    Out3 v{{a[0], a[1], dim == 3 ? a[2] : a[1]}};
    return v;
}

}  // namespace ib

using namespace ib;

struct ib_flow {
    Dims d;
    double* adv[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int cur = 0;          // adv[cur] receives C(u^n); adv[cur ^ 1] holds C(u^{n-1})
    int have_adv = 0;
    double* g[3] = {nullptr, nullptr, nullptr};
    double* ustar[3] = {nullptr, nullptr, nullptr};
    double* Hn = nullptr;     // H of the previous step (flow_step)
    double* rho_n = nullptr;
    double* mu = nullptr;
    int have_H = 0;
    int last_sweeps = 0;      // sweeps of the previous predictor call
    double* red = nullptr;    // 2 * kFlowRed partials + 2 sums
    double* host = nullptr;   // pinned: the two sums
    double* mred = nullptr;   // density-sum partials (kMeanParts) + the sum
    FreeFall ff;
    ib_indicator* ind = nullptr;  // conventional scheme: indicator of eq ind_psn
    SurfMesh mesh;                // 3D: the moving surface's connectivity on the device
    double* prop = nullptr;       // the indicator field of the step
};

static void free_flow(ib_flow* f) {
    if (!f) return;
    for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 3; ++q)
            if (f->adv[b][q]) hipFree(f->adv[b][q]);
    for (int q = 0; q < 3; ++q) {
        if (f->g[q]) hipFree(f->g[q]);
        if (f->ustar[q]) hipFree(f->ustar[q]);
    }
    for (double* p : {f->Hn, f->rho_n, f->mu, f->red, f->mred, f->prop})
        if (p) hipFree(p);
    if (f->ind) ib_indicator_destroy(f->ind);
    f->mesh.release();
    if (f->host) hipHostFree(f->host);
    delete f;
}

extern "C" int ib_flow_create(const ib_grid* g, ib_flow** out) {
    IB_CHECK(g && out, IB_EINVAL, "ib_flow_create: null argument");
    IB_CHECK(g->dim == 2 || g->dim == 3, IB_EINVAL, "ib_flow_create: dim must be 2 or 3");
    IB_CHECK(g->h > 0.0, IB_EINVAL, "ib_flow_create: h must be positive");
    long cells = 1;
    for (int e = 0; e < g->dim; ++e) {
        IB_CHECK(g->n[e] >= 4 && g->n[e] % 2 == 0, IB_EINVAL,
                 "ib_flow_create: cells per axis must be even and >= 4");
        cells *= g->n[e];
    }
    IB_CHECK(cells < (1L << 31), IB_EINVAL, "ib_flow_create: grid too large");
    ib_flow* f = new ib_flow();
    f->d = make_dims(*g);
    const size_t bytes = sizeof(double) * (size_t)cells;
    bool ok = true;
    auto alloc = [&](double** p, size_t b) {
        if (ok && hipMalloc((void**)p, b) != hipSuccess) ok = false;
    };
    for (int q = 0; q < g->dim; ++q) {
        alloc(&f->adv[0][q], bytes);
        alloc(&f->adv[1][q], bytes);
        alloc(&f->g[q], bytes);
        alloc(&f->ustar[q], bytes);
    }
    alloc(&f->Hn, bytes);
    alloc(&f->rho_n, bytes);
    alloc(&f->mu, bytes);
    alloc(&f->red, sizeof(double) * (2 * kFlowRed + 2));
    alloc(&f->mred, sizeof(double) * (kMeanParts + 1));
    if (ok && hipHostMalloc((void**)&f->host, 2 * sizeof(double)) != hipSuccess) ok = false;
    if (!ok) {
        free_flow(f);
        return fail(IB_ENOMEM, "ib_flow_create: out of memory");
    }
    *out = f;
    return IB_OK;
}

extern "C" void ib_flow_destroy(ib_flow* f) { free_flow(f); }

extern "C" int ib_flow_reset(ib_flow* f) {
    IB_CHECK(f, IB_EINVAL, "ib_flow_reset: null handle");
    f->have_adv = 0;
    f->have_H = 0;
    f->last_sweeps = 0;
    f->ff = FreeFall();
    return IB_OK;
}

extern "C" int ib_advection(ib_ctx* ctx, const double* const u[3], const double* rho,
                            double* const A[3], void* stream) {
    IB_CHECK(ctx && u && rho && A, IB_EINVAL, "ib_advection: null argument");
    Ctx* c = ctx;
    const int dim = c->d.dim;
    for (int q = 0; q < dim; ++q) IB_CHECK(u[q] && A[q], IB_EINVAL, "ib_advection: null array");
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(grid_for(c->d.cells())), blk(kBlock);
    if (dim == 2)
        hipLaunchKernelGGL(k_advection<2>, grid, blk, 0, st, vec3(u, 2), rho, c->d, out3(A, 2));
    else
        hipLaunchKernelGGL(k_advection<3>, grid, blk, 0, st, vec3(u, 3), rho, c->d, out3(A, 3));
    IB_HIP(hipGetLastError());
    return IB_OK;
}

extern "C" int ib_viscous(ib_ctx* ctx, const double* const u[3], const double* mu,
                          double* const V[3], void* stream) {
    IB_CHECK(ctx && u && mu && V, IB_EINVAL, "ib_viscous: null argument");
    Ctx* c = ctx;
    const int dim = c->d.dim;
    for (int q = 0; q < dim; ++q) IB_CHECK(u[q] && V[q], IB_EINVAL, "ib_viscous: null array");
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(grid_for(c->d.cells())), blk(kBlock);
    if (dim == 2)
        hipLaunchKernelGGL(k_viscous<2>, grid, blk, 0, st, vec3(u, 2), mu, c->d, out3(V, 2));
    else
        hipLaunchKernelGGL(k_viscous<3>, grid, blk, 0, st, vec3(u, 3), mu, c->d, out3(V, 3));
    IB_HIP(hipGetLastError());
    return IB_OK;
}

namespace ib {

int density_sum(const double* rho, long N, int nr, double h, int weighted, double* part, double* out,
                hipStream_t st) {
    const int nb = (int)std::min<long>(kMeanParts, (long)grid_for(N));
    hipLaunchKernelGGL(k_density_sum, dim3(nb), dim3(kBlock), 0, st, rho, N, nr, h, weighted, part);
    IB_HIP(hipGetLastError());
    return device_sum(part, nb, out, st);
}

int check_freefall(const ib_flow_params* fp, const char* who) {
    IB_CHECK(std::isfinite(fp->gravity) && std::isfinite(fp->c1) && std::isfinite(fp->c2) &&
                 (fp->frame == 0 || fp->frame == 1) && fp->mass_every >= 0 &&
                 std::isfinite(fp->mass_target),
             IB_EINVAL, std::string(who) + ": gravity, frame, c1, c2, mass_every, mass_target");
    return IB_OK;
}

}  // namespace ib

static int predict_impl(ib_flow* f, const double* const u[3], const double* rho_n,
                        const double* rho1, const double* mu, double dt, double rtol,
                        int max_sweeps, double* const ustar[3], ib_flow_stats* S, const Body& B,
                        hipStream_t st) {
    const Dims& d = f->d;
    const int dim = d.dim;
    const long N = d.cells();
    const double inv_dt = 1.0 / dt;
    const int first = f->have_adv ? 0 : 1;
    double* Acur[3] = {f->adv[f->cur][0], f->adv[f->cur][1], f->adv[f->cur][2]};
    const double* Aprev[3] = {f->adv[f->cur ^ 1][0], f->adv[f->cur ^ 1][1], f->adv[f->cur ^ 1][2]};
    const dim3 g1(grid_for(N)), gh(grid_for(N / 2)), blk(kBlock);
    const int nb = (int)std::min<long>(kFlowRed, (long)grid_for(N));
    for (int q = 0; q < dim; ++q)
        IB_HIP(hipMemcpyAsync(ustar[q], u[q], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    if (dim == 2)
        hipLaunchKernelGGL(k_pred_rhs<2>, g1, blk, 0, st, vec3(u, 2), rho_n, rho1, mu, vec3(Aprev, 2),
                           first, d, inv_dt, out3(Acur, 2), out3(f->g, 2), B, B.on() ? 1 : 0);
    else
        hipLaunchKernelGGL(k_pred_rhs<3>, g1, blk, 0, st, vec3(u, 3), rho_n, rho1, mu, vec3(Aprev, 3),
                           first, d, inv_dt, out3(Acur, 3), out3(f->g, 3), B, B.on() ? 1 : 0);
    IB_HIP(hipGetLastError());
    // the history advances whatever the solve does
    f->cur ^= 1;
    f->have_adv = 1;
    const double* gc[3] = {f->g[0], f->g[1], f->g[2]};
    int sweeps = 0;
    double rel = 0.0;
    S->first_step = first;
    S->checks = 0;
    while (true) {
        for (int colour = 0; colour < 2; ++colour) {
            if (dim == 2)
                hipLaunchKernelGGL(k_helm_sweep<2>, gh, blk, 0, st, out3(ustar, 2), vec3(gc, 2), rho1, mu,
                                   d, inv_dt, colour);
            else
                hipLaunchKernelGGL(k_helm_sweep<3>, gh, blk, 0, st, out3(ustar, 3), vec3(gc, 3), rho1, mu,
                                   d, inv_dt, colour);
        }
        ++sweeps;
        // the residual is read from one sweep before the previous call's count on
        if (sweeps < f->last_sweeps - 1 && sweeps < max_sweeps) continue;
        ++S->checks;
        const double* xc[3] = {ustar[0], ustar[1], ustar[2]};
        if (dim == 2)
            hipLaunchKernelGGL(k_helm_resid<2>, dim3(nb), blk, 0, st, vec3(xc, 2), vec3(gc, 2), rho1, mu, d,
                               inv_dt, f->red);
        else
            hipLaunchKernelGGL(k_helm_resid<3>, dim3(nb), blk, 0, st, vec3(xc, 3), vec3(gc, 3), rho1, mu, d,
                               inv_dt, f->red);
        IB_TRY(device_sum(f->red, nb, f->red + 2 * kFlowRed, st));
        IB_TRY(device_sum(f->red + kFlowRed, nb, f->red + 2 * kFlowRed + 1, st));
        IB_HIP(hipMemcpyAsync(f->host, f->red + 2 * kFlowRed, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        IB_HIP(hipStreamSynchronize(st));
        const double rr = f->host[0], gg = f->host[1];
        if (!std::isfinite(rr) || !std::isfinite(gg)) {
            S->sweeps = sweeps;
            S->rel_res = rr;
            return fail(IB_ENAN, "ib_predict: residual is not finite");
        }
        if (gg == 0.0) {
            // g = 0: the (nonsingular) system has the solution 0
            for (int q = 0; q < dim; ++q) IB_HIP(hipMemsetAsync(ustar[q], 0, sizeof(double) * N, st));
            rel = 0.0;
            break;
        }
        rel = std::sqrt(rr / gg);
        if (rel <= rtol) break;
        if (sweeps >= max_sweeps) {
            S->sweeps = sweeps;
            S->rel_res = rel;
            return fail(IB_ENOTCONV, "ib_predict: the implicit viscous system did not converge");
        }
    }
    S->sweeps = sweeps;
    S->rel_res = rel;
    f->last_sweeps = sweeps;
    return IB_OK;
}

extern "C" int ib_predict(ib_flow* f, const double* const u[3], const double* rho_n,
                          const double* rho_np1, const double* mu, double dt, double rtol,
                          int max_sweeps, double* const u_star[3], ib_flow_stats* stats,
                          void* stream) {
    IB_CHECK(f && u && rho_n && rho_np1 && mu && u_star, IB_EINVAL, "ib_predict: null argument");
    IB_CHECK(dt > 0 && rtol > 0 && max_sweeps > 0, IB_EINVAL, "ib_predict: dt, rtol, max_sweeps");
    for (int q = 0; q < f->d.dim; ++q) {
        IB_CHECK(u[q] && u_star[q], IB_EINVAL, "ib_predict: null velocity array");
        IB_CHECK(u[q] != u_star[q], IB_EINVAL, "ib_predict: u_star may not alias u");
    }
    ib_flow_stats loc{};
    const Body none{0.0, 0.0, 0.0, nullptr};
    return predict_impl(f, u, rho_n, rho_np1, mu, dt, rtol, max_sweeps, u_star, stats ? stats : &loc, none,
                        (hipStream_t)stream);
}

// 3D: the vertices advanced by dt U and moved onto the local least-squares
// surface on the device (its normals, curvature force and areas into the
// context's marker buffers); the host copy of the vertices follows
static int relocate_3d(ib_flow* f, Ctx* c, const ib_params* prm, ib_state* stt, const double* U_dev,
                       double* fs_host, ib_surface* s, hipStream_t st) {
    const int n = s->n_markers;
    IB_TRY(f->mesh.prepare(n, s->n_elems, stt->elems_host));
    IB_TRY(f->mesh.reconstruct(c->mX, U_dev, prm->dt, prm->sigma, c->mX, c->mfs, c->mds, c->mnrm, st));
    IB_HIP(hipMemcpyAsync(stt->X_host, c->mX, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, st));
    if (fs_host) IB_HIP(hipMemcpyAsync(fs_host, c->mfs, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    s->X = c->mX;
    s->fs = c->mfs;
    s->ds = c->mds;
    s->nrm = c->mnrm;
    return IB_OK;
}

extern "C" int flow_step(ib_ctx* ctx, ib_flow* f, mg_handle* m, const ib_params* prm,
                         const ib_flow_params* fp, ib_state* stt, ib_outputs* out,
                         ib_flow_stats* fstats, void* stream) {
    IB_CHECK(ctx && f && m && prm && fp && stt && out, IB_EINVAL, "flow_step: null argument");
    Ctx* c = ctx;
    const int dim = c->d.dim;
    IB_CHECK(f->d.nx == c->d.nx && f->d.ny == c->d.ny && f->d.nz == c->d.nz && f->d.dim == dim &&
                 f->d.h == c->d.h,
             IB_EINVAL, "flow_step: the flow handle belongs to another grid");
    IB_CHECK(out->p && out->U, IB_EINVAL, "flow_step: p and U outputs are required");
    for (int q = 0; q < dim; ++q)
        IB_CHECK(stt->u_star[q] && out->u[q], IB_EINVAL, "flow_step: null velocity array");
    IB_CHECK(prm->dt > 0 && prm->rho_in > 0 && prm->rho_out > 0, IB_EINVAL,
             "flow_step: dt and densities must be positive");
    IB_CHECK(fp->mu_in >= 0 && fp->mu_out >= 0 && fp->rtol > 0 && fp->max_sweeps > 0, IB_EINVAL,
             "flow_step: viscosities, rtol, max_sweeps");
    IB_TRY(check_freefall(fp, "flow_step"));
    IB_CHECK(fp->indicator_density == 0 ||
                 (fp->indicator_density == 1 && prm->spread_mode == IB_SPREAD_DELTA && dim == 2),
             IB_EINVAL, "flow_step: the indicator density goes with the conventional spreading in 2D");
    IB_CHECK(prm->warm_start == WS_ZERO || prm->warm_start == WS_PREV, IB_EINVAL,
             "flow_step: warm start must be WS_ZERO or WS_PREV");
    IB_CHECK(prm->spread_mode == IB_SPREAD_IRROT || prm->spread_mode == IB_SPREAD_DELTA, IB_EINVAL,
             "flow_step: spread mode");
    IB_CHECK(stt->X_host, IB_EINVAL, "flow_step: X_host is required");
    hipStream_t st = (hipStream_t)stream;
    ib_surface s = stt->surf;
    const int n = s.n_markers;
    if (dim == 3) {
        IB_CHECK(n >= 4 && n <= c->max_markers, IB_EINVAL, "flow_step: vertex count");
        IB_CHECK(s.n_elems >= 4 && s.n_elems <= c->max_elems && s.elems && stt->elems_host, IB_EINVAL,
                 "flow_step: 3D needs the triangles (device surf.elems and elems_host)");
    } else {
        IB_CHECK(n >= 3 && n <= c->max_markers, IB_EINVAL, "flow_step: marker count");
        s.elems = nullptr;
        s.n_elems = 0;
    }
    const long N = c->d.cells();
    IB_HIP(hipMemcpyAsync(c->mX, stt->X_host, sizeof(double) * dim * n, hipMemcpyHostToDevice, st));
    s.X = c->mX;
    // H of the incoming markers when there is no previous step (3D: offsets
    // along the normals of the incoming surface's reconstruction)
    if (!f->have_H) {
        if (dim == 3) {
            std::vector<double> Vt(3 * (size_t)n), fs(n), ds(n), nr(3 * (size_t)n);
            IB_TRY(ib_surface_lsq_3d(n, stt->X_host, s.n_elems, stt->elems_host, prm->sigma, Vt.data(), fs.data(),
                                     ds.data(), nr.data()));
            IB_HIP(hipMemcpyAsync(c->mnrm, nr.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
            IB_HIP(hipStreamSynchronize(st));
            s.nrm = c->mnrm;
        }
        IB_TRY(launch_heaviside(c, &s, f->Hn, st));
        int fl[3];
        IB_TRY(read_flags(c, fl, st));
        IB_CHECK(fl[0] == 0, IB_EGEOM, "flow_step: an offset surface comes within 4h of the box sides");
        f->have_H = 1;
    }
    // free fall: centroid and measure of the incoming markers (3D: the mesh)
    ib_flow_stats loc{};
    ib_flow_stats* FS = fstats ? fstats : &loc;
    const double* mass_target = nullptr;
    IB_CHECK(freefall_begin(&f->ff, fp, n, stt->X_host, NAN, prm->dt, FS, &mass_target, dim == 3 ? s.n_elems : 0,
                            dim == 3 ? stt->elems_host : nullptr) == IB_OK,
             IB_EGEOM, "flow_step: the markers enclose no area / volume");
    // markers: interpolation of u^n, advance, relocation (and mass correction)
    IB_TRY(launch_interp(c, stt->u_star, &s, out->U, st));
    if (dim == 2)
        IB_TRY(relocate_2d(c, prm, stt, out->U, out->fs_host, &s, st, NAN, mass_target, &FS->mass_delta));
    else {
        IB_TRY(relocate_3d(f, c, prm, stt, out->U, out->fs_host, &s, st));
        if (mass_target) {
            // the fitted vertices along their fitted normals, on the host
            std::vector<double> nh(3 * (size_t)n);
            IB_HIP(hipMemcpy(nh.data(), c->mnrm, sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
            IB_TRY(ib_mesh_mass_correct(n, stt->X_host, nh.data(), s.n_elems, stt->elems_host, *mass_target, c->d.h,
                                        1e-6, 1e-12, &FS->mass_delta));
            IB_HIP(hipMemcpyAsync(c->mX, stt->X_host, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
            IB_HIP(hipStreamSynchronize(st));
        }
    }
    // H^{n+1} and the face force
    double* H = out->H ? out->H : c->H;
    double* F[3];
    for (int e = 0; e < 3; ++e) F[e] = (out->F[e] && e < dim) ? out->F[e] : c->F[e];
    IB_TRY(spread_impl(c, &s, prm->spread_mode, F, H, st));
    // the field the properties follow: H, or the conventional indicator
    const double* P = H;
    if (fp->indicator_density) {
        if (!f->ind) IB_TRY(ib_indicator_create(&c->g, c->max_markers, &f->ind));
        if (!f->prop) IB_HIP(hipMalloc((void**)&f->prop, sizeof(double) * N));
        const int rci = ib_indicator_solve(ctx, f->ind, &s, prm->rtol, 100, f->prop, nullptr, st);
        if (rci != IB_OK) return rci;
        P = f->prop;
    }
    // rho^n, mu^{n+1}; rho^{n+1} and beta with the hierarchy
    IB_TRY(launch_coefficients(c, f->Hn, prm->rho_in, prm->rho_out, nullptr, f->rho_n, st));
    IB_TRY(launch_coefficients(c, P, fp->mu_in, fp->mu_out, nullptr, f->mu, st));
    IB_TRY(coefficients_and_hierarchy(c, m, prm, P, st));
    // predictor, with the body force (rho_mean: volume mean of rho^{n+1})
    Body B{fp->gravity, FS->frame_a, 1.0 / (double)N, nullptr};
    if (fp->gravity != 0.0) {
        IB_TRY(density_sum(c->rho, N, c->d.nx, c->d.h, 0, f->mred, f->mred + kMeanParts, st));
        B.rsum = f->mred + kMeanParts;
    }
    IB_TRY(predict_impl(f, stt->u_star, f->rho_n, c->rho, f->mu, prm->dt, fp->rtol, fp->max_sweeps,
                        f->ustar, FS, B, st));
    // projection of u*
    const double* us[3] = {f->ustar[0], f->ustar[1], dim == 3 ? f->ustar[2] : f->ustar[1]};
    int rc = solve_and_update(c, m, prm, stt, out, us, H, F, st);
    if (rc != IB_OK && rc != IB_ENOTCONV) return rc;
    IB_HIP(hipMemcpyAsync(f->Hn, P, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    return rc;
}
