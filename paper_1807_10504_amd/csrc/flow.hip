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
    int i, j, k;
    cell_ijk(c, d.nx, d.ny, i, j, k);
    return Sten<DIM>(d, i, j, k);
}

// The stencils below read their fields through accessors, u(q, a, s, b, t)
// = component q at cell c + s e_a + t e_b (f(a, s, b, t) for one field), so
// the one-thread-per-cell kernels (global memory through Sten) and the
// tiled ones (LDS planes) share one arithmetic. Every product and sum is
// rounded on its own: the two forms agree bit for bit.
template <int DIM>
struct GlobVec {
    const Sten<DIM>& S;
    const double* const* u;
    __device__ double operator()(int q, int a, int s, int b = 0, int t = 0) const { return u[q][S.at(a, s, b, t)]; }
};
template <int DIM>
struct GlobField {
    const Sten<DIM>& S;
    const double* f;
    __device__ double operator()(int a, int s, int b = 0, int t = 0) const { return f[S.at(a, s, b, t)]; }
};
// one component of a vector accessor as a field accessor
template <class UA>
struct CompOf {
    const UA& u;
    int q;
    __device__ double operator()(int a, int s, int b = 0, int t = 0) const { return u(q, a, s, b, t); }
};

// surface sum of u u . ds over the control volume of the d-face of cell c
// (eq ad_bf without the density), over h^(DIM-1); C_d is the face density
// times this over h (eq ns_1 has rho outside the divergence)
template <int DIM, class UA>
__device__ __forceinline__ double adv_flux(const UA& u, int d) {
#pragma clang fp contract(off)
    const double udc = u(d, 0, 0), udmd = u(d, d, -1);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        if (e == d) {
            const double up = 0.5 * (u(d, d, 1) + udc);
            const double um = 0.5 * (udc + udmd);
            acc += up * up - um * um;
        } else {
            const double vep = 0.5 * (u(e, e, 1) + u(e, e, 1, d, -1));
            const double udp = 0.5 * (udc + u(d, e, 1));
            const double vem = 0.5 * (u(e, 0, 0) + u(e, d, -1));
            const double udm = 0.5 * (udc + u(d, e, -1));
            acc += vep * udp - vem * udm;
        }
    }
    return acc;
}

// viscosity on the edge shared by the faces of cells c and c + e (both of
// orientation d, e != d): the mean of the four cells around it, mc = mu[c],
// md = mu[c - e_d], ma = mu[c + e], mad = mu[c + e - e_d]
__device__ __forceinline__ double edge_mu(double mc, double md, double ma, double mad) {
#pragma clang fp contract(off)
    const double base = mc + md;
    return 0.25 * ((base + ma) + mad);
}

// viscosities on the high (mp) and low (mm) side of the face of cell c along
// each axis: the cells c, c - e_d along d, the 4-cell edge means across
template <int DIM, class FA>
__device__ __forceinline__ void visc_coefs_acc(const FA& mu, int d, double* mp, double* mm) {
    const double mc = mu(0, 0), md = mu(d, -1);
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        if (e == d) {
            mp[e] = mc;
            mm[e] = md;
        } else {
            mp[e] = edge_mu(mc, md, mu(e, 1), mu(e, 1, d, -1));
            mm[e] = edge_mu(mc, md, mu(e, -1), mu(e, -1, d, -1));
        }
    }
}

template <int DIM>
__device__ void visc_coefs(const Sten<DIM>& S, long c, const double* __restrict__ mu, int d,
                           double* mp, double* mm) {
    (void)c;
    visc_coefs_acc<DIM>(GlobField<DIM>{S, mu}, d, mp, mm);
}

// Gauss-Seidel value of one face of (rho_f/dt - D/2) x = g: xp / xm the
// neighbours along +e / -e, mp / mm their viscosities (visc_coefs). Every
// product and sum is rounded on its own, so the value does not depend on
// how the kernel around it lets the compiler fuse multiply-adds (the
// single-pass and the one-colour sweeps agree bit for bit).
template <int DIM>
__device__ __forceinline__ double helm_face(const double* mp, const double* mm, const double* xp,
                                            const double* xm, double gv, double rf, double inv_dt,
                                            double half_h2) {
#pragma clang fp contract(off)
    double sdiag = 0.0, nb = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        sdiag += mp[e] + mm[e];
        nb += mp[e] * xp[e] + mm[e] * xm[e];
    }
    return (gv + half_h2 * nb) / (rf * inv_dt + half_h2 * sdiag);
}

// (rho_f/dt - D/2) x at one face, x = xc, its neighbours xp / xm along +e /
// -e and their viscosities mp / mm (every product and sum rounded on its own)
template <int DIM>
__device__ __forceinline__ double helm_apply(const double* mp, const double* mm, const double* xp,
                                             const double* xm, double xc, double rf, double inv_dt,
                                             double inv_h2) {
#pragma clang fp contract(off)
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) acc += mp[e] * (xp[e] - xc) - mm[e] * (xc - xm[e]);
    return rf * inv_dt * xc - 0.5 * acc * inv_h2;
}

// the viscosities of visc_coefs and rho_f of face q of the cell at offset c
// of LDS planes laid out with row length RX: M* the viscosities of the plane
// (c), below (d) and above (u) it, Rc / Rd the densities of the plane and below
template <int RX>
__device__ __forceinline__ void lds_coefs(int q, int c, const double* Mc, const double* Md, const double* Mu,
                                          const double* Rc, const double* Rd, double* mp, double* mm,
                                          double& rf) {
    if (q == 0) {
        mp[0] = Mc[c];
        mm[0] = Mc[c - 1];
        mp[1] = edge_mu(Mc[c], Mc[c - 1], Mc[c + RX], Mc[c + RX - 1]);
        mm[1] = edge_mu(Mc[c], Mc[c - 1], Mc[c - RX], Mc[c - RX - 1]);
        mp[2] = edge_mu(Mc[c], Mc[c - 1], Mu[c], Mu[c - 1]);
        mm[2] = edge_mu(Mc[c], Mc[c - 1], Md[c], Md[c - 1]);
        rf = 0.5 * (Rc[c] + Rc[c - 1]);
    } else if (q == 1) {
        mp[0] = edge_mu(Mc[c], Mc[c - RX], Mc[c + 1], Mc[c + 1 - RX]);
        mm[0] = edge_mu(Mc[c], Mc[c - RX], Mc[c - 1], Mc[c - 1 - RX]);
        mp[1] = Mc[c];
        mm[1] = Mc[c - RX];
        mp[2] = edge_mu(Mc[c], Mc[c - RX], Mu[c], Mu[c - RX]);
        mm[2] = edge_mu(Mc[c], Mc[c - RX], Md[c], Md[c - RX]);
        rf = 0.5 * (Rc[c] + Rc[c - RX]);
    } else {
        mp[0] = edge_mu(Mc[c], Md[c], Mc[c + 1], Md[c + 1]);
        mm[0] = edge_mu(Mc[c], Md[c], Mc[c - 1], Md[c - 1]);
        mp[1] = edge_mu(Mc[c], Md[c], Mc[c + RX], Md[c + RX]);
        mm[1] = edge_mu(Mc[c], Md[c], Mc[c - RX], Md[c - RX]);
        mp[2] = Mc[c];
        mm[2] = Md[c];
        rf = 0.5 * (Rc[c] + Rd[c]);
    }
}

// D_d at the face of cell c (eq cr_ni), times h^2; ud the face values of component d
template <int DIM, class FA>
__device__ __forceinline__ double visc_sum_acc(const FA& ud, const double* mp, const double* mm) {
#pragma clang fp contract(off)
    const double uc = ud(0, 0);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) acc += mp[e] * (ud(e, 1) - uc) - mm[e] * (uc - ud(e, -1));
    return acc;
}

// the right side of the implicit system and the advection term at face q of
// one cell: A = C(u^n), g = rho_f/dt u^n - (A or 3/2 A - 1/2 A_prev) + D u^n / 2
// (+ the body force on the y faces); rn, r1 the densities of levels n, n + 1
template <int DIM, class UA, class FA, class RA>
__device__ __forceinline__ void pred_rhs_face(const UA& u, const FA& mu, const RA& rn, const RA& r1, int q,
                                              double aprev, int first, double inv_dt, double inv_h,
                                              double inv_h2, const Body& B, int body_on, double& a_out,
                                              double& g_out) {
#pragma clang fp contract(off)
    const double a = 0.5 * (rn(0, 0) + rn(q, -1)) * adv_flux<DIM>(u, q) * inv_h;
    a_out = a;
    const double ab = first ? a : 1.5 * a - 0.5 * aprev;
    double mp[3], mm[3];
    visc_coefs_acc<DIM>(mu, q, mp, mm);
    const double vis = visc_sum_acc<DIM>(CompOf<UA>{u, q}, mp, mm) * inv_h2;
    const double rf = 0.5 * (r1(0, 0) + r1(q, -1));
    double gv = rf * inv_dt * u(q, 0, 0) - ab + 0.5 * vis;
    if (q == 1 && body_on) gv += B.at(rf);
    g_out = gv;
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
    const GlobVec<DIM> U{S, u.p};
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
#pragma clang fp contract(off)
        A.p[q][c] = 0.5 * (rho[c] + rho[S.at(q, -1)]) * adv_flux<DIM>(U, q) * inv_h;
    }
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
        V.p[q][c] = visc_sum_acc<DIM>(GlobField<DIM>{S, u.p[q]}, mp, mm) * inv_h2;
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
    const GlobVec<DIM> U{S, u.p};
    const GlobField<DIM> M{S, mu}, Rn{S, rho_n}, R1{S, rho1};
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        double a, gv;
        pred_rhs_face<DIM>(U, M, Rn, R1, q, first ? 0.0 : Aprev.p[q][c], first, inv_dt, inv_h, inv_h2, B, body_on,
                           a, gv);
        A.p[q][c] = a;
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
        double mp[3], mm[3], xp[3], xm[3];
        visc_coefs<DIM>(S, c, mu, q, mp, mm);
        const double rf = 0.5 * (rho1[c] + rho1[S.at(q, -1)]);
        const double* xq = x.p[q];
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            xp[e] = xq[S.at(e, 1)];
            xm[e] = xq[S.at(e, -1)];
        }
        x.p[q][c] = helm_face<DIM>(mp, mm, xp, xm, g.p[q][c], rf, inv_dt, half_h2);
    }
}

// One full red-black sweep of the 3D system, every component, in a single
// pass (nx % 32 == 0, ny % 8 == 0, nz % TZ == 0 with TZ even). A workgroup
// owns a 32 x 8 column tile and the z-range [z0, z1) and marches upward: at
// plane step k it updates the red cells of plane k on the tile and a
// one-cell ring around it, then the black cells of plane k - 1 on the tile,
// and writes plane k - 1. Ring values are recomputed by the neighbouring
// tile from the same inputs, and x is double-buffered (read xin, write
// xout), so no workgroup reads what another writes during the sweep: red
// reads only old black values, black only new red values, as in the two
// one-colour launches of k_helm_sweep, whose per-face arithmetic (helm_face,
// edge_mu) it shares. The components' planes, mu and rho_f's densities are
// staged in LDS over the tile and a two-cell halo, loaded into registers
// two steps ahead; g at the lane's red and black cells goes into registers
// once the step has used the values before it.
constexpr int kHTX = 32, kHTY = 8;
constexpr int kHRX = kHTX + 4, kHRY = kHTY + 4, kHRN = kHRX * kHRY;
constexpr int kHLoads = (kHRN + kBlock - 1) / kBlock;
constexpr int kHRedRow = (kHRX - 2) / 2, kHRedN = kHRedRow * (kHRY - 2);
constexpr int kHBlackRow = kHTX / 2, kHBlackN = kHBlackRow * kHTY;

__device__ __forceinline__ int hmod3(int k) { return ((k % 3) + 3) % 3; }

__global__ __launch_bounds__(kBlock) void k_helm_fused(Vec3 xin, Out3 xout, Vec3 g,
                                                       const double* __restrict__ rho1,
                                                       const double* __restrict__ mu, Dims d, double inv_dt,
                                                       int TZ, int ntx, int nty, int nzc) {
    __shared__ double X[3][4][kHRN];
    __shared__ double M[4][kHRN];
    __shared__ double R[3][kHRN];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // range of tiles so that halo rows are shared in its L2
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * kHTX - 2, j0 = ty * kHTY - 2;
    const int z0 = zc * TZ, z1 = z0 + TZ;
    const long plane = (long)d.nx * d.ny;
    const double half_h2 = 0.5 / (d.h * d.h);
    const int t = threadIdx.x;
    // tile origins are at least -2 and regions end within one period
    auto gofs = [&](int x, int y) { return wrap_near(j0 + y, d.ny) * d.nx + wrap_near(i0 + x, d.nx); };
    // every lane issues every load (slots past the region re-read its first
    // cell and are not stored)
    int gp[kHLoads];
    bool vp[kHLoads];
#pragma unroll
    for (int s = 0; s < kHLoads; ++s) {
        const int q = t + s * kBlock;
        vp[s] = q < kHRN;
        gp[s] = vp[s] ? gofs(q % kHRX, q / kHRX) : gofs(0, 0);
    }
    // planes z0 - 2 .. z1 + 2 lie within one period of the box
    auto pl = [&](int k) { return (long)wrap_near(k, d.nz) * plane; };
    // the lane's red cell of plane k (region position; lanes past the red
    // cells take the first) and black cell of plane k - 1 (past the black
    // cells: the first); every lane updates at most one of each
    static_assert(kHRedN <= kBlock && kHBlackN <= kBlock, "one red and one black cell per lane");
    const bool has_red = t < kHRedN, has_black = t < kHBlackN;
    const int ry = 1 + (has_red ? t : 0) / kHRedRow, rm = (has_red ? t : 0) % kHRedRow;
    const int by = 2 + (has_black ? t : 0) / kHBlackRow, bm = (has_black ? t : 0) % kHBlackRow;
    auto red_x = [&](int k) { return 1 + ((i0 + 1 + j0 + ry + k) & 1) + 2 * rm; };
    auto black_par = [&](int kb) { return (i0 + 3 + j0 + by + kb) & 1; };
    // register stages, alternating: x and mu of plane k + 1, the densities
    // of plane k, g at the lane's red cell of plane k and black cell of plane k - 1
    struct Stage {
        double x[3][kHLoads], m[kHLoads], r[kHLoads], gr[3], gb[3];
    };
    Stage SA, SB;
    // planes at the step's commit, g after the step has used it: no value is
    // overwritten while its load is in flight
    auto fetch_planes = [&](Stage& S, int k) {
        const long bu = pl(k + 1), bk = pl(k);
#pragma unroll
        for (int s = 0; s < kHLoads; ++s) {
#pragma unroll
            for (int q = 0; q < 3; ++q) S.x[q][s] = xin.p[q][bu + gp[s]];
            S.m[s] = mu[bu + gp[s]];
            S.r[s] = rho1[bk + gp[s]];
        }
    };
    auto fetch_g = [&](Stage& S, int k) {
        const long gr = pl(k) + gofs(red_x(k), ry);
        const long gb = pl(k - 1) + gofs(2 + black_par(k - 1) + 2 * bm, by);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            S.gr[q] = g.p[q][gr];
            S.gb[q] = g.p[q][gb];
        }
    };
    auto commit = [&](const Stage& S, int k) {
#pragma unroll
        for (int s = 0; s < kHLoads; ++s)
            if (s * kBlock + kBlock <= kHRN || vp[s]) {
                const int c = t + s * kBlock;
#pragma unroll
                for (int q = 0; q < 3; ++q) X[q][(k + 1) & 3][c] = S.x[q][s];
                M[(k + 1) & 3][c] = S.m[s];
                R[hmod3(k)][c] = S.r[s];
            }
    };
    {
        const long a = pl(z0 - 2), a1 = pl(z0 - 1);
#pragma unroll
        for (int s = 0; s < kHLoads; ++s)
            if (vp[s]) {
                const int c = t + s * kBlock;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    X[q][(z0 - 2) & 3][c] = xin.p[q][a + gp[s]];
                    X[q][(z0 - 1) & 3][c] = xin.p[q][a1 + gp[s]];
                }
                M[(z0 - 2) & 3][c] = mu[a + gp[s]];
                M[(z0 - 1) & 3][c] = mu[a1 + gp[s]];
                R[hmod3(z0 - 2)][c] = rho1[a + gp[s]];
            }
    }
    fetch_planes(SA, z0 - 1);
    fetch_g(SA, z0 - 1);
    __builtin_amdgcn_sched_barrier(0);
    fetch_planes(SB, z0);
    fetch_g(SB, z0);
    // component q of the cell at region position (x, y) of plane kk
    auto update = [&](int q, int x, int y, int kk, double gv) {
        const int c = y * kHRX + x;
        const double* Xc = X[q][kk & 3];
        const double* Xd = X[q][(kk - 1) & 3];
        const double* Xu = X[q][(kk + 1) & 3];
        const double* Mc = M[kk & 3];
        const double* Md = M[(kk - 1) & 3];
        const double* Mu = M[(kk + 1) & 3];
        const double* Rc = R[hmod3(kk)];
        const double xp[3] = {Xc[c + 1], Xc[c + kHRX], Xu[c]};
        const double xm[3] = {Xc[c - 1], Xc[c - kHRX], Xd[c]};
        double mp[3], mm[3], rf;
        lds_coefs<kHRX>(q, c, Mc, Md, Mu, Rc, R[hmod3(kk - 1)], mp, mm, rf);
        return helm_face<3>(mp, mm, xp, xm, gv, rf, inv_dt, half_h2);
    };
    auto step = [&](Stage& S, int k) {
        commit(S, k);
        // in flight for two steps; past the range it re-reads plane z1 (not
        // committed), which keeps the loads unconditional
        const int kn = k + 2 <= z1 ? k + 2 : z1;
        fetch_planes(S, kn);
        __syncthreads();
        // red cells of plane k on the tile and its one-cell ring
        if (has_red) {
            const int x = red_x(k);
            double v[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) v[q] = update(q, x, ry, k, S.gr[q]);
#pragma unroll
            for (int q = 0; q < 3; ++q) X[q][k & 3][ry * kHRX + x] = v[q];
        }
        __syncthreads();
        const int kb = k - 1;
        if (kb >= z0 && kb < z1 && has_black) {
            // black cells of plane k - 1 on the tile, written with the red cell
            // beside them (the pair starts at an even x)
            const long base = pl(kb) + (long)(j0 + 2) * d.nx + (i0 + 2);
            const int par = black_par(kb);
            const int xb = 2 + par + 2 * bm;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double v = update(q, xb, by, kb, S.gb[q]);
                const double r = X[q][kb & 3][by * kHRX + 3 - par + 2 * bm];
                double2 w2;
                w2.x = par ? r : v;
                w2.y = par ? v : r;
                *reinterpret_cast<double2*>(xout.p[q] + base + (long)(by - 2) * d.nx + 2 * bm) = w2;
            }
        }
        fetch_g(S, kn);
        // the next commit overwrites the planes below k - 1
        __syncthreads();
    };
    // steps z0 - 1 .. z1 in pairs (stage A, stage B); TZ is even
    for (int k = z0 - 1; k <= z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
    }
}

// Block partials of ||g - M x||^2 and ||g||^2 on 3D grids of whole 32 x 8
// column tiles: a workgroup marches its tile over the z-range [z0, z1), one
// cell per lane and plane, with x, mu and the densities of the tile and a
// one-cell ring staged in LDS two steps ahead and g in registers. The
// per-face values are those of k_helm_resid (helm_apply, lds_coefs); the sums
// run in another order.
constexpr int kQRX = kHTX + 2, kQRY = 8 + 2, kQRN = kQRX * kQRY;
constexpr int kQLoads = (kQRN + kBlock - 1) / kBlock;

__global__ __launch_bounds__(kBlock) void k_helm_resid_tiled(Vec3 x, Vec3 g, const double* __restrict__ rho1,
                                                             const double* __restrict__ mu, Dims d, double inv_dt,
                                                             int TZ, int ntx, int nty, int nzc,
                                                             double* __restrict__ part) {
    static_assert(kHTX * 8 == kBlock, "one tile cell per lane");
    __shared__ double X[3][3][kQRN];
    __shared__ double M[3][kQRN];
    __shared__ double R[2][kQRN];
    __shared__ double sh[kBlock];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * kHTX - 1, j0 = ty * 8 - 1;
    const int z0 = zc * TZ, z1 = z0 + TZ;
    const long plane = (long)d.nx * d.ny;
    const double inv_h2 = 1.0 / (d.h * d.h);
    const int t = threadIdx.x;
    auto gofs = [&](int xx, int yy) { return wrap_near(j0 + yy, d.ny) * d.nx + wrap_near(i0 + xx, d.nx); };
    int gp[kQLoads];
    bool vp[kQLoads];
#pragma unroll
    for (int s = 0; s < kQLoads; ++s) {
        const int q = t + s * kBlock;
        vp[s] = q < kQRN;
        gp[s] = vp[s] ? gofs(q % kQRX, q / kQRX) : gofs(0, 0);
    }
    auto pl = [&](int k) { return (long)wrap_near(k, d.nz) * plane; };
    // the lane's cell: region position (cx, cy), its offset in the plane
    const int cx = 1 + t % kHTX, cy = 1 + t / kHTX, cc = cy * kQRX + cx;
    const int go = gofs(cx, cy);
    auto m3 = [](int k) { return ((k % 3) + 3) % 3; };
    // register stages, alternating: x and mu of plane k + 1, the densities and g of plane k
    struct Stage {
        double x[3][kQLoads], m[kQLoads], r[kQLoads], gv[3];
    };
    Stage SA, SB;
    auto fetch_planes = [&](Stage& S, int k) {
        const long bu = pl(k + 1), bk = pl(k);
#pragma unroll
        for (int s = 0; s < kQLoads; ++s) {
#pragma unroll
            for (int q = 0; q < 3; ++q) S.x[q][s] = x.p[q][bu + gp[s]];
            S.m[s] = mu[bu + gp[s]];
            S.r[s] = rho1[bk + gp[s]];
        }
    };
    auto fetch_g = [&](Stage& S, int k) {
        const long b = pl(k) + go;
#pragma unroll
        for (int q = 0; q < 3; ++q) S.gv[q] = g.p[q][b];
    };
    auto commit = [&](const Stage& S, int k) {
#pragma unroll
        for (int s = 0; s < kQLoads; ++s)
            if (s * kBlock + kBlock <= kQRN || vp[s]) {
                const int c = t + s * kBlock;
#pragma unroll
                for (int q = 0; q < 3; ++q) X[q][m3(k + 1)][c] = S.x[q][s];
                M[m3(k + 1)][c] = S.m[s];
                R[k & 1][c] = S.r[s];
            }
    };
    {
        const long a = pl(z0 - 1), a1 = pl(z0);
#pragma unroll
        for (int s = 0; s < kQLoads; ++s)
            if (vp[s]) {
                const int c = t + s * kBlock;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    X[q][m3(z0 - 1)][c] = x.p[q][a + gp[s]];
                    X[q][m3(z0)][c] = x.p[q][a1 + gp[s]];
                }
                M[m3(z0 - 1)][c] = mu[a + gp[s]];
                M[m3(z0)][c] = mu[a1 + gp[s]];
                R[(z0 - 1) & 1][c] = rho1[a + gp[s]];
            }
    }
    fetch_planes(SA, z0);
    fetch_g(SA, z0);
    __builtin_amdgcn_sched_barrier(0);
    fetch_planes(SB, z0 + 1);
    fetch_g(SB, z0 + 1);
    double rr = 0.0, gg = 0.0;
    auto step = [&](Stage& S, int k) {
        commit(S, k);
        const int kn = k + 2 < z1 ? k + 2 : z1 - 1;
        fetch_planes(S, kn);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* Xc = X[q][m3(k)];
            const double xp[3] = {Xc[cc + 1], Xc[cc + kQRX], X[q][m3(k + 1)][cc]};
            const double xm[3] = {Xc[cc - 1], Xc[cc - kQRX], X[q][m3(k - 1)][cc]};
            double mp[3], mm[3], rf;
            lds_coefs<kQRX>(q, cc, M[m3(k)], M[m3(k - 1)], M[m3(k + 1)], R[k & 1], R[(k - 1) & 1], mp, mm, rf);
            const double Mx = helm_apply<3>(mp, mm, xp, xm, Xc[cc], rf, inv_dt, inv_h2);
            const double gv = S.gv[q];
            rr += (gv - Mx) * (gv - Mx);
            gg += gv * gv;
        }
        fetch_g(S, kn);
        // the next commit overwrites the plane below k
        __syncthreads();
    };
    // steps z0 .. z1 - 1 in pairs (stage A, stage B); TZ is even
    for (int k = z0; k < z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
    }
    double s = block_reduce_sum(rr, sh);
    if (t == 0) part[bid] = s;
    s = block_reduce_sum(gg, sh);
    if (t == 0) part[kFlowRed + bid] = s;
}

// accessors of the tiled kernels: LDS planes with row length kQRX, the
// plane k + oz of a ring of NS planes
template <int NS>
__device__ __forceinline__ int ring_slot(int k) {
    return NS == 2 ? (k & 1) : ((k % NS) + NS) % NS;
}
__device__ __forceinline__ int lds_offset(int a, int s, int b, int t, int& oz) {
    oz = (a == 2 ? s : 0) + (b == 2 ? t : 0);
    return (a == 0 ? s : 0) + (b == 0 ? t : 0) + ((a == 1 ? s : 0) + (b == 1 ? t : 0)) * kQRX;
}
struct LdsVec {
    const double (*U)[3][kQRN];
    int k, cc;
    __device__ double operator()(int q, int a, int s, int b = 0, int t = 0) const {
        int oz;
        const int o = lds_offset(a, s, b, t, oz);
        return U[q][ring_slot<3>(k + oz)][cc + o];
    }
};
template <int NS>
struct LdsField {
    const double (*F)[kQRN];
    int k, cc;
    __device__ double operator()(int a, int s, int b = 0, int t = 0) const {
        int oz;
        const int o = lds_offset(a, s, b, t, oz);
        return F[ring_slot<NS>(k + oz)][cc + o];
    }
};

// The right side and advection term of the 3D predictor (k_pred_rhs) on
// grids of whole 32 x 8 column tiles: a workgroup marches its tile over the
// z-range [z0, z1), one cell per lane and plane, with u, mu and the two
// density levels of the tile and a one-cell ring staged in LDS two steps
// ahead and A_prev in registers. Same per-face arithmetic (pred_rhs_face),
// so the same values bit for bit.
__global__ __launch_bounds__(kBlock) void k_pred_rhs_tiled(Vec3 u, const double* __restrict__ rho_n,
                                                           const double* __restrict__ rho1,
                                                           const double* __restrict__ mu, Vec3 Aprev, int first,
                                                           Dims d, double inv_dt, Out3 A, Out3 g, Body B,
                                                           int body_on, int TZ, int ntx, int nty, int nzc) {
    static_assert(kHTX * 8 == kBlock, "one tile cell per lane");
    __shared__ double UU[3][3][kQRN];
    __shared__ double MM[3][kQRN];
    __shared__ double RN[2][kQRN];
    __shared__ double R1[2][kQRN];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * kHTX - 1, j0 = ty * 8 - 1;
    const int z0 = zc * TZ, z1 = z0 + TZ;
    const long plane = (long)d.nx * d.ny;
    const double inv_h = 1.0 / d.h, inv_h2 = inv_h * inv_h;
    const int t = threadIdx.x;
    auto gofs = [&](int xx, int yy) { return wrap_near(j0 + yy, d.ny) * d.nx + wrap_near(i0 + xx, d.nx); };
    int gp[kQLoads];
    bool vp[kQLoads];
#pragma unroll
    for (int s = 0; s < kQLoads; ++s) {
        const int q = t + s * kBlock;
        vp[s] = q < kQRN;
        gp[s] = vp[s] ? gofs(q % kQRX, q / kQRX) : gofs(0, 0);
    }
    auto pl = [&](int k) { return (long)wrap_near(k, d.nz) * plane; };
    const int cx = 1 + t % kHTX, cy = 1 + t / kHTX, cc = cy * kQRX + cx;
    const int go = gofs(cx, cy);
    // register stages, alternating: u and mu of plane k + 1, the densities
    // of plane k, A_prev at the lane's cell of plane k
    struct Stage {
        double u[3][kQLoads], m[kQLoads], rn[kQLoads], r1[kQLoads], ap[3];
    };
    Stage SA, SB;
    auto fetch_planes = [&](Stage& S, int k) {
        const long bu = pl(k + 1), bk = pl(k);
#pragma unroll
        for (int s = 0; s < kQLoads; ++s) {
#pragma unroll
            for (int q = 0; q < 3; ++q) S.u[q][s] = u.p[q][bu + gp[s]];
            S.m[s] = mu[bu + gp[s]];
            S.rn[s] = rho_n[bk + gp[s]];
            S.r1[s] = rho1[bk + gp[s]];
        }
    };
    auto fetch_ap = [&](Stage& S, int k) {
        const long b = pl(k) + go;
#pragma unroll
        for (int q = 0; q < 3; ++q) S.ap[q] = Aprev.p[q][b];  // allocated; ignored on a first step
    };
    auto commit = [&](const Stage& S, int k) {
#pragma unroll
        for (int s = 0; s < kQLoads; ++s)
            if (s * kBlock + kBlock <= kQRN || vp[s]) {
                const int c = t + s * kBlock;
#pragma unroll
                for (int q = 0; q < 3; ++q) UU[q][ring_slot<3>(k + 1)][c] = S.u[q][s];
                MM[ring_slot<3>(k + 1)][c] = S.m[s];
                RN[k & 1][c] = S.rn[s];
                R1[k & 1][c] = S.r1[s];
            }
    };
    {
        const long a = pl(z0 - 1), a1 = pl(z0);
#pragma unroll
        for (int s = 0; s < kQLoads; ++s)
            if (vp[s]) {
                const int c = t + s * kBlock;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    UU[q][ring_slot<3>(z0 - 1)][c] = u.p[q][a + gp[s]];
                    UU[q][ring_slot<3>(z0)][c] = u.p[q][a1 + gp[s]];
                }
                MM[ring_slot<3>(z0 - 1)][c] = mu[a + gp[s]];
                MM[ring_slot<3>(z0)][c] = mu[a1 + gp[s]];
                RN[(z0 - 1) & 1][c] = rho_n[a + gp[s]];
                R1[(z0 - 1) & 1][c] = rho1[a + gp[s]];
            }
    }
    fetch_planes(SA, z0);
    fetch_ap(SA, z0);
    __builtin_amdgcn_sched_barrier(0);
    fetch_planes(SB, z0 + 1);
    fetch_ap(SB, z0 + 1);
    auto step = [&](Stage& S, int k) {
        commit(S, k);
        const int kn = k + 2 < z1 ? k + 2 : z1 - 1;
        fetch_planes(S, kn);
        __syncthreads();
        const LdsVec U{UU, k, cc};
        const LdsField<3> M{MM, k, cc};
        const LdsField<2> Rn{RN, k, cc}, Rb{R1, k, cc};
        const long o = pl(k) + go;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double a, gv;
            pred_rhs_face<3>(U, M, Rn, Rb, q, S.ap[q], first, inv_dt, inv_h, inv_h2, B, body_on, a, gv);
            A.p[q][o] = a;
            g.p[q][o] = gv;
        }
        fetch_ap(S, kn);
        // the next commit overwrites the plane below k
        __syncthreads();
    };
    // steps z0 .. z1 - 1 in pairs (stage A, stage B); TZ is even
    for (int k = z0; k < z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
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
            double mp[3], mm[3], xp[3], xm[3];
            visc_coefs<DIM>(S, c, mu, q, mp, mm);
            const double rf = 0.5 * (rho1[c] + rho1[S.at(q, -1)]);
            const double* xq = x.p[q];
#pragma unroll
            for (int e = 0; e < DIM; ++e) {
                xp[e] = xq[S.at(e, 1)];
                xm[e] = xq[S.at(e, -1)];
            }
            const double Mx = helm_apply<DIM>(mp, mm, xp, xm, xq[c], rf, inv_dt, inv_h2);
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
    double* alt[3] = {nullptr, nullptr, nullptr};  // second x of the single-pass 3D sweep
    int sweep = IB_FLOW_SWEEP_AUTO;
};

// the single-pass sweep applies to 3D grids of whole 32 x 8 column tiles
static bool helm_tiled_grid(const Dims& d) { return d.dim == 3 && d.nx % kHTX == 0 && d.ny % kHTY == 0; }

// planes per workgroup of the single-pass sweep: the largest of 16, 8, 4, 2
// that divides nz
static int helm_tz(const Dims& d) {
    for (int tz = 16; tz > 2; tz /= 2)
        if (d.nz % tz == 0) return tz;
    return 2;
}

static void free_flow(ib_flow* f) {
    if (!f) return;
    for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 3; ++q)
            if (f->adv[b][q]) hipFree(f->adv[b][q]);
    for (int q = 0; q < 3; ++q) {
        if (f->g[q]) hipFree(f->g[q]);
        if (f->ustar[q]) hipFree(f->ustar[q]);
    }
    for (double* p : {f->Hn, f->rho_n, f->mu, f->red, f->mred, f->prop, f->alt[0], f->alt[1], f->alt[2]})
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
    if (helm_tiled_grid(f->d))
        for (int q = 0; q < 3; ++q) alloc(&f->alt[q], bytes);
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

extern "C" int ib_flow_set_sweep(ib_flow* f, int kind) {
    IB_CHECK(f, IB_EINVAL, "ib_flow_set_sweep: null handle");
    IB_CHECK(kind == IB_FLOW_SWEEP_AUTO || kind == IB_FLOW_SWEEP_COLOUR, IB_EINVAL,
             "ib_flow_set_sweep: unknown kind");
    f->sweep = kind;
    return IB_OK;
}

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
    // the single-pass sweep and the tiled right side and residual apply to
    // 3D grids of whole 32 x 8 column tiles
    const bool tiled = f->sweep == IB_FLOW_SWEEP_AUTO && helm_tiled_grid(d) && f->alt[0];
    const int tz = helm_tz(d), hx = d.nx / kHTX, hy = d.ny / kHTY;
    if (tiled)
        hipLaunchKernelGGL(k_pred_rhs_tiled, dim3(hx * hy * (d.nz / tz)), blk, 0, st, vec3(u, 3), rho_n, rho1, mu,
                           vec3(Aprev, 3), first, d, inv_dt, out3(Acur, 3), out3(f->g, 3), B, B.on() ? 1 : 0, tz,
                           hx, hy, d.nz / tz);
    else if (dim == 2)
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
    // the single-pass sweep alternates between u* and f->alt; cur holds the
    // latest iterate, copied into u* at the end
    // planes per workgroup of the tiled residual: the fewest (even, dividing
    // nz) that keep the workgroups within the partial-sum buffer (0: none does)
    int rtz = 0;
    if (tiled)
        for (int z = 2; z <= d.nz && !rtz; z *= 2)
            if (d.nz % z == 0 && (long)hx * hy * (d.nz / z) <= kFlowRed) rtz = z;
    double* cur[3] = {ustar[0], ustar[1], ustar[2]};
    double* oth[3] = {f->alt[0], f->alt[1], f->alt[2]};
    auto settle = [&]() -> int {
        if (cur[0] != ustar[0])
            for (int q = 0; q < dim; ++q)
                IB_HIP(hipMemcpyAsync(ustar[q], cur[q], sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        return IB_OK;
    };
    while (true) {
        if (tiled) {
            hipLaunchKernelGGL(k_helm_fused, dim3(hx * hy * (d.nz / tz)), blk, 0, st, vec3(cur, 3), out3(oth, 3),
                               vec3(gc, 3), rho1, mu, d, inv_dt, tz, hx, hy, d.nz / tz);
            std::swap(cur, oth);
        } else {
            for (int colour = 0; colour < 2; ++colour) {
                if (dim == 2)
                    hipLaunchKernelGGL(k_helm_sweep<2>, gh, blk, 0, st, out3(ustar, 2), vec3(gc, 2), rho1, mu,
                                       d, inv_dt, colour);
                else
                    hipLaunchKernelGGL(k_helm_sweep<3>, gh, blk, 0, st, out3(ustar, 3), vec3(gc, 3), rho1, mu,
                                       d, inv_dt, colour);
            }
        }
        ++sweeps;
        // the residual is read from one sweep before the previous call's count on
        if (sweeps < f->last_sweeps - 1 && sweeps < max_sweeps) continue;
        ++S->checks;
        const double* xc[3] = {cur[0], cur[1], cur[2]};
        int nbr = nb;  // partial sums written
        if (tiled && rtz > 0) {
            nbr = hx * (d.ny / 8) * (d.nz / rtz);
            hipLaunchKernelGGL(k_helm_resid_tiled, dim3(nbr), blk, 0, st, vec3(xc, 3), vec3(gc, 3), rho1, mu, d,
                               inv_dt, rtz, hx, d.ny / 8, d.nz / rtz, f->red);
        } else if (dim == 2)
            hipLaunchKernelGGL(k_helm_resid<2>, dim3(nb), blk, 0, st, vec3(xc, 2), vec3(gc, 2), rho1, mu, d,
                               inv_dt, f->red);
        else
            hipLaunchKernelGGL(k_helm_resid<3>, dim3(nb), blk, 0, st, vec3(xc, 3), vec3(gc, 3), rho1, mu, d,
                               inv_dt, f->red);
        IB_TRY(device_sum(f->red, nbr, f->red + 2 * kFlowRed, st));
        IB_TRY(device_sum(f->red + kFlowRed, nbr, f->red + 2 * kFlowRed + 1, st));
        IB_HIP(hipMemcpyAsync(f->host, f->red + 2 * kFlowRed, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        IB_HIP(hipStreamSynchronize(st));
        const double rr = f->host[0], gg = f->host[1];
        if (!std::isfinite(rr) || !std::isfinite(gg)) {
            S->sweeps = sweeps;
            S->rel_res = rr;
            IB_TRY(settle());
            return fail(IB_ENAN, "ib_predict: residual is not finite");
        }
        if (gg == 0.0) {
            // g = 0: the (nonsingular) system has the solution 0
            for (int q = 0; q < dim; ++q) IB_HIP(hipMemsetAsync(ustar[q], 0, sizeof(double) * N, st));
            for (int q = 0; q < 3; ++q) cur[q] = ustar[q];
            rel = 0.0;
            break;
        }
        rel = std::sqrt(rr / gg);
        if (rel <= rtol) break;
        if (sweeps >= max_sweeps) {
            S->sweeps = sweeps;
            S->rel_res = rel;
            IB_TRY(settle());
            return fail(IB_ENOTCONV, "ib_predict: the implicit viscous system did not converge");
        }
    }
    IB_TRY(settle());
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
