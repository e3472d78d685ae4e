// C ABI entry points: context, transfer/spread/coefficients/rhs/update calls,
// diagnostics, and the projection step that chains them (Section 2.1
// fractional step with the surface tension in the projection, eq ns2_new).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace ib {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

int read_flags(Ctx* c, int* host_flags, hipStream_t st) {
    IB_HIP(hipMemcpyAsync(c->host_red, c->flags, sizeof(int) * 3, hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    std::memcpy(host_flags, c->host_red, sizeof(int) * 3);
    IB_HIP(hipMemsetAsync(c->flags, 0, sizeof(int) * 3, st));
    return IB_OK;
}

static int check_surface(Ctx* c, const ib_surface* s, bool need_force) {
    IB_CHECK(s, IB_EINVAL, "null surface");
    IB_CHECK(s->n_markers >= 0 && s->n_markers <= c->max_markers, IB_EINVAL,
             "surface: marker count outside [0, max_markers]");
    IB_CHECK(s->n_markers == 0 || s->X, IB_EINVAL, "surface: X is null");
    if (c->d.dim == 3) {
        IB_CHECK(s->n_elems >= 0 && s->n_elems <= c->max_elems, IB_EINVAL,
                 "surface: triangle count outside [0, max_elems]");
    }
    if (need_force) {
        IB_CHECK(s->n_markers == 0 || (s->fs && s->ds), IB_EINVAL, "surface: fs/ds are null");
    }
    return IB_OK;
}

}  // namespace ib

namespace ib {

static int free_ctx(ib_ctx* c) {
    if (!c) return IB_OK;
    void* ptrs[] = {c->bin_key, c->bin_order, c->tile_start, c->bin_count, c->scan_part, c->accA, c->accS, c->best, c->offv, c->mX, c->mfs, c->mds,
                    c->mnrm, c->H, c->F[0], c->F[1], c->F[2], c->beta[0], c->beta[1],
                    c->beta[2], c->rho, c->b, c->flags, c->red};
    for (void* p : ptrs)
        if (p) hipFree(p);
    if (c->host_red) hipHostFree(c->host_red);
    delete c;
    return IB_OK;
}

}  // namespace ib

using namespace ib;

extern "C" const char* ib_last_error(void) { return g_last_error.c_str(); }

extern "C" int ib_create(const ib_grid* g, int max_markers, int max_elems, ib_ctx** out) {
    IB_CHECK(g && out, IB_EINVAL, "ib_create: null argument");
    IB_CHECK(g->dim == 2 || g->dim == 3, IB_EINVAL, "ib_create: dim must be 2 or 3");
    IB_CHECK(g->h > 0.0, IB_EINVAL, "ib_create: h must be positive");
    long cells = 1;
    for (int e = 0; e < g->dim; ++e) {
        IB_CHECK(g->n[e] >= 16 && g->n[e] % kTile == 0, IB_EINVAL,
                 "ib_create: cells per axis must be >= 16 and a multiple of 4");
        cells *= g->n[e];
    }
    IB_CHECK(cells < (1L << 31), IB_EINVAL, "ib_create: grid too large");
    IB_CHECK(max_markers >= 3 && max_markers < (1 << 23), IB_EINVAL, "ib_create: max_markers");
    IB_CHECK(max_elems >= 0 && max_elems < (1 << 23), IB_EINVAL, "ib_create: max_elems");
    ib_ctx* c = new ib_ctx();
    c->g = *g;
    c->d = make_dims(*g);
    c->max_markers = max_markers;
    c->max_elems = max_elems;
    c->tnx = g->n[0] / kTile;
    c->tny = g->n[1] / kTile;
    c->tnz = g->dim == 3 ? g->n[2] / kTile : 1;
    c->n_tiles = c->tnx * c->tny * c->tnz;
    if ((long)c->n_tiles > kMaxTiles) {
        delete c;
        return fail(IB_EINVAL, "ib_create: more than 2^24 - 1 tiles of 4^dim cells");
    }
    int dim = g->dim;
    long M = max_markers;
    bool ok = true;
    auto alloc = [&](void** p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false;
    };
    alloc((void**)&c->bin_key, M * sizeof(int32_t));
    alloc((void**)&c->bin_order, M * sizeof(int32_t));
    alloc((void**)&c->tile_start, (c->n_tiles + 1) * sizeof(int32_t));
    alloc((void**)&c->bin_count, (c->n_tiles + 1) * sizeof(int32_t));
    alloc((void**)&c->scan_part, (kScanTile + 1) * sizeof(int32_t));
    alloc((void**)&c->accA, cells * sizeof(long long));
    alloc((void**)&c->accS, cells * sizeof(long long));
    alloc((void**)&c->best, (size_t)dim * cells * sizeof(unsigned long long));
    alloc((void**)&c->offv, 4 * M * dim * sizeof(double));
    alloc((void**)&c->mX, M * dim * sizeof(double));
    alloc((void**)&c->mfs, M * sizeof(double));
    alloc((void**)&c->mds, M * sizeof(double));
    alloc((void**)&c->mnrm, M * dim * sizeof(double));
    alloc((void**)&c->H, cells * sizeof(double));
    for (int e = 0; e < dim; ++e) {
        alloc((void**)&c->F[e], cells * sizeof(double));
        alloc((void**)&c->beta[e], cells * sizeof(double));
    }
    alloc((void**)&c->rho, cells * sizeof(double));
    alloc((void**)&c->b, cells * sizeof(double));
    alloc((void**)&c->flags, 4 * sizeof(int));
    c->red_len = 4096;
    alloc((void**)&c->red, c->red_len * sizeof(double));
    if (ok && hipHostMalloc((void**)&c->host_red, c->red_len * sizeof(double)) != hipSuccess)
        ok = false;
    if (!ok) {
        free_ctx(c);
        return fail(IB_ENOMEM, "ib_create: out of memory");
    }
    if (hipMemset(c->accA, 0, cells * sizeof(long long)) != hipSuccess ||
        hipMemset(c->accS, 0, cells * sizeof(long long)) != hipSuccess ||
        hipMemset(c->best, 0xff, (size_t)dim * cells * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->flags, 0, 4 * sizeof(int)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_ctx(c);
        return fail(IB_EHIP, "ib_create: initialisation failed");
    }
    *out = c;
    return IB_OK;
}

extern "C" void ib_destroy(ib_ctx* c) { free_ctx(c); }

extern "C" int ib_bin_markers(ib_ctx* c, const ib_surface* s, int32_t* tile_of_marker,
                              int32_t* order, int32_t* tile_start, void* stream) {
    IB_CHECK(c, IB_EINVAL, "ib_bin_markers: null context");
    IB_TRY(check_surface(c, s, false));
    hipStream_t st = (hipStream_t)stream;
    IB_TRY(launch_bin_markers(c, s, st));
    int n = s->n_markers;
    if (tile_of_marker && n)
        IB_HIP(hipMemcpyAsync(tile_of_marker, c->bin_key, n * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, st));
    if (order && n)
        IB_HIP(hipMemcpyAsync(order, c->bin_order, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (tile_start)
        IB_HIP(hipMemcpyAsync(tile_start, c->tile_start, (c->n_tiles + 1) * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, st));
    return IB_OK;
}

extern "C" int ib_interp(ib_ctx* c, const double* const u[3], const ib_surface* s, double* U,
                         void* stream) {
    IB_CHECK(c && u && U, IB_EINVAL, "ib_interp: null argument");
    IB_TRY(check_surface(c, s, false));
    for (int e = 0; e < c->d.dim; ++e) IB_CHECK(u[e], IB_EINVAL, "ib_interp: null velocity");
    return launch_interp(c, u, s, U, (hipStream_t)stream);
}

namespace ib {

int spread_impl(Ctx* c, const ib_surface* s, int mode, double* const F[3], double* H,
                hipStream_t st) {
    if (mode == IB_SPREAD_IRROT || H) IB_TRY(launch_heaviside(c, s, H, st));
    if (mode == IB_SPREAD_IRROT) IB_TRY(launch_irrot_force(c, s, H, F, st));
    else IB_TRY(launch_spread_delta(c, s, F, st));
    if (mode == IB_SPREAD_IRROT || H) {
        int fl[3];
        IB_TRY(read_flags(c, fl, st));
        IB_CHECK(fl[2] == 0, IB_EINVAL, "ib_spread: a triangle refers to a vertex outside [0, n_markers)");
        IB_CHECK(fl[0] == 0, IB_EGEOM, "ib_spread: an offset surface comes within 4h of the box faces");
        IB_CHECK(fl[1] == 0, IB_EGEOM, "ib_spread: a band face found no interface element within 3h");
    }
    return IB_OK;
}

// 2D: markers of stt->X_host (n of them) advanced by dt U (U on the device)
// and relocated on the least-squares B-spline on the host; X_host is updated
// in place and s points at the relocated device copies with their force data.
int relocate_2d(Ctx* c, const ib_params* prm, ib_state* stt, const double* U_dev, double* fs_host,
                ib_surface* s, hipStream_t st, double axis_x, const double* mass_target,
                double* mass_delta) {
    const int n = s->n_markers;
    std::vector<double> U(2 * (size_t)n), Xn(2 * (size_t)n), fs(n), ds(n), nr(2 * (size_t)n);
    IB_HIP(hipMemcpyAsync(U.data(), U_dev, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    IB_TRY(ib_relocate_bspline(n, stt->X_host, U.data(), prm->dt, c->d.h, prm->sigma, Xn.data(),
                               fs.data(), ds.data(), nr.data()));
    if (mass_target)
        IB_TRY(ib_mass_correct(n, Xn.data(), nr.data(), *mass_target, axis_x, c->d.h, 1e-6, 1e-12,
                               mass_delta));
    if (std::isfinite(axis_x)) {
        // a meridian curve mirrored about the axis x = axis_x: add the azimuthal
        // curvature -n_r / r (eq curv_ax). Within a quarter cell of the axis
        // n_r / r is rounding noise over a tiny radius (a pole marker drifts off
        // the axis by ~1e-9): take the limit, the in-plane curvature (exact to
        // O(r^2) for a surface meeting the axis square)
        const double h = c->d.h;
        for (int k = 0; k < n; ++k) {
            const double r = Xn[2 * k] - axis_x;
            fs[k] += std::fabs(r) < 0.25 * h ? fs[k] : prm->sigma * (-nr[2 * k] / r);
        }
    }
    std::memcpy(stt->X_host, Xn.data(), sizeof(double) * 2 * n);
    if (fs_host) std::memcpy(fs_host, fs.data(), sizeof(double) * n);
    IB_HIP(hipMemcpyAsync(c->mX, Xn.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
    IB_HIP(hipMemcpyAsync(c->mfs, fs.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    IB_HIP(hipMemcpyAsync(c->mds, ds.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    IB_HIP(hipMemcpyAsync(c->mnrm, nr.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
    // the host vectors must outlive the copies
    IB_HIP(hipStreamSynchronize(st));
    s->X = c->mX;
    s->fs = c->mfs;
    s->ds = c->mds;
    s->nrm = c->mnrm;
    return IB_OK;
}

// a6 + a8: rho and beta of level n+1 into the context, the hierarchy from them
int coefficients_and_hierarchy(Ctx* c, mg_handle* m, const ib_params* prm, const double* H,
                               hipStream_t st) {
    // when the hierarchy takes the densities, nothing reads a stored beta: the
    // right side and the update form it from rho as well
    c->beta_from_rho = mg_takes_density(m) != 0;
    IB_TRY(launch_coefficients(c, H, prm->rho_in, prm->rho_out, c->beta_from_rho ? nullptr : c->beta, c->rho,
                               st));
    if (c->beta_from_rho) IB_TRY(mg_update_density(m, c->rho, st));
    else IB_TRY(mg_update_coeffs(m, c->beta, st));
    return IB_OK;
}

// a7, a10, a9, a11 on the context's beta: right side from u_star and F, warm
// start, solve, update. Returns IB_OK or IB_ENOTCONV (the update is done).
int solve_and_update(Ctx* c, mg_handle* m, const ib_params* prm, ib_state* stt, ib_outputs* out,
                     const double* const u_star[3], const double* H, double* const F[3],
                     hipStream_t st);

}  // namespace ib

extern "C" int ib_spread(ib_ctx* c, const ib_surface* s, int mode, double* const F[3], double* H,
                         void* stream) {
    IB_CHECK(c && F, IB_EINVAL, "ib_spread: null argument");
    IB_CHECK(mode == IB_SPREAD_IRROT || mode == IB_SPREAD_DELTA, IB_EINVAL, "ib_spread: mode");
    IB_CHECK(mode != IB_SPREAD_IRROT || H, IB_EINVAL, "ib_spread: irrotational mode needs H");
    IB_TRY(check_surface(c, s, true));
    IB_CHECK(s->n_markers >= 3, IB_EINVAL, "ib_spread: fewer than 3 markers");
    for (int e = 0; e < c->d.dim; ++e) IB_CHECK(F[e], IB_EINVAL, "ib_spread: null force array");
    return spread_impl(c, s, mode, F, H, (hipStream_t)stream);
}

extern "C" int ib_coefficients(ib_ctx* c, const double* H, double rin, double rout,
                               double* const beta[3], void* stream) {
    IB_CHECK(c && H && beta, IB_EINVAL, "ib_coefficients: null argument");
    IB_CHECK(rin > 0 && rout > 0, IB_EINVAL, "ib_coefficients: densities must be positive");
    return launch_coefficients(c, H, rin, rout, beta, nullptr, (hipStream_t)stream);
}

extern "C" int ib_density(ib_ctx* c, const double* H, double rin, double rout, double* rho,
                          void* stream) {
    IB_CHECK(c && H && rho, IB_EINVAL, "ib_density: null argument");
    IB_CHECK(rin > 0 && rout > 0, IB_EINVAL, "ib_density: densities must be positive");
    return launch_coefficients(c, H, rin, rout, nullptr, rho, (hipStream_t)stream);
}

extern "C" int ib_rhs(ib_ctx* c, const double* const us[3], const double* const F[3],
                      const double* const beta[3], double dt, double* b, void* stream) {
    IB_CHECK(c && us && F && beta && b, IB_EINVAL, "ib_rhs: null argument");
    IB_CHECK(dt > 0, IB_EINVAL, "ib_rhs: dt must be positive");
    return launch_rhs(c, us, F, beta, dt, b, (hipStream_t)stream);
}

extern "C" int ib_update(ib_ctx* c, const double* const us[3], const double* const F[3],
                         const double* const beta[3], const double* p, double dt,
                         double* const un[3], void* stream) {
    IB_CHECK(c && us && F && beta && p && un, IB_EINVAL, "ib_update: null argument");
    return launch_update(c, us, F, beta, p, dt, un, (hipStream_t)stream);
}

extern "C" int ib_diagnostics(ib_ctx* c, const double* p, const double* H,
                              const double* const u[3], const double* const F[3], ib_diag* out,
                              void* stream) {
    IB_CHECK(c && out, IB_EINVAL, "ib_diagnostics: null argument");
    return launch_diagnostics(c, p, H, u, F, out, (hipStream_t)stream);
}

extern "C" int project_step(ib_ctx* c, mg_handle* m, const ib_params* prm, ib_state* stt,
                            ib_outputs* out, void* stream) {
    IB_CHECK(c && m && prm && stt && out, IB_EINVAL, "project_step: null argument");
    IB_CHECK(out->p && out->U, IB_EINVAL, "project_step: p and U outputs are required");
    hipStream_t st = (hipStream_t)stream;
    int dim = c->d.dim;
    for (int e = 0; e < dim; ++e)
        IB_CHECK(stt->u_star[e] && out->u[e], IB_EINVAL, "project_step: null velocity array");
    IB_CHECK(prm->dt > 0 && prm->rho_in > 0 && prm->rho_out > 0, IB_EINVAL,
             "project_step: dt and densities must be positive");
    ib_surface s = stt->surf;
    int n = s.n_markers;
    IB_CHECK(n >= 3 && n <= c->max_markers, IB_EINVAL, "project_step: marker count");
    if (dim == 2) {
        IB_CHECK(stt->X_host, IB_EINVAL, "project_step: 2D steps need X_host");
        IB_HIP(hipMemcpyAsync(c->mX, stt->X_host, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
        s.X = c->mX;
        s.elems = nullptr;
        s.n_elems = 0;
    } else {
        IB_TRY(check_surface(c, &s, true));
        IB_CHECK(s.elems && s.nrm, IB_EINVAL, "project_step: 3D surfaces need elems and nrm");
    }
    // a2: marker velocities
    IB_TRY(launch_interp(c, stt->u_star, &s, out->U, st));
    // a3: 2D marker advance and least-squares relocation on the host
    if (dim == 2) IB_TRY(relocate_2d(c, prm, stt, out->U, out->fs_host, &s, st, NAN, nullptr, nullptr));
    // a4, a5: Heaviside and face force
    double* H = out->H ? out->H : c->H;
    double* F[3];
    for (int e = 0; e < 3; ++e) F[e] = (out->F[e] && e < dim) ? out->F[e] : c->F[e];
    IB_CHECK(prm->spread_mode == IB_SPREAD_IRROT || prm->spread_mode == IB_SPREAD_DELTA, IB_EINVAL,
             "project_step: spread mode");
    IB_TRY(spread_impl(c, &s, prm->spread_mode, F, H, st));
    // a6: coefficients, a8: hierarchy
    IB_TRY(coefficients_and_hierarchy(c, m, prm, H, st));
    return solve_and_update(c, m, prm, stt, out, stt->u_star, H, F, st);
}

int ib::nn_warm_start(mg_handle* m, ib_state* stt, ib_outputs* out, double rho_in, double rho_out,
                      const double* b, const double* H, long N, hipStream_t st) {
    IB_CHECK(stt->nn, IB_EINVAL, "WS_NN needs a network");
    IB_CHECK(stt->p_prev != out->p, IB_EINVAL, "WS_NN needs p_prev distinct from p");
    IB_CHECK(nn_cells(stt->nn) == N, IB_EINVAL, "WS_NN: the network's grid differs from the step's");
    IB_TRY(ib_nn_predict(stt->nn, b, H, stt->p_prev, rho_in, rho_out, out->p, st));
    // multigrid judges the guess by its error in the operator's energy norm,
    // the norm in which the conjugate gradients and the V-cycles converge:
    // with K = -A, E(x) = x . (b + r(x)) = ||x - p||_K^2 - ||p||_K^2 is
    // computable from the residual, so the guess is used when it is finite
    // and E(guess) < E(fallback) (p_prev, or zero with E = 0). The residual
    // alone judges a learned guess badly: its high-frequency error, which the
    // first sweeps remove, dominates the residual but not the energy
    double eg = 0.0, ef = 0.0;
    IB_TRY(mg_energy(m, b, out->p, &out->guess_rel_res, &eg, st));
    IB_TRY(mg_energy(m, b, stt->p_prev, &out->prev_rel_res, &ef, st));
    out->guess_energy = eg;
    out->prev_energy = ef;
    if (std::isfinite(eg) && std::isfinite(out->guess_rel_res) && eg < ef) {
        out->guess_accepted = 1;
    } else if (stt->p_prev) {
        IB_HIP(hipMemcpyAsync(out->p, stt->p_prev, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    } else {
        IB_HIP(hipMemsetAsync(out->p, 0, sizeof(double) * N, st));
        mg_hint_zero_guess(m);
    }
    return IB_OK;
}

int ib::solve_and_update(Ctx* c, mg_handle* m, const ib_params* prm, ib_state* stt, ib_outputs* out,
                         const double* const u_star[3], const double* H, double* const F[3],
                         hipStream_t st) {
    // a7: right side
    const double* Fc[3] = {F[0], F[1], F[2]};
    const double* bc[3] = {c->beta[0], c->beta[1], c->beta[2]};
    const double* rho_f = c->beta_from_rho ? c->rho : nullptr;
    IB_TRY(launch_rhs(c, u_star, Fc, bc, prm->dt, c->b, st, rho_f));
    // a9, a10: warm start and solve
    long N = c->d.cells();
    if (out->b) IB_HIP(hipMemcpyAsync(out->b, c->b, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    out->guess_accepted = 0;
    out->guess_rel_res = out->prev_rel_res = 0.0;
    out->guess_energy = out->prev_energy = 0.0;
    if (prm->warm_start == WS_NN) {
        IB_TRY(nn_warm_start(m, stt, out, prm->rho_in, prm->rho_out, c->b, H, N, st));
    } else if (prm->warm_start == WS_PREV && stt->p_prev) {
        if (stt->p_prev != out->p)
            IB_HIP(hipMemcpyAsync(out->p, stt->p_prev, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    } else {
        IB_HIP(hipMemsetAsync(out->p, 0, sizeof(double) * N, st));
        mg_hint_zero_guess(m);
    }
    int rc = mg_solve(m, c->b, out->p, prm->rtol, prm->max_cycles, prm->fixed_cycles, &out->stats, st);
    if (rc != IB_OK && rc != IB_ENOTCONV) return rc;
    // a11: velocity update
    IB_TRY(launch_update(c, u_star, Fc, bc, out->p, prm->dt, out->u, st, rho_f));
    return rc;
}
