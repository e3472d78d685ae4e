/*
 * ibproj.h -- C ABI of the MI355X immersed-boundary projection step.
 *
 * Method: Ong & Miura, "New Immersed Boundary Method with Irrotational
 * Discrete Delta Vector for Droplet Simulations with Large Density Ratio"
 * (arXiv 1807.10504). One projection step interpolates the MAC velocity to
 * the interface markers (Section 2.2, eq jump_condu), spreads the marker
 * surface tension to the grid with the irrotational delta vector grad_h H
 * (Section 3.2, eqs delta_hea_xy, new_hea, new_hea2) or the conventional
 * delta function (Section 3.1, eq delta_vec), builds the density from the
 * indicator (eq indicator), solves div(beta grad p) = div(u_star / dt + beta F)
 * (eq ps with the force in the projection, eq ns2_new) by geometric
 * multigrid, and corrects the velocity (eq ns2_new).
 *
 * Conventions shared by every entry point
 *  - Grid: uniform spacing h, periodic box of n[0] x n[1] (x n[2]) cells.
 *    Cell arrays are SoA, x fastest: index c = (k*n[1] + j)*n[0] + i.
 *    The velocity/force component along axis d is stored at the face on the
 *    low side of the cell along d (u[c] at x = i*h), one array per
 *    component, same length as a cell array.
 *  - Floating point is IEEE binary64 unless a name says otherwise.
 *  - "device" pointers are HIP device memory owned by the caller; the
 *    library never frees caller memory. "host" pointers are ordinary host
 *    memory, read or written before the call returns.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream). All
 *    device work is enqueued on it. Calls that must read a device scalar
 *    (residual norms, error flags, the 2D marker round trip) synchronise
 *    that stream before returning; such calls are marked "syncs".
 *  - Return value: IB_OK (0) or a negative error code below. On error the
 *    outputs are unspecified unless stated; ib_last_error() returns a
 *    message for the calling thread. No exception crosses this ABI.
 *  - Handles (ib_ctx, mg_handle) own their device workspace, allocated in
 *    the create/setup call and freed in destroy. A handle may be used from
 *    one host thread at a time; calls on one handle must not overlap.
 */
#ifndef IBPROJ_H
#define IBPROJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IB_OK        0
#define IB_EINVAL   -1  /* bad argument: null pointer, size, mode, grid not coarsenable */
#define IB_EHIP     -2  /* a HIP runtime call failed */
#define IB_ENOMEM   -3  /* device allocation failed */
#define IB_ENOTCONV -4  /* multigrid hit max_cycles; p holds the last iterate, stats filled */
#define IB_EGEOM    -5  /* geometry: marker or offset surface outside the box interior,
                           a band face with no element in reach, or the B-spline normal
                           matrix not positive definite (Schoenberg-Whitney violated) */
#define IB_ENAN     -6  /* NaN/Inf residual */

enum { IB_SPREAD_IRROT = 0, IB_SPREAD_DELTA = 1 };
enum { MG_FP64 = 0, MG_MIXED = 1 };
enum { WS_ZERO = 0, WS_PREV = 1, WS_NN = 2 };

typedef struct {
    int dim;      /* 2 or 3 */
    int n[3];     /* cells per axis; n[2] ignored when dim == 2 */
    double h;     /* uniform spacing */
} ib_grid;

/* An interface: closed counter-clockwise polyline (2D) or closed triangle
 * mesh with outward counter-clockwise triangles (3D). */
typedef struct {
    int n_markers;
    const double* X;       /* device, n_markers*dim, interleaved (x, y[, z]) */
    int n_elems;           /* 3D: triangle count; 2D: 0 (elements are k -> k+1 mod n) */
    const int32_t* elems;  /* device, n_elems*3 vertex indices (3D); NULL in 2D */
    const double* nrm;     /* device, n_markers*dim unit normals toward the drop
                              (3D: required, they define the offset surfaces;
                              2D: may be NULL, then the left perpendicular of the
                              chord X_{k+1} - X_{k-1} is used) */
    const double* fs;      /* device, n_markers: surface tension times curvature */
    const double* ds;      /* device, n_markers: arc length (2D) / area (3D) */
} ib_surface;

typedef struct ib_ctx ib_ctx;
typedef struct mg_handle mg_handle;
typedef struct ib_nn ib_nn;

/* ---------------------------------------------------------------------------
 * Context: workspace for binning, spreading and the step. max_markers and
 * max_elems bound every later surface. Cells per axis must be even and the
 * total below 2^31. Allocates device memory (about 40 bytes per cell plus
 * 24 bytes per face per axis).  Errors: IB_EINVAL, IB_ENOMEM, IB_EHIP. */
int  ib_create(const ib_grid* g, int max_markers, int max_elems, ib_ctx** out);
void ib_destroy(ib_ctx* ctx);

/* a1 -- marker binning (deterministic counting sort into 4^dim-cell tiles).
 * tile_of_marker: device int32[n_markers] tile key of each marker;
 * order:          device int32[n_markers] marker indices sorted by tile,
 *                 ascending marker index within a tile (stable);
 * tile_start:     device int32[n_tiles + 1], n_tiles = prod(n[d] / 4),
 *                 markers of tile t are order[tile_start[t] .. tile_start[t+1]).
 * Marker positions are wrapped into the periodic box. Any output may be NULL
 * (the context keeps its own copy for ib_spread). */
int ib_bin_markers(ib_ctx* ctx, const ib_surface* s, int32_t* tile_of_marker,
                   int32_t* order, int32_t* tile_start, void* stream);

/* a2 -- interpolation, eq jump_condu:
 * U[s*dim + d] = sum over faces f of orientation d of u_d(f) phi(dx/h)...,
 * phi(q) = (1 + cos(pi q/2))/4 for |q| < 2 (eq cherby in grid units), with
 * minimum-image periodic offsets. u: dim device face arrays; U: device
 * n_markers*dim. Errors: IB_EINVAL. */
int ib_interp(ib_ctx* ctx, const double* const u[3], const ib_surface* s, double* U,
              void* stream);

/* a4 + a5 -- spreading.
 * IB_SPREAD_IRROT: H (device cell array, required) is the discrete Heaviside
 *   built from the interface offset by -1.5h, -0.5h, 0.5h, 1.5h (mitred in
 *   2D, along nrm in 3D) with region values H(q) = 1/2 + q/4 +
 *   sin(pi q/2)/(2 pi) at q = -2..2 (Section 3.2); F_d = f (H_c - H_{c-e_d})/h
 *   with f = fs at the foot point on the nearest element (linear/barycentric).
 *   The offset surfaces must stay more than 4h from every box face (they are
 *   not wrapped across the periodic seam): else IB_EGEOM (syncs).
 * IB_SPREAD_DELTA: F_d(x_f) = sum_s fs_s ds_s n_s,d delta_h(x_f - X_s)
 *   (eq delta_vec); H may be NULL (then not computed) or is filled as above.
 * F: dim device face arrays, fully overwritten. Deterministic: repeated calls
 * give bitwise identical results. */
int ib_spread(ib_ctx* ctx, const ib_surface* s, int mode, double* const F[3], double* H,
              void* stream);

/* a6 -- density and face coefficient (eq indicator with I = H):
 * rho_c = rho_out + (rho_in - rho_out) H_c, beta_d[c] = 2/(rho_c + rho_{c-e_d}).
 * H device cell array; beta: dim device face arrays. */
int ib_coefficients(ib_ctx* ctx, const double* H, double rho_in, double rho_out,
                    double* const beta[3], void* stream);

/* a6 -- the cell densities alone, rho_c = rho_out + (rho_in - rho_out) H_c
 * (eq indicator with I = H), rounded as in ib_coefficients (a separate
 * multiply and add), so that 2/(rho_c + rho_{c-e_d}) is bitwise beta_d[c].
 * H, rho: device cell arrays. */
int ib_density(ib_ctx* ctx, const double* H, double rho_in, double rho_out, double* rho,
               void* stream);

/* a7 -- right side (eqs ps, ns2_new):
 * b_c = (1/h) sum_d [w_d(c+e_d) - w_d(c)], w = u_star / dt + beta F, mean removed. */
int ib_rhs(ib_ctx* ctx, const double* const u_star[3], const double* const F[3],
           const double* const beta[3], double dt, double* b, void* stream);

/* a11 -- velocity update (eq ns2_new): u_d = u*_d + dt beta_d (F_d - (p_c - p_{c-e_d})/h).
 * u_new may alias u_star. */
int ib_update(ib_ctx* ctx, const double* const u_star[3], const double* const F[3],
              const double* const beta[3], const double* p, double dt,
              double* const u_new[3], void* stream);

/* ---------------------------------------------------------------------------
 * Multigrid for A p = b, (A p)_c = (1/h^2) sum_faces beta_f (p_nb - p_c),
 * periodic, zero-mean solution (Section 2.1: centred second order, solved by
 * multigrid). Cell-centred V(nu1, nu2) cycles: red-black Gauss-Seidel (red =
 * index sum even, first), restriction = mean of the 2^dim children,
 * prolongation = cell-centred (bi/tri)linear, coarse face coefficient = mean
 * of the fine faces on it, coarsest n_coarsest^dim grid solved exactly with
 * the zero-mean constraint, mean removed once after the last cycle (a cycle
 * commutes with adding a constant).
 * MG_MIXED: float32 V-cycles on the float64 defect r = b - A p (float64
 * residual, update and coarsest solve), same stopping test.
 * krylov = 1 (an extension; the paper names multigrid only): flexible
 * conjugate gradients in float64 preconditioned by one V-cycle from a zero
 * guess (float32 V-cycle under MG_MIXED),
 *   r = b - A p, z = V(r), d = z;  each iteration q = A d, alpha = (r,z)/(d,q),
 *   p += alpha d, r -= alpha q, z = V(r), beta = -alpha (q,z)/(r,z)_old,
 *   d = z + beta d;
 * the recursively updated r is checked first; once it reaches rtol the true
 * residual b - A p is formed and decides the stop (if it has not reached
 * rtol, it replaces r and the iteration goes on). Four more float64 cell
 * arrays. Deterministic: every sum has a fixed order. */
typedef struct {
    int precision;   /* MG_FP64 or MG_MIXED */
    int nu1, nu2;    /* smoothing sweeps before / after the coarse correction (2, 2) */
    int n_coarsest;  /* cells per axis on the coarsest grid (4); n[d] = n_coarsest * 2^L */
    int krylov;      /* 0: V-cycles; 1: flexible CG preconditioned by one V-cycle */
    int split_coarse; /* 0: the levels of at most 32768 cells (generic restriction) run as
                         one persistent workgroup per cycle, and on a 3D density level the
                         prolongation is folded into the first post-smoothing sweep;
                         1: one launch per phase (same results bit for bit; for
                         comparison) */
} mg_opts;

typedef struct {
    int cycles;              /* V-cycles (outer iterations in MG_MIXED; CG iterations, one
                                V-cycle each, with krylov) performed */
    double rel_res0;         /* ||b - A p0|| / ||b|| of the initial guess */
    double rel_res;          /* final ||b - A p|| / ||b|| (with krylov: the true residual when
                                the solve stopped on rtol, the recursive one after
                                fixed_cycles) */
    double res_hist[128];    /* rel_res after each cycle (first 128); -1 for cycles run
                                without a check (the solver skips norms it can predict) */
    int true_checks;         /* krylov: true residuals formed to confirm the stop */
} mg_stats;

/* Allocates the hierarchy. Errors: IB_EINVAL (grid not n_coarsest * 2^L), IB_ENOMEM. */
int  mg_setup(const ib_grid* g, const mg_opts* o, mg_handle** out);
/* beta: dim device face arrays of the finest level. The handle keeps these
 * pointers (no copy) until the next call: they must stay valid and unchanged
 * while mg_solve runs. Coarsens the coefficients and factorises the coarsest
 * grid. */
int  mg_update_coeffs(mg_handle* m, const double* const beta[3], void* stream);
/* The same from cell densities (device cell array, from ib_density): the
 * finest face coefficient is beta_d[c] = 2/(rho_c + rho_{c-e_d}) (eq
 * indicator, the face density being the mean of its two cells), bitwise the
 * mg_update_coeffs hierarchy for the beta of ib_coefficients. The handle keeps
 * the pointer (no copy) until the next update. On 3D grids with x a multiple
 * of 64, y of 8, at least 128^3 cells and one coarse level, the finest-level
 * kernels form the coefficients from rho where they use them (one array read
 * instead of three); on other grids the face arrays are formed once into
 * storage of the handle (IB_ENOMEM if that allocation fails). */
int  mg_update_density(mg_handle* m, const double* rho, void* stream);
/* b: device cell array (zero mean); p: device cell array, in: initial guess,
 * out: zero-mean solution. Stops when ||b - A p||_2 / ||b||_2 <= rtol or after
 * max_cycles (IB_ENOTCONV); fixed_cycles > 0 instead runs exactly that many
 * cycles (no test). stats may be NULL. Syncs once per cycle (one scalar).
 * b = 0 returns p = 0. Errors: IB_EINVAL, IB_ENOTCONV, IB_ENAN. */
int  mg_solve(mg_handle* m, const double* b, double* p, double rtol, int max_cycles,
              int fixed_cycles, mg_stats* stats, void* stream);
void mg_destroy(mg_handle* m);
/* ||b - A p||_2 / ||b||_2 on the finest level with the coefficients of the last
 * mg_update_coeffs (0 when b = 0). Syncs. */
int  mg_residual_norm(mg_handle* m, const double* b, const double* p, double* rel, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the residual norm of
 * mg_residual_norm without a handle and without any allocation or host sync.
 * rho: device cell densities, the operator's face coefficients being
 * 2 / (rho_c + rho_{c-e_d}) as after mg_update_density; b, p: device cell
 * arrays; rel: one device double that receives ||b - A p||_2 / ||b||_2 (0 when
 * b = 0) in stream order. Same kernels and summation order as
 * mg_residual_norm on a handle given these densities. The partial sums live
 * in a fixed device array of the library (128 KB per GPU, held until the
 * process ends; nothing needs clearing between calls), shared by every call
 * on that GPU: calls that overlap on one GPU race. At most 2^31 - 1 cells
 * (IB_EINVAL beyond). Errors: IB_EINVAL, IB_EHIP. */
int  mg_residual_norm_noalloc(const ib_grid* g, const double* rho, const double* b, const double* p,
                              double* rel, void* stream);

/* ---------------------------------------------------------------------------
 * One projection step (a1..a11). */
typedef struct {
    double rho_in, rho_out;  /* drop and ambient densities */
    double sigma;            /* surface tension coefficient (2D relocation) */
    double dt;
    double rtol;             /* multigrid stopping tolerance */
    int max_cycles;
    int fixed_cycles;        /* > 0: exactly this many cycles (parity runs) */
    int spread_mode;         /* IB_SPREAD_IRROT or IB_SPREAD_DELTA */
    int warm_start;          /* WS_ZERO, WS_PREV (p_prev as initial guess) or WS_NN
                                (network guess from (b, 1/rho, p_prev), the start when it
                                is finite and its error in the operator's energy norm is
                                below the fallback's, p_prev or 0 when p_prev is NULL,
                                judged by the energy functional of ib_outputs; else the
                                fallback) */
} ib_params;

typedef struct {
    const double* u_star[3]; /* device face arrays */
    const double* p_prev;    /* device cell array (WS_PREV) or NULL */
    ib_surface surf;         /* 3D: the static surface (all fields required).
                                2D: only n_markers is read; markers come from X_host. */
    double* X_host;          /* 2D: host n_markers*2, in: markers at step n, out: advanced
                                by dt U and relocated on the least-squares B-spline.
                                3D project_step: NULL. 3D flow_step: host
                                n_markers*3 vertices, advanced by dt U and moved
                                onto the local least-squares surface. */
    ib_nn* nn;               /* WS_NN: the network (of the grid's dimension), else NULL */
    const int32_t* elems_host; /* 3D flow_step: host copy of surf.elems (the moving
                                  surface's triangles); NULL otherwise */
} ib_state;

typedef struct {
    double* p;               /* device cell array (required) */
    double* u[3];            /* device face arrays (required; may alias u_star) */
    double* U;               /* device n_markers*dim marker velocities (required) */
    double* H;               /* device cell array or NULL */
    double* F[3];            /* device face arrays or NULL */
    double* fs_host;         /* 2D: host n_markers sigma*kappa after relocation, or NULL */
    double* b;               /* device cell array: copy of the right side, or NULL */
    mg_stats stats;
    int guess_accepted;      /* WS_NN: 1 when the network guess was used */
    double guess_rel_res;    /* WS_NN: ||b - A p_nn|| / ||b|| */
    double prev_rel_res;     /* WS_NN: the same of the fallback (1 for the zero start) */
    double guess_energy;     /* WS_NN: E(p_nn) = p_nn . (b + r), r = b - A p_nn; with
                                K = -A, E(x) = ||x - p||_K^2 - ||p||_K^2 */
    double prev_energy;      /* WS_NN: E of the fallback (0 for the zero start) */
} ib_outputs;

/* Runs interp -> (2D: D2H U, host advance + B-spline relocation, H2D) ->
 * spread -> coefficients -> rhs -> mg_solve -> update on `stream`. The mg
 * handle must be set up for the same grid. Syncs (per multigrid cycle and, in
 * 2D, for the marker round trip). Errors: any of the above. */
int project_step(ib_ctx* ctx, mg_handle* m, const ib_params* prm, ib_state* st,
                 ib_outputs* out, void* stream);

/* ---------------------------------------------------------------------------
 * Momentum predictor (Section 2.1, eq ns1_new with the surface tension moved
 * to the projection):
 *   rho^{n+1}_f (u* - u^n)/dt = -(3/2 C(u^n) - 1/2 C(u^{n-1})) + 1/2 (D u* + D u^n)
 * Adams-Bashforth advection C (eqs ns_1, ad_bf), Crank-Nicolson viscous
 * stress D (eq cr_ni), per face component d on the periodic staggered grid:
 *   C_d = rho_f (1/h) sum_e [flux on the high side - flux on the low side along e],
 *     e = d: ((u_d + u_d of the cell's other face)/2)^2 at the cells c and
 *            c - e_d;
 *     e != d: mean of the two u_e faces meeting at the edge x mean of the two
 *            u_d faces there;
 *   the density stays outside the surface sum, as eq ns_1 writes rho div(u u)
 *   (with rho inside, a moving interface would take a -u d rho/dt source);
 *   D_d = (1/h^2) sum_e [mu_+ (u_d(c+e_e) - u_d(c)) - mu_- (u_d(c) - u_d(c-e_e))],
 *     mu at the cells c, c - e_d for e = d, the 4-cell edge mean otherwise;
 *   rho_f = (rho_c + rho_{c-e_d})/2 (the projection's face density).
 * mu is the dynamic viscosity; every array below is a device cell/face array
 * of the context's grid, FP64, owned by the caller. */
typedef struct ib_flow ib_flow;

typedef struct {
    int sweeps;              /* red-black Gauss-Seidel sweeps of the implicit system */
    double rel_res;          /* ||g - M u*|| / ||g|| at exit (M = rho_f/dt - D/2) */
    int first_step;          /* 1: the advection history was empty (explicit Euler) */
    /* free-fall bookkeeping of flow_step / axi_flow_step (zero when off) */
    double frame_a;          /* frame acceleration applied in this step */
    double com;              /* vertical centroid of the incoming markers */
    double measure;          /* their enclosed area / volume of revolution */
    double mass_delta;       /* normal displacement of the mass correction (0: none) */
    int checks;              /* residual evaluations of the implicit system */
} ib_flow_stats;

typedef struct {
    double mu_in, mu_out;    /* drop and ambient dynamic viscosities (>= 0) */
    double rtol;             /* tolerance of the implicit viscous system */
    int max_sweeps;          /* sweeps allowed (IB_ENOTCONV beyond) */
    /* free-fall runs (Section 2.1: non-inertial frame, conservation of mass);
       all zero for none. The vertical axis is y in 2D and the axis of the
       meridian plane. */
    double gravity;          /* g along the vertical axis, applied as the force
                                density (rho - rho_mean) g on the vertical faces
                                (rho_mean: volume mean of rho^{n+1}; the periodic
                                box takes no net force) */
    int frame;               /* 1: frame acceleration a = -c1 (COM_n - COM_0)/dt
                                - c2 (COM_n - COM_{n-1})/dt on the drop's centre of
                                mass (eq fictitious read as a restoring control),
                                force density rho a on the vertical faces */
    double c1, c2;           /* its constants (Section 2.1: 0.1 and 0.1) */
    int mass_every;          /* > 0: every this many steps, when the enclosed
                                area / volume differs from the first step's by more
                                than 1e-6 relatively, all markers move by one
                                distance along their normals (bisection to 1e-12) */
    double mass_target;      /* > 0: the area / volume the correction restores
                                instead of the first step's */
    int indicator_density;   /* 1 (flow_step with IB_SPREAD_DELTA only): rho^{n+1}
                                and mu^{n+1} follow the indicator of eq ind_psn
                                (ib_indicator_solve to the projection's rtol)
                                instead of H -- the conventional scheme of
                                Section 2.2. The first such step creates the
                                indicator's hierarchy in the flow handle; the
                                first step after a reset takes rho^n from H. */
} ib_flow_params;

/* C(u) as above for every component; rho: device cell densities (rho_f is
 * the mean of the face's two cells). A may not alias u. */
int ib_advection(ib_ctx* ctx, const double* const u[3], const double* rho, double* const A[3],
                 void* stream);

/* D u of eq cr_ni for every component; mu: device cell viscosities. V may not
 * alias u. */
int ib_viscous(ib_ctx* ctx, const double* const u[3], const double* mu, double* const V[3],
               void* stream);

/* The predictor's state: the advection term of the previous step (Adams-
 * Bashforth history), H of the previous step (flow_step), and workspace, all
 * allocated here (about 4 dim + 4 grid arrays). Errors: IB_EINVAL, IB_ENOMEM. */
int  ib_flow_create(const ib_grid* g, ib_flow** out);
void ib_flow_destroy(ib_flow* f);
/* forget the history: the next predictor step is explicit Euler in the
 * advection and flow_step recomputes H of the current markers */
int  ib_flow_reset(ib_flow* f);
/* Sweep kernel of the predictor's red-black Gauss-Seidel. IB_FLOW_SWEEP_AUTO
 * (the default): on 3D grids with n[0] a multiple of 32 and n[1] of 8, one
 * single-pass sweep (a workgroup marches a 32 x 8 column tile along z,
 * updating red cells of a plane and black cells of the plane below it from
 * LDS); otherwise, and with IB_FLOW_SWEEP_COLOUR, one launch per colour. Both
 * give identical results. IB_EINVAL for another kind. */
enum { IB_FLOW_SWEEP_AUTO = 0, IB_FLOW_SWEEP_COLOUR = 1 };
int  ib_flow_set_sweep(ib_flow* f, int kind);

/* u* of eq ns1_new from u^n, the cell densities of levels n (rho_n, in C) and
 * n+1 (rho_np1, on the left), and the cell viscosities mu (both halves of
 * the Crank-Nicolson term). The implicit system (rho_f/dt - D/2) u* = g is
 * solved by red-black Gauss-Seidel on the faces of each component (red =
 * index sum even), starting from u^n, until ||g - M u*||_2 <= rtol ||g||_2
 * over all components (the norm is read on the host after every sweep from
 * one sweep before the previous call's count on, so a call may run one sweep
 * past the tolerance: syncs). Stores C(u^n) as the next step's history.
 * u_star may not alias u.
 * Errors: IB_EINVAL, IB_ENOTCONV (u_star holds the last sweep), IB_ENAN. */
int ib_predict(ib_flow* f, const double* const u[3], const double* rho_n, const double* rho_np1,
               const double* mu, double dt, double rtol, int max_sweeps, double* const u_star[3],
               ib_flow_stats* stats, void* stream);

/* One step of the full method, 2D or 3D:
 *   markers: U = interp(u^n) (st->u_star holds u^n), advanced by dt U and
 *   relocated on the least-squares B-spline (2D) or moved onto the local
 *   least-squares surface of ib_surface_lsq_3d (3D; the surface's normals,
 *   curvature force and areas come from the same fit) -- X_host in place;
 *   3D also needs st->surf.n_elems, st->surf.elems (device) and
 *   st->elems_host; the mesh keeps its connectivity (no remeshing); the
 *   free-fall frame and mass correction use the mesh's volume and the y of
 *   its centroid (ib_mesh_measure, ib_mesh_mass_correct on the fitted
 *   vertices along their fitted normals);
 *   H^{n+1}, F from the relocated markers; rho^n from the previous step's H
 *   (the first step after create/reset computes H of the incoming markers,
 *   in 3D offset along the normals of their reconstruction);
 *   u* = ib_predict; projection with u*: coefficients, right side, warm start
 *   (WS_ZERO or WS_PREV), solve, update into out->u (which may alias u^n).
 * out->p, out->u, out->U required; out->H, out->F, out->b optional as in
 * project_step. Syncs (marker round trip, predictor and multigrid norms).
 * Errors: as project_step and ib_predict. */
int flow_step(ib_ctx* ctx, ib_flow* f, mg_handle* m, const ib_params* prm,
              const ib_flow_params* fp, ib_state* st, ib_outputs* out, ib_flow_stats* fstats,
              void* stream);

/* ---------------------------------------------------------------------------
 * Axisymmetric projection step (Section 2.1: the same discretisation in
 * cylindrical coordinates; eq curv_ax; the static drop of Section 5.1).
 * The grid g (dim 2, n = {nr, nz}) is the meridian half plane r in [0, nr h],
 * z in [0, nz h], periodic in z; arrays nz x nr with r fastest. u_r lives on
 * the face at r = i h: face column 0 is the axis and (one period on) the
 * outer wall, and holds u_r = 0. With r_i = i h, r_c = (i + 1/2) h:
 *   b_c = r_c div(u_star/dt + beta F) = (r_{i+1} w_r(i+1) - r_i w_r(i))/h
 *                                   + r_c (w_z(k+1) - w_z(k))/h, mean removed,
 *   (1/h^2) sum_faces beta'_f (p_nb - p_c) = b with beta'_r = r_i beta_r,
 *   beta'_z = r_c beta_z (solved by the mg handle, set up for g),
 *   u = u_star + dt beta (F - grad p), u_r = 0 on face column 0.
 * The interface is given as the meridian curve mirrored about the axis: a
 * closed counter-clockwise polyline in a doubled plane x in [0, 2 nr h] whose
 * axis is x = nr h (X_host, n_markers points, advanced by dt U and relocated
 * on the least-squares B-spline like a 2D curve). sigma kappa adds the
 * azimuthal curvature -n_r / r to the in-plane one (eq curv_ax; r = x - nr h,
 * n toward the drop; within a quarter cell of the axis it is taken equal to the in-plane one). H and the
 * irrotational face force are built on the doubled plane and copied to the
 * half plane. The handle holds a context for each plane. */
typedef struct ib_axi ib_axi;
int  ib_axi_create(const ib_grid* g, int max_markers, ib_axi** out);
void ib_axi_destroy(ib_axi* a);
/* st->u_star: the half-plane velocity (u_r, u_z); st->p_prev with WS_PREV;
 * out: p, u (may alias u_star), U (n_markers x 2, doubled-plane marker
 * velocities) required; H, F (half plane), b, fs_host optional. Spreading:
 * IB_SPREAD_IRROT, or IB_SPREAD_DELTA (the marker force fs ds n spread by the
 * delta function on the doubled plane: an axisymmetric surface's delta on the
 * meridian plane is the curve's); warm start WS_ZERO or WS_PREV. Syncs as
 * project_step.
 * Errors: as project_step. */
int  axi_project_step(ib_axi* a, mg_handle* m, const ib_params* prm, ib_state* st,
                      ib_outputs* out, void* stream);

/* Momentum predictor on the meridian plane (eq ns1_new with eqs ad_bf and
 * cr_ni written on the annular control volumes, no swirl). With r_i = i h,
 * r_c = (i + 1/2) h, cell means ur_c(i) = (u_r(i) + u_r(i+1))/2,
 * uz_c(k) = (u_z(k) + u_z(k+1))/2, edge values the means of the two faces
 * (four cells for mu) meeting at the edge and rho_f the mean of the face's
 * two cells (the density outside the surface sum, as in the planar form):
 *   C_r = rho_f { [r_c(i) ur_c^2 |cell i - |cell i-1] / (r_i h) + [u_z u_r |top - |bottom] / h }
 *   C_z = rho_f { [r u_r u_z |right edge - |left edge] / (r_c h) + [uz_c^2 |cell k - |cell k-1] / h }
 *   D_r = [r_c mu (u_r(i+1) - u_r(i)) - r_c mu (u_r(i) - u_r(i-1))] / (r_i h^2)
 *         + [mu_e du_r/dz |top - |bottom] / h - (mu(i-1) + mu(i))/2 u_r / r_i^2
 *   D_z = [r mu_e du_z/dr |right - |left] / (r_c h^2) + [mu du_z/dz |k - |k-1] / h
 * u_r = 0 on face column 0 (axis, outer wall); the outer wall is free of
 * shear; the axis edges have zero radius. The implicit system is solved by
 * red-black Gauss-Seidel (index sum parity) to ||g - M u*|| <= rtol ||g||,
 * read as in ib_predict (syncs). The handle keeps the Adams-Bashforth
 * history; ib_axi_reset forgets it (and the previous H of axi_flow_step). */
int  ib_axi_reset(ib_axi* a);
int  axi_predict(ib_axi* a, const double* const u[2], const double* rho_n, const double* rho_np1,
                 const double* mu, double dt, double rtol, int max_sweeps, double* const u_star[2],
                 ib_flow_stats* stats, void* stream);
/* One step of the full axisymmetric method: markers advanced with u^n
 * (st->u_star) and relocated (eq curv_ax), H^{n+1} and F, rho^n from the
 * previous step's H (computed from the incoming markers after create/reset),
 * predictor, projection of u* into out (p, u, U required; u may alias u^n).
 * Warm start WS_ZERO or WS_PREV. Errors: as axi_project_step and axi_predict. */
int  axi_flow_step(ib_axi* a, mg_handle* m, const ib_params* prm, const ib_flow_params* fp,
                   ib_state* st, ib_outputs* out, ib_flow_stats* fstats, void* stream);

/* ---------------------------------------------------------------------------
 * a3 -- host FP64 least-squares B-spline relocation (Section 4), 2D closed
 * curve of n markers. X, U: host n*2. Advances X* = X + dt U, fits a
 * periodic cubic B-spline (knot spacing L/round(L/1.5h), at least 7 spans)
 * to the chord-length parametrised markers by least squares, places n new
 * markers at constant arc spacing starting at the first marker's parameter,
 * and returns fs = sigma kappa (eq ten_f with tangents half-way between
 * markers, eq b_tan), ds (the spacing) and unit inward normals. Outputs are
 * host arrays: X_out n*2, fs_out n, ds_out n, nrm_out n*2 (nrm_out may be
 * NULL). Arithmetic is binary64 with a fixed operation order (no contraction),
 * so results are reproducible bit for bit. Errors: IB_EINVAL, IB_EGEOM. */
int ib_relocate_bspline(int n, const double* X, const double* U, double dt, double h,
                        double sigma, double* X_out, double* fs_out, double* ds_out,
                        double* nrm_out);

/* ---------------------------------------------------------------------------
 * Indicator function of the conventional scheme (Section 2.2, eqs indicator
 * and ind_psn; the Poisson problem of eq poisson_delta in Section 3.1):
 *   div grad I = div delta_vec,  delta_vec = sum_k n_k ds_k delta_h(x - X_k)
 * (eq delta_vec with the unit normal toward the drop, spread as IB_SPREAD_DELTA),
 * 5-point Laplacian of the projection, periodic; the free constant makes the
 * integral of I the shoelace area A of the markers: I = P + A / |Omega|, P the
 * zero-mean solution. 2D. The handle owns a multigrid hierarchy with unit
 * coefficients (flexible CG, V(2,2)) and its workspace (about 5 cell arrays). */
typedef struct ib_indicator ib_indicator;

/* Errors: IB_EINVAL (not 2D, grid not n_coarsest 2^L), IB_ENOMEM. Syncs. */
int  ib_indicator_create(const ib_grid* g, int max_markers, ib_indicator** out);
void ib_indicator_destroy(ib_indicator* ind);
/* s: device X, nrm (unit, toward the drop), ds of a closed counter-clockwise
 * curve (fs is not read); I: device cell array (output). Solves from zero to
 * ||b - A P|| <= rtol ||b|| in at most max_cycles CG iterations (IB_ENOTCONV
 * beyond; I then holds the last iterate, shifted). Uses the context's bins.
 * stats may be NULL. Syncs once per iteration. */
int  ib_indicator_solve(ib_ctx* ctx, ib_indicator* ind, const ib_surface* s, double rtol, int max_cycles,
                        double* I, mg_stats* stats, void* stream);

/* Enclosed area (axis_x NaN: the closed planar polygon X, n x 2) or volume
 * of revolution about x = axis_x of the region the mirrored meridian curve
 * encloses on the side x >= axis_x, and the y (axial) coordinate of its
 * centroid. Host arrays. Errors: IB_EINVAL, IB_EGEOM (empty curve). */
int ib_enclosed_measure(int n, const double* X, double axis_x, double* measure, double* com);

/* Volume enclosed by a closed triangulated surface (V: nv x 3, T: nt x 3
 * outward counter-clockwise, host) and the y coordinate of its centroid (the
 * vertical axis of 3D runs), by the divergence theorem. Errors: IB_EINVAL,
 * IB_EGEOM (no positive volume). */
int ib_mesh_measure(int nv, const double* V, int nt, const int32_t* T, double* volume, double* com);

/* The mass correction below for such a mesh: every vertex moves by one
 * distance delta along its unit normal nrm (nv x 3, toward the drop), delta by
 * bisection on [-h, h] to |V - target| <= tol target, when |V - target| >
 * trigger target. V in place. Errors: IB_EINVAL. */
int ib_mesh_mass_correct(int nv, double* V, const double* nrm, int nt, const int32_t* T, double target,
                         double h, double trigger, double tol, double* delta);

/* Mass correction (Section 2.1, conservation of mass): when |V - target| >
 * trigger target (V as ib_enclosed_measure), move every marker of X (host,
 * n x 2, in place) by one distance delta along its unit normal nrm (n x 2,
 * toward the drop), delta by bisection on [-h, h] until |V - target| <=
 * tol target (at most 200 halvings). delta (may be NULL) receives it (0 when
 * no correction was needed). Errors: IB_EINVAL. */
int ib_mass_correct(int n, double* X, const double* nrm, double target, double axis_x, double h,
                    double trigger, double tol, double* delta);

/* Marker deletion / addition of the conventional front tracking (Section 2.2,
 * the foil of the B-spline relocation): the closed curve X (host, n x 2) is
 * walked from marker 0; a marker closer than lo h to the last kept one is
 * deleted (and the last kept one if it ends closer than lo h to marker 0,
 * while more than three remain); every kept gap longer than hi h then gets one
 * marker at its midpoint (the paper: lo = 1/2, hi = 3/2). X_out (host,
 * max_out x 2) receives the curve, *n_out its length. Errors: IB_EINVAL
 * (arguments, or max_out too small). */
int ib_markers_add_delete(int n, const double* X, double h, double lo, double hi, int max_out,
                          double* X_out, int* n_out);

/* Local least-squares reconstruction of a moving closed triangulated surface
 * (the 3D counterpart of the least-squares B-spline of Section 4; the paper
 * leaves surfaces to future work). Per vertex: the inward angle-weighted
 * normal n and a tangent frame (t1 = projection of the coordinate axis least
 * aligned with n, t2 = n x t1); the vertex's two-ring (itself included) in
 * frame coordinates scaled by L (mean distance of the other ring vertices);
 * the least-squares quadric z = g + d x + e y + a x^2 + b xy + c y^2. Outputs
 * (host): V_out = V + g L n (the vertex on the fitted surface), nrm = (n - d t1
 * - e t2)/sqrt(1 + d^2 + e^2), fs = sigma [(1 + e^2) 2a - 2de b + (1 + d^2) 2c] /
 * (L (1 + d^2 + e^2)^(3/2)) (sigma times the sum of principal curvatures,
 * positive for a convex drop), ds = a third of the adjacent triangles' areas of
 * V_out. V: nv x 3, T: nt x 3 outward counter-clockwise. Errors: IB_EINVAL,
 * IB_EGEOM (a degenerate neighbourhood). */
int ib_surface_lsq_3d(int nv, const double* V, int nt, const int* T, double sigma, double* V_out, double* fs,
                      double* ds, double* nrm);

/* 3D surface geometry (the paper stops at curves; this is the library's
 * extension for static closed meshes): cotangent-formula curvature force
 * F_v = -sigma d(area)/dX_v, vertex area A_v = sum(adjacent areas)/3, unit
 * angle-weighted normal toward the drop; fs = F_v . n_v / A_v, ds = A_v.
 * All host arrays: X nv*3, tris nt*3; outputs fs nv, ds nv, nrm nv*3. */
int ib_surface_geometry_3d(int nv, const double* X, int nt, const int32_t* tris, double sigma,
                           double* fs_out, double* ds_out, double* nrm_out);

/* ---------------------------------------------------------------------------
 * a12 -- diagnostics (Section 5): Delta P = mean(p | H >= 1-1e-12) -
 * mean(p | H <= 1e-12) (eq sd_pres_diff); TKE = sum of squared face
 * velocities times h^dim (eq tke); grid force sum; max |index-form curl| of F
 * (Section 3.2); max |F|. Any of p/H, u, F may be NULL (its fields are then 0).
 * Syncs. */
typedef struct {
    double dP;
    double tke;
    double force_sum[3];
    double curl_max;
    double f_max;
} ib_diag;

int ib_diagnostics(ib_ctx* ctx, const double* p, const double* H, const double* const u[3],
                   const double* const F[3], ib_diag* out, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel timing for measurement (not part of the method). When enabled, the
 * multigrid records a pair of HIP events on the solve stream around every
 * launch of a finest-level kernel and reads them at its next stream
 * synchronisation; the totals accumulate until reset. Kinds:
 *   IB_PROF_SMOOTH64 / IB_PROF_SMOOTH32 -- one colour of red-black Gauss-Seidel
 *     (levels smoothed colour by colour)
 *   IB_PROF_SWEEP64 / IB_PROF_SWEEP32 -- one full red-black sweep in a single
 *     pass (3D levels of at least 128^3 cells), stored face coefficients
 *   IB_PROF_SWEEP64_RHO -- the same float64 sweep forming the coefficients
 *     from cell densities (mg_update_density)
 *   IB_PROF_SWEEP_ZERO -- a single-pass sweep from p = 0 (the first sweep of a
 *     V-cycle whose level starts from zero; p is not read), either precision
 *   IB_PROF_SWEEP_DOTS -- the density sweep that also takes the flexible-CG
 *     inner products (the last post-smoothing sweep of the finest level),
 *     either precision (float32: against the float64 residual)
 *   IB_PROF_SWEEP_PRO -- the density sweep that first adds the prolongated
 *     coarse correction (the first post-smoothing sweep of the finest level,
 *     in place of a separate prolongation), either precision
 *   IB_PROF_RESTRICT64 / IB_PROF_RESTRICT32 -- residual + restriction
 *   IB_PROF_PROLONG64 / IB_PROF_PROLONG32 -- prolongation + correction
 *   IB_PROF_RESID -- float64 residual norm / defect
 * ib_profile_read returns the launch count and the summed duration (ms).
 * Process-wide; not thread safe. */
enum { IB_PROF_SMOOTH64 = 0, IB_PROF_SMOOTH32, IB_PROF_RESTRICT64, IB_PROF_RESTRICT32,
       IB_PROF_PROLONG64, IB_PROF_PROLONG32, IB_PROF_RESID, IB_PROF_SWEEP64,
       IB_PROF_SWEEP32, IB_PROF_SWEEP64_RHO, IB_PROF_SWEEP_ZERO, IB_PROF_SWEEP_DOTS,
       IB_PROF_SWEEP_PRO, IB_PROF_KINDS };
void ib_profile_enable(int on);
void ib_profile_reset(void);
int  ib_profile_read(int kind, long long* launches, double* total_ms);

/* ---------------------------------------------------------------------------
 * a10 -- learned warm start (project addition). A 6-layer convolutional
 * network with 3x3 (2D) or 3x3x3 (3D) taps (circular padding, channels
 * 3 -> 32 x5 -> 1, ReLU between) in bfloat16 on the matrix cores with float32
 * accumulation maps x = (b h^2 / s_b, (1/rho) / max(1/rho), p_prev / s_p)
 * (s = RMS) to y, and the guess is p0 = p_prev + s_p y; trained with Adam on
 * the mean squared error to t = (p - p_prev) / s_p, p being the multigrid
 * solution. n[0] must be a multiple of 64. Parameters cross the ABI as host
 * float32, per layer W[co][ci][(kz)][ky][kx] (unpadded channel counts) then
 * b[co]; count from ib_nn_param_count(dim) (0 for another dim). The network
 * starts with all parameters zero. */
int  ib_nn_param_count(int dim);
int  ib_nn_create(const ib_grid* g, ib_nn** out);
void ib_nn_destroy(ib_nn* nn);
int  ib_nn_set_params(ib_nn* nn, const float* params, int count);
int  ib_nn_get_params(ib_nn* nn, float* params, int count);
/* Convolution kernel. IB_NN_CONV_AUTO (the default): in 3D with n[1] a
 * multiple of 8, the tiled kernel (a workgroup keeps the layer's weights in
 * LDS and marches a 64 x 8 tile along z, staging each input plane once for
 * the three output planes it touches); otherwise, and with
 * IB_NN_CONV_DIRECT, the direct kernel (a wave reads its input slab from
 * memory for every tap). Both form every output from the same products in
 * the same order (in 3D the 3-channel first layer with its 27 in-plane
 * products of each kz packed into one operand, and the 1-channel last layer
 * with its three kz taps as rows of one product, in both) and give identical
 * results. IB_EINVAL for another kind. */
enum { IB_NN_CONV_AUTO = 0, IB_NN_CONV_DIRECT = 1 };
int  ib_nn_set_conv(ib_nn* nn, int kind);
/* p0 (device cells) from b, H (device cells; rho from H as in ib_coefficients),
 * p_prev (device cells or NULL = 0). */
int  ib_nn_predict(ib_nn* nn, const double* b, const double* H, const double* p_prev,
                   double rho_in, double rho_out, double* p0, void* stream);
/* Gradient of the loss for one sample (no update): host float32 in the
 * parameter layout (may be NULL), loss returned. Syncs. */
int  ib_nn_gradients(ib_nn* nn, const double* b, const double* H, const double* p_prev,
                     const double* p, double rho_in, double rho_out, float* grads,
                     int count, double* loss, void* stream);
/* One Adam step (lr; beta 0.9, 0.999; eps 1e-8) on the mean gradient of
 * `count` samples (arrays of device pointers, host arrays of length count;
 * p_prev may be NULL). Returns the mean loss. Syncs per sample. */
int  ib_nn_train_step(ib_nn* nn, int count, const double* const* b, const double* const* H,
                      const double* const* p_prev, const double* const* p, double rho_in,
                      double rho_out, float lr, double* loss, void* stream);

/* Message of the last error on the calling thread ("" if none). */
const char* ib_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IBPROJ_H */
