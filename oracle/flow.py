"""Momentum predictor and the full flow step (oracle; test infrastructure
only -- the product path never imports this package).

Section 2.1, eq ns1_new (the surface tension is applied in the projection,
eq ns2_new):
    rho^{n+1} (u* - u^n) / dt = -ADV + VISC,
with the advection by Adams-Bashforth (two levels) and the viscous stress by
Crank-Nicolson:
    ADV  = 3/2 C(u^n) - 1/2 C(u^{n-1})      (first step: C(u^n)),
    VISC = 1/2 (D u* + D u^n).
Staggered grid (same convention as the rest of the oracle): component d lives
on the face at the low side of cell c along d, arrays (nz, ny, nx), periodic,
uniform h.

C (eqs ns_1 and ad_bf): the face density times the surface sum of u u . ds
of the face's control volume, divided by its volume h^dim. The control volume
of face (c, d) exchanges u u through
  * the two cell centres along d (cells c and c - e_d): the square of the
    mean of the two faces of that cell;
  * the four edges across the other axes e: the mean of u_e on the two
    e-faces meeting there times the mean of u_d on the two d-faces meeting
    there;
(h^{dim-1} per face), and the density is that of the face,
rho_f = (rho_c + rho_{c-e_d})/2.
D (eq cr_ni): the same control volume with fluxes mu du_d/dn, mu at the cell
centres along d and the mean of the four cells around each edge across the
other axes, divided by h^2.

Readings (the paper is silent or inconsistent):
  * eq ns_1 has the density outside the divergence (rho div(u u)) while eq
    ad_bf writes the surface sum with rho at the flux points; the two agree
    only where rho is constant. Inside the flux, div(rho u u) = rho div(u u) +
    u div(rho u) adds -u d rho/dt at a moving interface, a momentum source
    that grows without bound at density ratio 100 (a drop stretched by 1.3
    blows up within 0.05 time units); the density is taken outside, at the
    face, as eq ns_1 writes it;
  * mu is the dynamic viscosity (the free-fall data of Section 5 are dynamic
    viscosities) and follows H like the density:
    mu = mu_out + (mu_in - mu_out) H;
  * the density in C is that of time level n; the face density on the left
    of eq ns1_new is the arithmetic mean of the two cells at level n+1 (the
    same face density the projection uses, beta = 1/rho_face);
  * both Crank-Nicolson halves use the viscosity of level n+1;
  * the implicit system is solved here exactly (sparse direct factorisation).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bspline, force, heaviside, poisson, transfer


def _at(a, dim, shifts):
    """a evaluated at c + sum_e s_e e_e for shifts = {e: s_e} (periodic)."""
    for e, s in shifts.items():
        if s:
            a = np.roll(a, -s, axis=dim - 1 - e)
    return a


def _edge_mean(a, dim, d, e, s):
    """Mean of the four cells around the edge of face (c, d) on the side s
    (+1 or -1) along axis e: cells c, c - e_d, c + s e_e, c + s e_e - e_d."""
    return 0.25 * (a + _at(a, dim, {d: -1}) + _at(a, dim, {e: s}) + _at(a, dim, {e: s, d: -1}))


def advection(u, rho, h):
    """C(u) per face, for every component (list of arrays): rho_f times the
    surface sum of eq ad_bf taken without the density, over h."""
    dim = len(u)
    out = []
    for d in range(dim):
        acc = np.zeros_like(u[d])
        for e in range(dim):
            if e == d:
                up = 0.5 * (_at(u[d], dim, {d: 1}) + u[d])          # cell c
                um = 0.5 * (u[d] + _at(u[d], dim, {d: -1}))         # cell c - e_d
                acc += up * up - um * um
            else:
                # edge on the high side along e
                ve_p = 0.5 * (_at(u[e], dim, {e: 1}) + _at(u[e], dim, {e: 1, d: -1}))
                ud_p = 0.5 * (u[d] + _at(u[d], dim, {e: 1}))
                # edge on the low side along e
                ve_m = 0.5 * (u[e] + _at(u[e], dim, {d: -1}))
                ud_m = 0.5 * (u[d] + _at(u[d], dim, {e: -1}))
                acc += ve_p * ud_p - ve_m * ud_m
        out.append(face_density(rho, dim, d) * acc / h)
    return out


def _visc_coefs(mu, dim, d):
    """Per axis e: (mu on the high side, mu on the low side) of face (c, d)."""
    co = []
    for e in range(dim):
        if e == d:
            co.append((mu, _at(mu, dim, {d: -1})))
        else:
            co.append((_edge_mean(mu, dim, d, e, 1), _edge_mean(mu, dim, d, e, -1)))
    return co


def viscous(u, mu, h):
    """D u of eq cr_ni per face, for every component."""
    dim = len(u)
    out = []
    for d in range(dim):
        acc = np.zeros_like(u[d])
        for e, (mp, mm) in enumerate(_visc_coefs(mu, dim, d)):
            acc += mp * (_at(u[d], dim, {e: 1}) - u[d]) - mm * (u[d] - _at(u[d], dim, {e: -1}))
        out.append(acc / (h * h))
    return out


def viscous_matrix(mu, h, d, dim):
    """Sparse matrix of D for component d (row = flattened face index)."""
    shape = mu.shape
    N = mu.size
    idx = np.arange(N).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(shape)
    for e, (mp, mm) in enumerate(_visc_coefs(mu, dim, d)):
        rows += [idx.ravel(), idx.ravel()]
        cols += [_at(idx, dim, {e: 1}).ravel(), _at(idx, dim, {e: -1}).ravel()]
        vals += [mp.ravel() / (h * h), mm.ravel() / (h * h)]
        diag -= (mp + mm) / (h * h)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def face_density(rho, dim, d):
    return 0.5 * (rho + _at(rho, dim, {d: -1}))


def predict(u, rho_n, rho_np1, mu, dt, h, adv_prev=None, f_body=None):
    """u* of eq ns1_new; returns (u_star, C(u^n)) -- the latter is the
    Adams-Bashforth history for the next step. f_body: optional body force
    density per component (faces), added to the right side."""
    dim = len(u)
    adv = advection(u, rho_n, h)
    ab = adv if adv_prev is None else [1.5 * a - 0.5 * b for a, b in zip(adv, adv_prev)]
    vis = viscous(u, mu, h)
    u_star = []
    for d in range(dim):
        rf = face_density(rho_np1, dim, d)
        g = rf / dt * u[d] - ab[d] + 0.5 * vis[d]
        if f_body is not None and f_body[d] is not None:
            g = g + f_body[d]
        M = sp.diags(rf.ravel() / dt) - 0.5 * viscous_matrix(mu, h, d, dim)
        u_star.append(spla.spsolve(M.tocsc(), g.ravel()).reshape(u[d].shape))
    return u_star, adv


def flow_step_2d(n, h, rho_in, rho_out, mu_in, mu_out, sigma, dt, u, X, H_prev, adv_prev=None,
                 p_prev=None, rtol=1e-10, max_cycles=100, gravity=0.0, frame_a=0.0, mass_target=None,
                 conventional=False, indicator_density=False):
    """One step of the full 2D method (Section 2.1 fractional step, Section 2.2
    transfer, Section 3.2 irrotational force, Section 4 relocation):
      1. U = interpolation of u^n to the markers; markers advanced by dt U and
         relocated on the least-squares B-spline (sigma kappa, arc element);
      2. H^{n+1} from the offset polygons, F = f grad_h H^{n+1};
      3. rho^n from H_prev, rho^{n+1} and mu^{n+1} from H^{n+1};
      4. u* from the predictor (eq ns1_new);
      5. projection: b = div(u*/dt + beta F), multigrid, u^{n+1} = u* +
         dt beta (F - grad p) (eqs ps, ns2_new).
    conventional: F is the marker force spread by the discrete delta function
    (eq delta) instead of the irrotational one; indicator_density: rho^{n+1} and
    mu^{n+1} follow the indicator of eq ind_psn instead of H. H_prev is the field
    the previous step's properties followed (returned as 'prop')."""
    U = transfer.interp(u, X, h)
    Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in X], [tuple(v) for v in U], dt, h, sigma)
    Xn, fs = np.array(Xn), np.array(fs)
    if mass_target is not None:
        from . import dynamics
        Xn, _ = dynamics.mass_correct(Xn, np.array(nrm), mass_target, None, h)
    H = heaviside.heaviside_2d(Xn, n, h)
    if conventional:
        F = transfer.spread_delta(transfer.marker_forces(fs, ds, nrm), Xn, n, h)
    else:
        F = force.irrotational_force(H, Xn, fs, h)
    prop = H
    if indicator_density:
        from . import indicator
        prop = indicator.indicator(Xn, np.array(ds), np.array(nrm), n, h)
    rho_n = poisson.density(H_prev, rho_in, rho_out)
    rho1 = poisson.density(prop, rho_in, rho_out)
    mu = poisson.density(prop, mu_in, mu_out)
    f_body = None
    if gravity != 0.0 or frame_a != 0.0:
        from . import dynamics
        rf = face_density(rho1, 2, 1)
        f_body = [None, dynamics.body_force(rf, rho1.mean(), gravity, frame_a)]
    u_star, adv = predict(u, rho_n, rho1, mu, dt, h, adv_prev, f_body)
    beta = poisson.face_beta(rho1)
    b = poisson.rhs(u_star, F, beta, dt, h)
    p, cycles, _ = poisson.mg_solve(b, beta, h, p0=p_prev, rtol=rtol, max_cycles=max_cycles)
    u_new = poisson.velocity_update(u_star, F, beta, p, dt, h)
    return dict(U=U, X=Xn, fs=fs, H=H, prop=prop, F=F, u_star=u_star, adv=adv, p=p, u=u_new, cycles=cycles)


def flow_step_3d(n, h, rho_in, rho_out, mu_in, mu_out, sigma, dt, u, V, T, H_prev, adv_prev=None,
                 p_prev=None, rtol=1e-10, max_cycles=100, gravity=0.0, frame_a=0.0, mass_target=None):
    """One step with a moving closed triangulated surface (the 3D counterpart of
    flow_step_2d; the paper leaves moving surfaces to future work):
      1. U = interpolation of u^n to the vertices; V + dt U moved onto the local
         least-squares surface (surface3d.lsq_reconstruct: vertices, normals,
         sigma kappa, vertex areas); the triangles are kept;
      2. H^{n+1} from the surfaces offset along those normals, F the
         irrotational face force (nearest triangle);
      3. - 5. as flow_step_2d (gravity, frame_a: the weight (rho - rho_mean) g
         and the frame force rho a on the y faces; mass_target: the fitted
         vertices moved along their normals to that enclosed volume, as in the
         planar step)."""
    from . import surface3d
    U = transfer.interp(u, V, h)
    Vn, fs, ds, nrm = surface3d.lsq_reconstruct(np.asarray(V) + dt * U, T, sigma)
    if mass_target is not None:
        from . import dynamics
        Vn, _ = dynamics.mass_correct(Vn, nrm, mass_target, None, h, T=T)
    H = heaviside.heaviside_3d(Vn, T, n, h, nrm=nrm)
    F = force.irrotational_force(H, Vn, fs, h, tris=T)
    rho_n = poisson.density(H_prev, rho_in, rho_out)
    rho1 = poisson.density(H, rho_in, rho_out)
    mu = poisson.density(H, mu_in, mu_out)
    f_body = None
    if gravity != 0.0 or frame_a != 0.0:
        from . import dynamics
        f_body = [None, dynamics.body_force(face_density(rho1, 3, 1), rho1.mean(), gravity, frame_a), None]
    u_star, adv = predict(u, rho_n, rho1, mu, dt, h, adv_prev, f_body)
    beta = poisson.face_beta(rho1)
    b = poisson.rhs(u_star, F, beta, dt, h)
    p, cycles, _ = poisson.mg_solve(b, beta, h, p0=p_prev, rtol=rtol, max_cycles=max_cycles)
    u_new = poisson.velocity_update(u_star, F, beta, p, dt, h)
    return dict(U=U, X=Vn, fs=fs, H=H, F=F, u_star=u_star, adv=adv, p=p, u=u_new, cycles=cycles)
