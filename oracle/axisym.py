"""Axisymmetric projection step (oracle; test infrastructure only -- the
product path never imports this package).

Section 2.1 states that the same discretisation serves the axisymmetric
cylindrical coordinates; Section 4 gives the axisymmetric curvature (eq
curv_ax); Section 5.1 the static drop on the axis (Table staticdrop_axis).

Grid: the meridian half plane r in [0, nr h], z in [0, nz h]; arrays (nz, nr)
with r fastest; u_r on the face at r = i h (i = 0 is the axis), u_z on the face
at z = k h; periodic in z. Finite volumes of the annular cells (volume
2 pi r_c h^2, r-face area 2 pi r_i h, z-face area 2 pi r_c h), r_i = i h,
r_c = (i + 1/2) h:
    div(w)_c = (r_{i+1} w_r(i+1) - r_i w_r(i)) / (r_c h) + (w_z(k+1) - w_z(k)) / h,
and the gradient on faces as in the plane. The axis face and the outer wall
r = nr h carry no flux: u_r = 0 there. In the periodic array layout the wall
is the axis face of the next period, so one column of faces (i = 0) holds
both, always zero.
The pressure equation multiplied by r_c is symmetric:
    (1/h^2) sum over faces of beta'_f (p_nb - p_c) = r_c div(u*/dt + beta F),
    beta'_r = r_i beta_r (zero on the axis / wall column), beta'_z = r_c beta_z,
and the plane multigrid solves it unchanged.

Interface: the meridian curve is passed closed, mirrored about the axis, in
the coordinates of a doubled plane x in [0, 2 nr h] whose axis is x = nr h.
H and the irrotational face force are the planar constructions on that doubled
grid (symmetric about the axis, so the axis faces carry no force), restricted
to the half plane. Curvature (eq curv_ax): the in-plane curvature of the curve
plus the azimuthal one, kappa_2 = -n_r / r with n the unit normal toward the
drop and r = x - nr h (the same expression on both halves), kappa_2 = kappa_1
within a quarter cell of the axis; f = sigma (kappa_1 + kappa_2).
"""
import numpy as np

from . import bspline, force, heaviside, poisson, transfer


def radii(nr, h):
    """Face radii r_i = i h and cell radii r_c = (i + 1/2) h (length nr)."""
    i = np.arange(nr, dtype=np.float64)
    return i * h, (i + 0.5) * h


def divergence(w, h):
    """div(w) of annular cells; w = [w_r, w_z], w_r[:, 0] must be zero."""
    nz, nr = w[0].shape
    ri, rc = radii(nr, h)
    rip = ri + h                                   # radius of the high r-face
    wr_hi = np.roll(w[0], -1, axis=1)              # the wall face for i = nr - 1 (zero)
    return (rip * wr_hi - ri * w[0]) / (rc * h) + (np.roll(w[1], -1, axis=0) - w[1]) / h


def weighted_beta(beta, h):
    """beta'_r = r_i beta_r, beta'_z = r_c beta_z."""
    nz, nr = beta[0].shape
    ri, rc = radii(nr, h)
    return [beta[0] * ri[None, :], beta[1] * rc[None, :]]


def curvature_total(X, nrm, fs_plane, sigma, axis_x, h):
    """f = sigma kappa_1 + sigma kappa_2 with kappa_2 = -n_r / r (eq curv_ax)."""
    X = np.asarray(X)
    r = X[:, 0] - axis_x
    k1 = np.asarray(fs_plane) / sigma
    # within a quarter cell of the axis n_r / r is rounding noise over a tiny
    # radius (the pole marker drifts off the axis by ~1e-9): take the limit
    # kappa_2 = kappa_1, exact to O(r^2) for a surface meeting the axis square
    on_axis = np.abs(r) < 0.25 * h
    k2 = np.where(on_axis, k1, -np.asarray(nrm)[:, 0] / np.where(on_axis, 1.0, r))
    return sigma * (k1 + k2)


def mirror_velocity(u, nr):
    """The doubled-plane velocity of the half-plane u (u_r odd, u_z even)."""
    nz = u[0].shape[0]
    ur = np.zeros((nz, 2 * nr))
    uz = np.zeros((nz, 2 * nr))
    ur[:, nr:] = u[0]
    ur[:, 1:nr] = -u[0][:, :0:-1]            # face x = nr h - i h  <-  -u_r(i), i = nr-1 .. 1
    uz[:, nr:] = u[1]
    uz[:, :nr] = u[1][:, ::-1]               # cell nr - 1 - i  <-  u_z(i)
    return [ur, uz]


def interface(Xd, fs_total, nr, nz, h, ds=None, nrm=None, conventional=False):
    """H and F of the half plane from the closed mirrored curve Xd. conventional:
    F is the marker force fs ds n spread by the discrete delta function on the
    doubled plane (the surface delta of an axisymmetric surface, restricted to
    the meridian plane, is the curve's delta)."""
    H2 = heaviside.heaviside_2d(Xd, (2 * nr, nz), h)
    if conventional:
        F2 = transfer.spread_delta(transfer.marker_forces(fs_total, ds, nrm), Xd, (2 * nr, nz), h)
    else:
        F2 = force.irrotational_force(H2, Xd, fs_total, h)
    H = H2[:, nr:].copy()
    F = [F2[0][:, nr:].copy(), F2[1][:, nr:].copy()]
    F[0][:, 0] = 0.0
    return H, F


def project(u_star, H, F, rho_in, rho_out, dt, h, p_prev=None, rtol=1e-10, max_cycles=100):
    """Projection of u_star with the face force F on the half plane."""
    rho = poisson.density(H, rho_in, rho_out)
    beta = poisson.face_beta(rho)
    beta[0][:, 0] = 0.0
    us = [u_star[0].copy(), u_star[1]]
    us[0][:, 0] = 0.0
    w = [us[d] / dt + beta[d] * F[d] for d in range(2)]
    nz, nr = H.shape
    _, rc = radii(nr, h)
    b = rc[None, :] * divergence(w, h)
    b = b - b.mean()
    p, cycles, hist = poisson.mg_solve(b, weighted_beta(beta, h), h, p0=p_prev, rtol=rtol,
                                       max_cycles=max_cycles)
    g = poisson.gradient(p, h)
    u = [us[d] + dt * beta[d] * (F[d] - g[d]) for d in range(2)]
    return dict(p=p, u=u, b=b, beta=beta, cycles=cycles, hist=hist)


def project_step(nr, nz, h, rho_in, rho_out, sigma, dt, u_star, Xd, rtol=1e-10, p_prev=None, conventional=False):
    """One axisymmetric projection step: markers (closed mirrored curve in the
    doubled plane) advanced with the interpolated velocity and relocated on the
    least-squares B-spline, f from eq curv_ax, H and F, projection."""
    ud = mirror_velocity(u_star, nr)
    U = transfer.interp(ud, Xd, h)
    Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in Xd], [tuple(v) for v in U], dt, h, sigma)
    Xn, fs, nrm = np.array(Xn), np.array(fs), np.array(nrm)
    ft = curvature_total(Xn, nrm, fs, sigma, nr * h, h)
    H, F = interface(Xn, ft, nr, nz, h, np.array(ds), nrm, conventional)
    out = project(u_star, H, F, rho_in, rho_out, dt, h, p_prev=p_prev, rtol=rtol)
    out.update(U=U, X=Xn, fs=ft, H=H, F=F)
    return out


# ----------------------------------------------------------------------------
# Momentum predictor in the meridian plane (eq ns1_new with eqs ad_bf, cr_ni
# written on the annular control volumes; no swirl)
# ----------------------------------------------------------------------------
# Control volumes (per radian): u_r of face (i, k) spans r in [r_i - h/2,
# r_i + h/2], volume r_i h^2; u_z of face (i, k) is the cell's column, volume
# r_c h^2. Fluxes through each side carry its radius as area factor.
#   C_r = rho_f { [r_c(i) ur_c(i)^2 - r_c(i-1) ur_c(i-1)^2] / (r_i h)
#                 + [uz_e ur_e |top - |bottom] / h },
#   C_z = rho_f { [r_{i+1} ur_e uz_e |right - r_i ur_e uz_e |left] / (r_c h)
#                 + [uz_c(k)^2 - uz_c(k-1)^2] / h },
# with cell means ur_c(i) = (u_r(i) + u_r(i+1))/2, uz_c(k) = (u_z(k) + u_z(k+1))/2,
# edge values the means of the two faces meeting there, and rho_f the mean of
# the two cells of the face (the density outside the divergence, as in the
# planar predictor). The viscous stress is the vector Laplacian form of
# div(mu grad u) per component, with the hoop term of u_r:
#   D_r = [r_c(i) mu(i) (u_r(i+1) - u_r(i)) - r_c(i-1) mu(i-1) (u_r(i) - u_r(i-1))] / (r_i h^2)
#         + [mu_e (u_r(k+1) - u_r(k)) |top - mu_e (u_r(k) - u_r(k-1)) |bottom] / h^2
#         - mu_f u_r / r_i^2,       mu_f = (mu(i-1) + mu(i)) / 2,
#   D_z = [r_{i+1} mu_e (u_z(i+1) - u_z(i)) |right - r_i mu_e (u_z(i) - u_z(i-1)) |left] / (r_c h^2)
#         + [mu(k) (u_z(k+1) - u_z(k)) - mu(k-1) (u_z(k) - u_z(k-1))] / h^2.
# Boundaries: u_r = 0 on the axis and the outer wall (face column 0); the outer
# wall is free of shear (the right edge of the last column carries no D_z flux);
# the axis edges have zero radius. Readings: the paper only says the planar
# schemes are used in cylindrical coordinates.
def advection(u, rho, h):
    ur, uz = u
    nz, nr = ur.shape
    ri, rc = radii(nr, h)
    R = lambda a, s: np.roll(a, -s, axis=1)      # value at i + s
    Z = lambda a, s: np.roll(a, -s, axis=0)      # value at k + s
    # C_r on face (i, k)
    urc = 0.5 * (ur + R(ur, 1))                  # cell i mean (wall face of the last column is 0)
    rcv = rc[None, :]
    flux_c = rcv * urc * urc                     # at cell i
    radial = (flux_c - R(flux_c, -1)) / np.where(ri > 0, ri, 1.0)[None, :]
    # top edge of face (i, k): between cells (i-1, k), (i, k), (i-1, k+1), (i, k+1)
    uz_e = 0.5 * (Z(uz, 1) + Z(R(uz, -1), 1))
    ur_e = 0.5 * (ur + Z(ur, 1))
    ftop = uz_e * ur_e
    Cr = 0.5 * (rho + R(rho, -1)) * (radial + ftop - Z(ftop, -1)) / h
    Cr[:, 0] = 0.0
    # C_z on face (i, k): right edge between cells (i, k-1), (i+1, k-1), (i, k), (i+1, k)
    ur_e2 = 0.5 * (R(ur, 1) + Z(R(ur, 1), -1))
    uz_e2 = 0.5 * (uz + R(uz, 1))
    rip = (ri + h)[None, :]
    fr = rip * ur_e2 * uz_e2                     # right edge (zero at the wall: u_r = 0 there)
    fl = R(fr, -1) * (ri > 0)[None, :]           # left edge = right edge of column i - 1; zero on the axis
    uzc = 0.5 * (uz + Z(uz, 1))
    fz = uzc * uzc
    Cz = 0.5 * (rho + Z(rho, -1)) * ((fr - fl) / rcv + fz - Z(fz, -1)) / h
    return [Cr, Cz]


def _visc_coefs(mu, h):
    """Per component the coefficients (c_lo, c_hi) along r and z and the
    diagonal extra term, such that D x = sum c_hi (x_hi - x) - c_lo (x - x_lo) - extra x."""
    nz, nr = mu.shape
    ri, rc = radii(nr, h)
    R = lambda a, s: np.roll(a, -s, axis=1)
    Z = lambda a, s: np.roll(a, -s, axis=0)
    rsafe = np.where(ri > 0, ri, 1.0)[None, :]
    h2 = h * h
    # u_r
    r_hi = rc[None, :] * mu / (rsafe * h2)
    r_lo = R(rc[None, :] * mu, -1) / (rsafe * h2)
    e_top = 0.25 * (mu + R(mu, -1) + Z(mu, 1) + Z(R(mu, -1), 1))
    z_hi = e_top / h2
    z_lo = Z(e_top, -1) / h2
    mu_f = 0.5 * (mu + R(mu, -1))
    extra = mu_f / (rsafe * rsafe)
    cr = dict(r=(r_lo, r_hi), z=(z_lo, z_hi), extra=extra)
    # u_z
    e_right = 0.25 * (mu + R(mu, 1) + Z(mu, -1) + Z(R(mu, 1), -1))
    last = np.zeros(nr, dtype=bool)
    last[-1] = True
    rhi = np.where(last[None, :], 0.0, (ri + h)[None, :] * e_right) / (rc[None, :] * h2)
    rlo = np.where((ri > 0)[None, :], ri[None, :] * R(e_right, -1), 0.0) / (rc[None, :] * h2)
    cz = dict(r=(rlo, rhi), z=(Z(mu, -1) / h2, mu / h2), extra=np.zeros_like(mu))
    return cr, cz


def viscous(u, mu, h):
    R = lambda a, s: np.roll(a, -s, axis=1)
    Z = lambda a, s: np.roll(a, -s, axis=0)
    out = []
    for x, co in zip(u, _visc_coefs(mu, h)):
        (rlo, rhi), (zlo, zhi) = co["r"], co["z"]
        D = (rhi * (R(x, 1) - x) - rlo * (x - R(x, -1)) + zhi * (Z(x, 1) - x) - zlo * (x - Z(x, -1))
             - co["extra"] * x)
        out.append(D)
    out[0][:, 0] = 0.0
    return out


def _matrix(co, shape):
    import scipy.sparse as sp
    nz, nr = shape
    N = nz * nr
    idx = np.arange(N).reshape(shape)
    (rlo, rhi), (zlo, zhi) = co["r"], co["z"]
    rows = [idx] * 5
    cols = [idx, np.roll(idx, -1, axis=1), np.roll(idx, 1, axis=1), np.roll(idx, -1, axis=0),
            np.roll(idx, 1, axis=0)]
    vals = [-(rhi + rlo + zhi + zlo + co["extra"]), rhi, rlo, zhi, zlo]
    return sp.csr_matrix((np.concatenate([v.ravel() for v in vals]),
                          (np.concatenate([r.ravel() for r in rows]),
                           np.concatenate([c.ravel() for c in cols]))), shape=(N, N))


def predict(u, rho_n, rho_np1, mu, dt, h, adv_prev=None, f_body=None):
    """u* of eq ns1_new on the meridian plane (Adams-Bashforth advection, Crank-
    Nicolson viscous stress, system solved exactly); u_r stays zero on face
    column 0. Returns (u_star, C(u^n))."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    adv = advection(u, rho_n, h)
    ab = adv if adv_prev is None else [1.5 * a - 0.5 * b for a, b in zip(adv, adv_prev)]
    vis = viscous(u, mu, h)
    shape = u[0].shape
    cos = _visc_coefs(mu, h)
    out = []
    for d in range(2):
        ax = 1 if d == 0 else 0
        rf = 0.5 * (rho_np1 + np.roll(rho_np1, 1, axis=ax))
        g = rf / dt * u[d] - ab[d] + 0.5 * vis[d]
        if f_body is not None and f_body[d] is not None:
            g = g + f_body[d]
        M = sp.diags(rf.ravel() / dt) - 0.5 * _matrix(cos[d], shape)
        if d == 0:
            # face column 0 is fixed at zero: identity rows, and no coupling into it
            fix = np.zeros(shape, dtype=bool)
            fix[:, 0] = True
            f = fix.ravel()
            M = M.tolil()
            M[f, :] = 0.0
            M = M.tocsr()
            M = M + sp.diags(f.astype(np.float64))
            g = np.where(fix, 0.0, g)
        out.append(spla.spsolve(M.tocsc(), g.ravel()).reshape(shape))
    return out, adv


def flow_step(nr, nz, h, rho_in, rho_out, mu_in, mu_out, sigma, dt, u, Xd, H_prev, adv_prev=None,
              p_prev=None, rtol=1e-10, gravity=0.0, frame_a=0.0, mass_target=None, conventional=False):
    """One step of the full axisymmetric method: markers advanced with u^n and
    relocated (eq curv_ax), H^{n+1} and F, rho^n from H_prev, the predictor, the
    projection of u*."""
    ud = mirror_velocity(u, nr)
    U = transfer.interp(ud, Xd, h)
    Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in Xd], [tuple(v) for v in U], dt, h, sigma)
    Xn, fs, nrm = np.array(Xn), np.array(fs), np.array(nrm)
    if mass_target is not None:
        from . import dynamics
        Xn, _ = dynamics.mass_correct(Xn, nrm, mass_target, nr * h, h)
    ft = curvature_total(Xn, nrm, fs, sigma, nr * h, h)
    H, F = interface(Xn, ft, nr, nz, h, np.array(ds), nrm, conventional)
    rho_n = poisson.density(H_prev, rho_in, rho_out)
    rho1 = poisson.density(H, rho_in, rho_out)
    mu = poisson.density(H, mu_in, mu_out)
    f_body = None
    if gravity != 0.0 or frame_a != 0.0:
        from . import dynamics
        _, rc = radii(nr, h)
        rho_mean = float(np.sum(rho1 * rc[None, :]) / (nz * np.sum(rc)))
        rf = 0.5 * (rho1 + np.roll(rho1, 1, axis=0))
        f_body = [None, dynamics.body_force(rf, rho_mean, gravity, frame_a)]
    u_star, adv = predict(u, rho_n, rho1, mu, dt, h, adv_prev, f_body)
    out = project(u_star, H, F, rho_in, rho_out, dt, h, p_prev=p_prev, rtol=rtol)
    out.update(U=U, X=Xn, fs=ft, H=H, F=F, u_star=u_star, adv=adv)
    return out
