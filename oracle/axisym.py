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
on the axis; f = sigma (kappa_1 + kappa_2).
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
    on_axis = np.abs(r) < 1e-8 * h
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


def interface(Xd, fs_total, nr, nz, h):
    """H and F of the half plane from the closed mirrored curve Xd."""
    H2 = heaviside.heaviside_2d(Xd, (2 * nr, nz), h)
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


def project_step(nr, nz, h, rho_in, rho_out, sigma, dt, u_star, Xd, rtol=1e-10, p_prev=None):
    """One axisymmetric projection step: markers (closed mirrored curve in the
    doubled plane) advanced with the interpolated velocity and relocated on the
    least-squares B-spline, f from eq curv_ax, H and F, projection."""
    ud = mirror_velocity(u_star, nr)
    U = transfer.interp(ud, Xd, h)
    Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in Xd], [tuple(v) for v in U], dt, h, sigma)
    Xn, fs, nrm = np.array(Xn), np.array(fs), np.array(nrm)
    ft = curvature_total(Xn, nrm, fs, sigma, nr * h, h)
    H, F = interface(Xn, ft, nr, nz, h)
    out = project(u_star, H, F, rho_in, rho_out, dt, h, p_prev=p_prev, rtol=rtol)
    out.update(U=U, X=Xn, fs=ft, H=H, F=F)
    return out
