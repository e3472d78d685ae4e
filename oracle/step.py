"""One projection step composed from the oracle parts.

Order (Section 2.1 fractional step with eq ns2_new, Section 2.2 transfer,
Sections 3.2 and 4 interface treatment):
  1. U = interpolation of u* to the markers (eq jump_condu);
  2. 2D: markers advanced by dt U and relocated on the least-squares B-spline,
     giving sigma*kappa, arc element and normals (Section 4); 3D: the surface
     is static and its curvature force comes from the cotangent formula;
  3. H from the offset polygons / polyhedra (Section 3.2);
  4. face force: irrotational f grad_h H (eq delta_hea_xy) or conventional
     delta-function spreading (eq delta_vec);
  5. rho from H (eq indicator), beta = 1/rho on faces;
  6. b = div(u*/dt + beta F), mean removed (eqs ps, ns2_new);
  7. multigrid solve (FP64, or float32 V-cycles inside FP64 defect correction);
  8. u^{n+1} = u* + dt beta (F - grad p) (eq ns2_new).
"""
import numpy as np

from . import bspline, force, heaviside, poisson, surface3d, transfer


def surface_forces(dim, X, tris, sigma, U=None, dt=0.0, h=None):
    if dim == 2:
        N = len(X)
        Uz = np.zeros((N, 2)) if U is None else U
        Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in X], [tuple(u) for u in Uz], dt, h, sigma)
        return np.array(Xn), np.array(fs), np.array(ds), np.array(nrm)
    fs, ds, nrm, _ = surface3d.surface_geometry(X, tris, sigma)
    return np.asarray(X, dtype=np.float64), fs, ds, nrm


def project_step(dim, n, h, rho_in, rho_out, sigma, dt, u_star, X, tris=None, p_prev=None,
                 mode="irrot", precision="fp64", rtol=1e-10, max_cycles=100, fixed_cycles=None,
                 surface=None):
    U = transfer.interp(u_star, X, h)
    if surface is None:
        Xn, fs, ds, nrm = surface_forces(dim, X, tris, sigma, U, dt, h)
    else:
        Xn, fs, ds, nrm = surface
    if dim == 2:
        H = heaviside.heaviside_2d(Xn, n, h)
    else:
        H = heaviside.heaviside_3d(Xn, tris, n, h, nrm=nrm)
    if mode == "irrot":
        F = force.irrotational_force(H, Xn, fs, h, tris)
    else:
        F = transfer.spread_delta(transfer.marker_forces(fs, ds, nrm), Xn, n, h)
    rho = poisson.density(H, rho_in, rho_out)
    beta = poisson.face_beta(rho)
    b = poisson.rhs(u_star, F, beta, dt, h)
    solve = poisson.mg_solve if precision == "fp64" else poisson.mg_solve_mixed
    p, cycles, hist = solve(b, beta, h, p0=p_prev, rtol=rtol, max_cycles=max_cycles,
                            fixed_cycles=fixed_cycles)
    u_new = poisson.velocity_update(u_star, F, beta, p, dt, h)
    return dict(U=U, X=Xn, fs=fs, ds=ds, nrm=nrm, H=H, F=F, beta=beta, b=b, p=p, u=u_new,
                cycles=cycles, hist=hist)
