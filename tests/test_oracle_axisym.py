"""Oracle pins for the axisymmetric projection (Section 2.1 in cylindrical
coordinates, eq curv_ax, Table staticdrop_axis).

* the r-weighted operator maps p = r^2 to 4 r_c (the exact axisymmetric
  Laplacian of r^2), the axis cell included, away from the outer wall;
* a drop on the axis with a constant face value f: the projection gives
  p = f H + C and u = 0 exactly (the discrete force is the weighted
  gradient's balance);
* any projected field has zero annular divergence;
* eq curv_ax on a relocated circle about the axis is 2/R (sphere);
* the static drop of Table staticdrop_axis (D = 0.4 on the axis, dx = 0.02,
  rho 1 / 0.01, one step of 1e-3): the pressure jump's error falls within the
  band of the paper's errors.
"""
import json
import os

import numpy as np

from oracle import axisym, bspline, diag, poisson
from paper_1807_10504_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_operator_on_r_squared():
    nr, nz, h = 16, 8, 0.1
    ri, rc = axisym.radii(nr, h)
    p = np.broadcast_to(rc[None, :] ** 2, (nz, nr)).copy()
    beta = [np.ones((nz, nr)), np.ones((nz, nr))]
    beta[0][:, 0] = 0.0
    Ap = poisson.apply_A(p, axisym.weighted_beta(beta, h), h)
    lap = Ap / rc[None, :]
    assert np.abs(lap[:, :-1] - 4.0).max() <= 1e-11
    # the outer wall column sees only its inner face
    assert np.all(lap[:, -1] < 0.0)


def _drop(nr, nz, h, n=128, R=0.2):
    Xd = W.circle_markers(n, R, centre=(nr * h, 0.5 * nz * h))
    return Xd


def test_constant_f_gives_f_times_H():
    nr, nz, h = 32, 64, 0.02
    Xd = _drop(nr, nz, h)
    f = 10.0
    H, F = axisym.interface(Xd, np.full(len(Xd), f), nr, nz, h)
    zero = [np.zeros((nz, nr)), np.zeros((nz, nr))]
    out = axisym.project(zero, H, F, 1.0, 0.01, 1e-3, h, rtol=1e-13)
    d = out["p"] - f * H
    assert np.ptp(d) <= 1e-9 * f
    assert max(np.abs(c).max() for c in out["u"]) <= 1e-12
    assert abs(diag.pressure_jump(out["p"], H) - f) <= 1e-9 * f


def test_projection_is_divergence_free():
    nr, nz, h = 32, 32, 1.0 / 32
    rng = np.random.default_rng(9)
    u = [rng.standard_normal((nz, nr)), rng.standard_normal((nz, nr))]
    u[0][:, 0] = 0.0
    Xd = W.circle_markers(96, 0.25, centre=(nr * h, 0.5))
    H, F = axisym.interface(Xd, np.full(len(Xd), 8.0), nr, nz, h)
    out = axisym.project(u, H, F, 1.0, 1e-3, 1e-3, h, rtol=1e-13)
    div_before = np.abs(axisym.divergence(u, h)).max()
    div_after = np.abs(axisym.divergence(out["u"], h)).max()
    assert div_after <= 1e-8 * div_before
    assert np.all(out["u"][0][:, 0] == 0.0)


def test_curvature_of_sphere_meridian():
    nr, nz, h, R = 32, 64, 0.02, 0.2
    Xd = _drop(nr, nz, h, n=128, R=R)
    Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in Xd], [(0.0, 0.0)] * len(Xd), 0.0, h, 1.0)
    ft = axisym.curvature_total(np.array(Xn), np.array(nrm), np.array(fs), 1.0, nr * h, h)
    assert np.abs(ft - 2.0 / R).max() < 0.02 * (2.0 / R)


def test_static_drop_axis_table_band():
    g = GOLD["static_drop_axis_table"]
    h = g["dx"][0]
    nr, nz = 32, 64
    Xd = W.circle_markers(int(round(2 * np.pi * 0.2 / (0.63 * h))) // 4 * 4, 0.2,
                          centre=(nr * h, 0.5 * nz * h))
    zero = [np.zeros((nz, nr)), np.zeros((nz, nr))]
    out = axisym.project_step(nr, nz, h, 1.0, 0.01, 1.0, 1e-3, zero, Xd, rtol=1e-12)
    err = abs(diag.pressure_jump(out["p"], out["H"]) - 10.0)
    print(f"axisymmetric static drop at dx = {h}: |dP - 10| = {err:.3e} (paper: new {g['new'][0]}, "
          f"conventional {g['conventional'][0]})")
    assert err < 5.0 * max(g["conventional"])
