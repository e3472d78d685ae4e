"""Oracle pins for gravity, the non-inertial frame and the mass correction.

* the enclosed area / volume of revolution and the vertical centroid of
  polygons against closed forms (circle, sphere by revolution, an off-axis
  square's annulus) and their convergence to pi R^2 and 4/3 pi R^3;
* the mass correction returns a shrunk or grown drop to its target to 1e-12
  with a displacement equal to the shrinkage, and leaves a drop within the
  trigger untouched;
* the frame acceleration restores: zero at rest on the initial centre,
  opposite to a displacement and to a velocity;
* the body force has no net force on a periodic box; a resting fluid under
  the predictor takes exactly dt (rho_f - rho_mean) g / rho_f.
"""
import numpy as np

from oracle import axisym, dynamics, flow
from paper_1807_10504_amd import workloads as W


def test_area_volume_centroid_closed_forms():
    sq = np.array([[1.0, 0.0], [3.0, 0.0], [3.0, 2.0], [1.0, 2.0]])
    A, cx, cy = dynamics.polygon_area_centroid(sq)
    assert (A, cx, cy) == (4.0, 2.0, 1.0)
    # the square revolved about x = 0: an annulus r in [1, 3], height 2
    V, zc = dynamics.revolution_volume_centroid(sq, 0.0)
    assert abs(V - np.pi * (9 - 1) * 2) <= 1e-12 * V and abs(zc - 1.0) <= 1e-14
    for n in (200, 400):
        X = W.circle_markers(n, 0.3, centre=(1.0, 0.7))
        A, _, cy = dynamics.polygon_area_centroid(X)
        V, zc = dynamics.revolution_volume_centroid(X, 1.0)
        # inscribed polygons: errors fall as 1/n^2
        assert abs(A - np.pi * 0.09) <= 2.5 * (np.pi * 0.09) * (2 * np.pi / n) ** 2 / 6
        assert abs(V - 4 / 3 * np.pi * 0.027) <= 4 / 3 * np.pi * 0.027 * 2 * (2 * np.pi / n) ** 2
        assert abs(cy - 0.7) <= 1e-12 and abs(zc - 0.7) <= 1e-12


def test_mass_correction():
    R, n = 0.25, 256
    X0 = W.circle_markers(n, R)
    nrm = (np.array([0.5, 0.5]) - X0) / R                 # toward the drop
    target, _ = dynamics.measure(X0)
    for s in (1e-4, -2e-4):
        X = X0 + s * nrm                                    # shrunk (s > 0) or grown
        Xc, delta = dynamics.mass_correct(X, nrm, target, None, h=1 / 64)
        A, _ = dynamics.measure(Xc)
        assert abs(A - target) <= 1e-12 * target
        assert abs(delta + s) <= 1e-9
    # axisymmetric: the same on the volume of revolution
    Xd = W.circle_markers(n, R, centre=(1.0, 0.5))
    nd = (np.array([1.0, 0.5]) - Xd) / R
    Vt, _ = dynamics.measure(Xd, 1.0)
    Xc, delta = dynamics.mass_correct(Xd + 3e-5 * nd, nd, Vt, 1.0, h=1 / 64)
    assert abs(dynamics.measure(Xc, 1.0)[0] - Vt) <= 1e-12 * Vt and abs(delta + 3e-5) <= 1e-9
    # within the trigger: untouched
    Xs, delta = dynamics.mass_correct(X0 + 1e-9 * nrm, nrm, target, None, h=1 / 64)
    assert delta == 0.0


def test_frame_acceleration_restores():
    dt = 1e-3
    assert dynamics.frame_acceleration(1.0, 1.0, 1.0, dt) == 0.0
    assert dynamics.frame_acceleration(1.0, 0.99, 0.99, dt) > 0.0     # below the start: push up
    assert dynamics.frame_acceleration(1.0, 1.0, 0.999, dt) > 0.0     # moving down: push up
    assert dynamics.frame_acceleration(1.0, 1.01, 1.01, dt) < 0.0


def test_body_force_net_zero_and_resting_fluid():
    n = 16
    H = np.zeros((n, n))
    H[4:10, 5:11] = 1.0
    rho = 0.01 + 0.99 * H
    rf = flow.face_density(rho, 2, 1)
    fb = dynamics.body_force(rf, rho.mean(), -9.81, 0.0)
    assert abs(fb.sum()) <= 1e-12 * np.abs(fb).sum()
    # a resting fluid, no viscosity: u* = dt f / rho_f on the vertical faces
    zero = np.zeros((n, n))
    dt = 1e-3
    us, _ = flow.predict([zero, zero], rho, rho, zero, dt, 1.0 / n, f_body=[None, fb])
    assert np.abs(us[0]).max() == 0.0
    assert np.abs(us[1] - dt * fb / rf).max() <= 1e-15
    # axisymmetric: the volume-weighted mean makes the r-weighted total vanish
    nz, nr, h = 12, 10, 0.1
    Ha = np.zeros((nz, nr))
    Ha[3:8, 0:4] = 1.0
    ra = 0.1 + 0.9 * Ha
    _, rc = axisym.radii(nr, h)
    rho_mean = np.sum(ra * rc[None, :]) / (nz * np.sum(rc))
    rfa = 0.5 * (ra + np.roll(ra, 1, axis=0))
    fa = dynamics.body_force(rfa, rho_mean, -1.0, 0.0)
    assert abs(np.sum(fa * rc[None, :])) <= 1e-12 * np.sum(np.abs(fa) * rc[None, :])


def test_mesh_volume_centroid_and_correction():
    # a unit cube's 12 outward triangles: volume 1, centroid at its centre
    Vc = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]],
                  dtype=float) + np.array([0.2, 0.3, 0.1])
    Tc = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                   [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]])
    vol, cy = dynamics.mesh_volume_centroid(Vc, Tc)
    assert abs(vol - 1.0) <= 1e-14 and abs(cy - 0.8) <= 1e-14
    # icospheres: inscribed volumes converge to 4/3 pi R^3 at second order, centroid exact
    R = 0.25
    errs = []
    for level in (3, 4):
        V, T = W.sphere_mesh(level, R, seed=3)
        vol, cy = dynamics.mesh_volume_centroid(V, T)
        errs.append(abs(vol - 4 / 3 * np.pi * R ** 3))
        assert abs(cy - 0.5) <= 1e-12
    assert 3.5 < errs[0] / errs[1] < 4.5
    # the correction restores a shrunk mesh along the (inward) normals
    from oracle import surface3d
    V, T = W.sphere_mesh(3, R, seed=3)
    target, _ = dynamics.measure(V, T=T)
    nrm = surface3d.vertex_normals(V, T)
    Vc2, delta = dynamics.mass_correct(V + 2e-4 * nrm, nrm, target, None, h=1 / 64, T=T)
    assert abs(dynamics.measure(Vc2, T=T)[0] - target) <= 1e-12 * target and abs(delta + 2e-4) <= 1e-9
