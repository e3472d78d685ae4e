"""Oracle pins for the local least-squares surface reconstruction (the 3D
counterpart of Section 4's least-squares B-spline).

* on a quadric patch z = a x^2 + b x y + c y^2 sampled on a centrally symmetric
  mesh, the apex's fit is exact: curvature sum 2 (a + c), normal along z, the
  apex not moved;
* on icospheres the curvature sum converges to 2/R at second order, the
  normals to the radial ones, and the moved vertices stay on the sphere to
  fourth order;
* radial noise on the vertices is smoothed (the reconstruction is a filter,
  as the B-spline is in 2D).
"""
import numpy as np

from oracle import surface3d
from paper_1807_10504_amd import workloads as W


def _quadric_patch(a, b, c, s=0.05, k=3):
    idx = np.arange(-k, k + 1)
    gx, gy = np.meshgrid(idx * s, idx * s, indexing="ij")
    V = np.stack([gx.ravel(), gy.ravel(), (a * gx * gx + b * gx * gy + c * gy * gy).ravel()], axis=1)
    m = 2 * k + 1
    T = []
    for i in range(m - 1):
        for j in range(m - 1):
            p, q, r, t = i * m + j, (i + 1) * m + j, (i + 1) * m + j + 1, i * m + j + 1
            # clockwise seen from +z: the "inward" normal of the patch is +z
            T += [[p, t, r], [p, r, q]]
    return V, np.array(T), (m * m) // 2


def test_quadric_apex_exact():
    for a, b, c in ((1.3, 0.4, -0.7), (2.0, 0.0, 2.0), (-0.5, 1.1, 0.9)):
        V, T, apex = _quadric_patch(a, b, c)
        Vn, fs, ds, nrm = surface3d.lsq_reconstruct(V, T, 1.0)
        assert abs(fs[apex] - 2 * (a + c)) <= 1e-10 * (1 + abs(a + c))
        assert np.abs(nrm[apex] - np.array([0.0, 0.0, 1.0])).max() <= 1e-12
        assert np.abs(Vn[apex] - V[apex]).max() <= 1e-15


def test_sphere_second_order():
    R = 0.25
    ek, en, er = [], [], []
    for level in (2, 3, 4):
        V, T = W.sphere_mesh(level, R, seed=3)
        Vn, fs, ds, nrm = surface3d.lsq_reconstruct(V, T, 1.0)
        r = np.linalg.norm(Vn - 0.5, axis=1)
        ek.append(np.abs(fs - 2 / R).max() * R / 2)
        en.append(np.abs(nrm - (0.5 - Vn) / r[:, None]).max())
        er.append(np.abs(r - R).max() / R)
    assert 3.0 < ek[0] / ek[1] < 5.5 and 3.0 < ek[1] / ek[2] < 5.5, ek
    assert en[0] / en[1] > 3.0 and en[1] / en[2] > 3.0, en
    assert er[0] / er[1] > 10 and er[1] / er[2] > 10, er
    assert ek[2] < 0.01


def test_noise_is_smoothed():
    R = 0.25
    V, T = W.sphere_mesh(4, R, seed=3)
    rng = np.random.default_rng(6)
    d = V - 0.5
    Vj = 0.5 + d * (1 + 2e-3 * rng.uniform(-1, 1, len(V)))[:, None]
    Vn, fs, ds, nrm = surface3d.lsq_reconstruct(Vj, T, 1.0)
    before = np.sqrt(np.mean((np.linalg.norm(Vj - 0.5, axis=1) - R) ** 2))
    after = np.sqrt(np.mean((np.linalg.norm(Vn - 0.5, axis=1) - R) ** 2))
    assert after < 0.5 * before
