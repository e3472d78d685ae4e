"""Oracle pins worked by hand: the nearest-element face value, the
diagnostics, and the least-squares B-spline solve.

Face value f (Section 3.2 defers it; the reading: sigma*kappa at the foot
point on the nearest segment / triangle, interpolated linearly /
barycentrically, exact distance ties to the lower index). With the marker
values taken from a linear function g(x) = g0 + w . x, any correct foot
point and interpolation return g at the foot point exactly (up to rounding),
so the expected value is g at the foot point found by hand; a wrong foot
parameter, swapped weights or a wrong tie rule return g elsewhere.

Diagnostics (eq tke, eq sd_pres_diff, the force ratio of the
large-deformation figure, the index-form curl of Section 3.2) on small
fields with values worked out by hand.

Least squares (eq bspline_ls): points sampled from a closed cubic at known
parameters (three per span) are fitted back to its own control points; for
noisy points the residual is orthogonal to every basis function (the normal
equations).
"""
import math

import numpy as np
import pytest

from oracle import bspline, diag, force

W_LIN = np.array([0.7, -1.3, 0.45])
G0 = 2.0


def g_lin(x):
    x = np.asarray(x, dtype=np.float64)
    return G0 + float(W_LIN[: len(x)] @ x)


# ----------------------------------------------------------------------------
# 2D polyline
def _poly_fs(X):
    return np.array([g_lin(x) for x in X])


SQUARE = np.array([[0.25, 0.25], [0.75, 0.25], [0.75, 0.75], [0.25, 0.75]])


@pytest.mark.parametrize("p,foot", [
    ((0.5, 0.2), (0.5, 0.25)),        # below the bottom edge: interior foot
    ((0.8, 0.375), (0.75, 0.375)),    # right of the right edge
    ((0.6, 0.7), (0.6, 0.75)),        # inside, nearest the top edge
    ((0.2, 0.1), (0.25, 0.25)),       # beyond a corner: the vertex
])
def test_nearest_on_polyline_square(p, foot):
    fs = _poly_fs(SQUARE)
    got = force.nearest_on_polyline(np.array(p), SQUARE, fs)
    assert abs(got - g_lin(foot)) <= 1e-15 * abs(g_lin(foot))


def test_nearest_on_polyline_sloped_segment():
    # triangle with a sloped side from (0.2, 0.2) to (0.8, 0.5); the point lies
    # 0.01 off it along the inward normal above t = 1/3, i.e. the foot (0.4, 0.3)
    X = np.array([[0.2, 0.2], [0.8, 0.5], [0.3, 0.9]])
    d = np.array([0.6, 0.3])
    nrm = np.array([-d[1], d[0]]) / np.linalg.norm(d)
    foot = np.array([0.4, 0.3])
    got = force.nearest_on_polyline(foot + 0.01 * nrm, X, _poly_fs(X))
    assert abs(got - g_lin(foot)) <= 1e-14


def test_nearest_on_polyline_exact_tie_goes_to_lower_index():
    # rectangle [0.25, 0.75] x [0.375, 0.625]: the centre is 0.125 from the
    # bottom edge (index 0) and the top edge (index 2), exactly (dyadic values)
    X = np.array([[0.25, 0.375], [0.75, 0.375], [0.75, 0.625], [0.25, 0.625]])
    lo, hi = g_lin((0.5, 0.375)), g_lin((0.5, 0.625))   # 0.325 apart
    got = force.nearest_on_polyline(np.array([0.5, 0.5]), X, _poly_fs(X))
    assert abs(got - lo) <= 1e-15
    # the same curve listed from the top edge: now the top edge wins
    Xr = np.roll(X, -2, axis=0)
    assert abs(force.nearest_on_polyline(np.array([0.5, 0.5]), Xr, _poly_fs(Xr)) - hi) <= 1e-15


# ----------------------------------------------------------------------------
# 3D mesh: the cube [0.25, 0.75]^3, vertex index x + 2y + 4z
LO, HI = 0.25, 0.75
CUBE_V = np.array([(x, y, z) for z in (LO, HI) for y in (LO, HI) for x in (LO, HI)])
CUBE_T = np.array([[0, 2, 3], [0, 3, 1], [4, 5, 7], [4, 7, 6], [0, 1, 5], [0, 5, 4],
                   [2, 6, 7], [2, 7, 3], [0, 4, 6], [0, 6, 2], [1, 3, 7], [1, 7, 5]])


def _mesh_fs(V):
    return np.array([g_lin(v) for v in V])


@pytest.mark.parametrize("p,foot", [
    ((0.45, 0.6, 0.2), (0.45, 0.6, 0.25)),    # below the bottom face: triangle interior
    ((0.3, 0.35, 0.8), (0.3, 0.35, 0.75)),    # above the top face
    ((0.81, 0.4, 0.55), (0.75, 0.4, 0.55)),   # right of the x = 0.75 face
    ((0.5, 0.2, 0.2), (0.5, 0.25, 0.25)),     # outside an edge: its foot
    ((0.2, 0.8, 0.1), (0.25, 0.75, 0.25)),    # outside a corner: the vertex
    ((0.6, 0.3, 0.45), (0.6, 0.25, 0.45)),    # inside, nearest the y = 0.25 face
])
def test_nearest_on_mesh_cube(p, foot):
    got = force.nearest_on_mesh(np.array(p), CUBE_V, CUBE_T, _mesh_fs(CUBE_V))
    assert abs(got - g_lin(foot)) <= 1e-14


def test_nearest_on_mesh_sloped_triangle():
    # a tetrahedron with one sloped face: the foot is worked out from the plane
    V = np.array([[0.2, 0.2, 0.2], [0.8, 0.25, 0.3], [0.3, 0.85, 0.35], [0.35, 0.4, 0.9]])
    T = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]])
    a, b, c = V[1], V[2], V[3]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n)
    foot = (a + b + c) / 3.0 + 0.05 * (b - a) - 0.02 * (c - a)   # inside face (1, 2, 3)
    p = foot + 0.01 * n                                           # just outside it
    got = force.nearest_on_mesh(p, V, T, _mesh_fs(V))
    assert abs(got - g_lin(foot)) <= 1e-14


# ----------------------------------------------------------------------------
# diagnostics
def test_tke_by_hand():
    # eq tke as printed: sum of u^2 + v^2 over the faces times the cell area
    h = 0.5
    u = np.full((4, 4), 1.0)
    v = np.full((4, 4), 2.0)
    assert diag.tke([u, v], h) == 20.0          # 16 cells x (1 + 4) x 0.25
    w = np.zeros((2, 2, 2))
    w[1, 0, 1] = 3.0
    assert diag.tke([w, w, w], 0.5) == 3 * 9.0 * 0.125


def test_force_ratio_by_hand():
    h = 0.5
    Fx = np.array([[1.0, 2.0], [3.0, 4.0]])     # sum 10 -> 2.5 after h^2
    Fy = np.array([[0.0, 0.0], [0.0, -1.0]])    # sum -1 -> -0.25
    Fs = np.array([[3.0, 4.0], [0.0, 1.0]])     # |F_s| = 5 and 1
    # |(2.5, -0.25)| / 6 = sqrt(6.3125) / 6
    assert abs(diag.force_ratio([Fx, Fy], Fs, h) - 0.418744817547) < 1e-11


def test_pressure_jump_by_hand():
    H = np.array([[0.0, 0.0, 0.0, 0.0], [0.0, 1.0, 1.0, 0.3], [0.0, 1.0, 1.0, 0.0], [0.0, 0.0, 0.0, 0.0]])
    p = np.where(H == 1.0, 5.0, 1.0)
    p[0, 0] = 3.0          # outside mean (3 + 10 x 1) / 11
    p[1, 3] = 100.0        # interface cell: excluded
    assert abs(diag.pressure_jump(p, H) - (5.0 - 13.0 / 11.0)) < 1e-14


def test_curl_by_hand():
    # 2D: one y-face force F_y[j=1, i=2] = 2: the node curl
    # (F_y[c] - F_y[c - e_x]) - (F_x[c] - F_x[c - e_y]) is +2 at c = (2, 1) and -2 at (3, 1)
    Fx = np.zeros((4, 4))
    Fy = np.zeros((4, 4))
    Fy[1, 2] = 2.0
    assert diag.curl_max([Fx, Fy]) == 2.0
    # a discrete gradient has zero curl
    p = np.random.default_rng(0).standard_normal((5, 6))
    g = [p - np.roll(p, 1, axis=1), p - np.roll(p, 1, axis=0)]
    assert diag.curl_max(g) <= 1e-15
    # 3D: F_z[k, j, i] = 1 at one face; curl in the (x, z) and (y, z) planes
    F3 = [np.zeros((3, 4, 5)) for _ in range(3)]
    F3[2][1, 2, 3] = 1.0
    assert diag.curl_max(F3) == 1.0


# ----------------------------------------------------------------------------
# least squares
def test_least_squares_recovers_control_points():
    rng = np.random.default_rng(7)
    g = 12
    th = 2 * np.pi * np.arange(g) / g
    cx = list(0.5 + 0.2 * np.cos(th) + 0.01 * rng.standard_normal(g))
    cy = list(0.5 + 0.2 * np.sin(th) + 0.01 * rng.standard_normal(g))
    C = bspline.ClosedCubic(cx, cy)
    v, X = [], []
    for s in range(g):
        for u in np.sort(rng.uniform(0.0, 1.0, 3)):
            v.append(s + u)
            X.append(C.point(s, u))
    fit = bspline.lsq_closed_cubic(X, v, g)
    assert max(abs(a - b) for a, b in zip(fit.cx, cx)) <= 1e-12
    assert max(abs(a - b) for a, b in zip(fit.cy, cy)) <= 1e-12


def test_least_squares_residual_orthogonal_to_basis():
    rng = np.random.default_rng(8)
    N, g = 70, 11
    th = 2 * np.pi * (np.arange(N) + 0.3 * rng.uniform(size=N)) / N
    X = [(0.5 + 0.25 * math.cos(t) + 1e-3 * rng.standard_normal(), 0.5 + 0.2 * math.sin(t)) for t in th]
    v = list(np.sort(rng.uniform(0.0, g, N)))
    fit = bspline.lsq_closed_cubic(X, v, g)
    # sum_k B_i(v_k) (X_k - C(v_k)) = 0 for every control point i
    acc = np.zeros((g, 2))
    for k in range(N):
        s = min(int(math.floor(v[k])), g - 1)
        u = v[k] - s
        B3, _ = bspline.cox_de_boor(u)
        px, py = fit.point(s, u)
        for r in range(4):
            acc[(s - 3 + r) % g] += B3[r] * np.array([X[k][0] - px, X[k][1] - py])
    assert np.max(np.abs(acc)) <= 1e-14
