"""Oracle pins: discrete Heaviside, irrotational force, static-drop closed form.

Pins: area/volume identities against shoelace / divergence-theorem formulas,
a closed form for the regular N-gon, hand integration for an axis-aligned
edge, the index-form curl identity of Section 3.2 (curl-free for constant f,
not for the conventional spread), and the static-drop identity
p = f H + C (u* = 0, constant f) that gives the Laplace jump exactly.
"""
import math

import numpy as np
import pytest

from oracle import diag, force, heaviside, kernel, poisson, transfer
from paper_1807_10504_amd import workloads as W


def _offset_area_sum(X, h):
    return sum(dH * heaviside.shoelace(heaviside.offset_polygon_2d(X, c * h))
               for c, dH in zip(kernel.OFFSETS, kernel.region_jumps()))


def test_h2d_area_identity_and_bounds():
    wl = W.static_drop_2d_64()
    H = heaviside.heaviside_2d(wl.X, wl.n, wl.h)
    tot = H.sum() * wl.h ** 2
    ref = _offset_area_sum(wl.X, wl.h)
    assert abs(tot - ref) <= 1e-12 * ref
    assert H.min() > -1e-14 and H.max() < 1.0 + 1e-14
    # outside the band H is 0 or 1 (to the rounding of the column sums)
    yy, xx = np.mgrid[0:64, 0:64]
    r = np.hypot((xx + 0.5) * wl.h - 0.5, (yy + 0.5) * wl.h - 0.5)
    assert np.all(np.abs(H[r < 0.25 - 3 * wl.h] - 1.0) < 1e-14)
    assert np.all(np.abs(H[r > 0.25 + 3 * wl.h]) < 1e-14)
    # and strictly between 0 and 1 on cells the interface crosses
    band = np.abs(r - 0.25) < 0.3 * wl.h
    assert np.all((H[band] > 0.2) & (H[band] < 0.8))


def test_h2d_regular_polygon_closed_form():
    # sum_m dH_m c_m = 0 and sum_m dH_m c_m^2 = 2(dH_1 2.25 + dH_2 0.25) h^2, so
    # sum_c H_c h^2 = A + (sum dH c^2) N tan(pi/N) for a regular N-gon.
    N, R, h = 40, 0.3, 1.0 / 64
    X = W.circle_markers(N, R)
    A = 0.5 * N * R * R * math.sin(2 * math.pi / N)
    j = kernel.region_jumps()
    c2 = 2 * (j[0] * 2.25 + j[1] * 0.25)
    assert abs(c2 - 0.613380) < 1e-6
    ref = A + c2 * h * h * N * math.tan(math.pi / N)
    H = heaviside.heaviside_2d(X, (64, 64), h)
    assert abs(H.sum() * h * h - ref) < 1e-13


def test_h2d_axis_aligned_edge_by_hand():
    # a large square whose left edge is at x = a; away from corners the cell
    # value is sum_m dH_m * |[x_c - h/2, x_c + h/2] ∩ (a - c_m h, inf)| / h
    h = 1.0 / 32
    a = 0.3 + 0.37 * h
    X = np.array([[a, 0.2], [0.8, 0.2], [0.8, 0.8], [a, 0.8]])
    H = heaviside.heaviside_2d(X, (32, 32), h)
    j = 16
    for i in range(5, 16):
        xc = (i + 0.5) * h
        ref = 0.0
        for c, dH in zip(kernel.OFFSETS, kernel.region_jumps()):
            lo = max(xc - h / 2, a + c * h)
            ref += dH * max(0.0, xc + h / 2 - lo) / h
        assert abs(H[j, i] - ref) < 1e-14


def test_irrotational_force_curl_free_and_conventional_not():
    # E2 setup (caption of the curl figure): circle R = 0.2, unit inward force
    n, h = (64, 64), 1.0 / 64
    X = W.circle_markers(200, 0.2)
    fs = np.ones(len(X))
    H = heaviside.heaviside_2d(X, n, h)
    F = force.irrotational_force(H, X, fs, h)
    fmax = max(np.abs(F[0]).max(), np.abs(F[1]).max())
    assert diag.curl_max(F) <= 1e-12 * fmax
    # telescoping: total grid force vanishes for constant f
    tot = diag.grid_force_sum(F, h)
    assert np.max(np.abs(tot)) < 1e-12
    # the conventional delta vector is rotational (Section 3.1)
    ds = np.full(len(X), 2 * math.pi * 0.2 / len(X))
    Fc = transfer.spread_delta(transfer.marker_forces(fs, ds, transfer.marker_normals_2d(X)), X, n, h)
    fcmax = max(np.abs(Fc[0]).max(), np.abs(Fc[1]).max())
    assert diag.curl_max(Fc) > 1e-3 * fcmax


def test_irrotational_force_points_inward():
    n, h = (64, 64), 1.0 / 64
    X = W.circle_markers(128, 0.25)
    H = heaviside.heaviside_2d(X, n, h)
    F = force.irrotational_force(H, X, np.full(128, 4.0), h)
    # on the left of the drop the x-force points to +x (toward the centre)
    assert F[0][32, 32 - 16 - 1:32 - 16 + 2].sum() > 0
    assert F[0][32, 32 + 16 - 1:32 + 16 + 2].sum() < 0


@pytest.mark.parametrize("rho_out", [1e-3, 1e-2])
def test_static_drop_closed_form(rho_out):
    """u* = 0 and constant f: p = f H + C makes F - grad p vanish on every face."""
    wl = W.static_drop_2d_64()
    f = 1.0 / 0.25
    H = heaviside.heaviside_2d(wl.X, wl.n, wl.h)
    F = force.irrotational_force(H, wl.X, np.full(len(wl.X), f), wl.h)
    beta = poisson.face_beta(poisson.density(H, 1.0, rho_out))
    u0 = [np.zeros(H.shape), np.zeros(H.shape)]
    b = poisson.rhs(u0, F, beta, wl.dt, wl.h)
    p, _, _ = poisson.mg_solve(b, beta, wl.h, rtol=1e-13)
    ref = f * H
    ref -= ref.mean()
    assert np.max(np.abs(p - ref)) < 1e-9 * f
    u = poisson.velocity_update(u0, F, beta, p, wl.dt, wl.h)
    assert max(np.abs(c).max() for c in u) < 1e-10
    assert abs(diag.pressure_jump(p, H) - f) < 1e-9


def test_h3d_volume_identity_and_bounds():
    V, T = W.sphere_mesh(2, 0.3, seed=5)
    n, h = (24, 24, 24), 1.0 / 24
    nrm = heaviside.vertex_normals(V, T)
    H = heaviside.heaviside_3d(V, T, n, h, nrm=nrm)
    tot = H.sum() * h ** 3
    ref = sum(dH * heaviside.mesh_volume(heaviside.offset_mesh(V, nrm, c * h), T)
              for c, dH in zip(kernel.OFFSETS, kernel.region_jumps()))
    assert abs(tot - ref) <= 1e-12 * ref
    assert H.min() > -1e-13 and H.max() < 1 + 1e-13
    # column sampling gives the same values as the full evaluation
    cols = [(12, 12), (5, 13), (18, 9)]
    Hc = heaviside.heaviside_3d(V, T, n, h, nrm=nrm, columns=cols)
    for (i, j) in cols:
        assert np.max(np.abs(Hc[(i, j)] - H[:, j, i])) < 1e-14


def test_h3d_axis_aligned_cube_by_hand():
    # closed cube mesh [a, b]^3 with vertex normals along the diagonals is not a
    # parallel offset, so test the zero-offset volume function directly
    a, b = 0.3 + 0.2 / 16, 0.7 - 0.33 / 16
    h = 1.0 / 16
    P = np.array([[a, a, a], [b, a, a], [b, b, a], [a, b, a],
                  [a, a, b], [b, a, b], [b, b, b], [a, b, b]])
    T = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                  [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]])
    vol = heaviside.mesh_column_volumes(P, T, (16, 16, 16), h)
    assert abs(heaviside.mesh_volume(P, T) - (b - a) ** 3) < 1e-15
    c = (np.arange(16) * h)
    ov = np.clip(np.minimum(c + h, b) - np.maximum(c, a), 0, None)
    ref = ov[:, None, None] * ov[None, :, None] * ov[None, None, :]
    assert np.max(np.abs(vol - ref)) < 1e-17


def test_irrotational_force_3d_curl_free():
    V, T = W.sphere_mesh(2, 0.3, seed=5)
    n, h = (16, 16, 16), 1.0 / 16
    nrm = heaviside.vertex_normals(V, T)
    H = heaviside.heaviside_3d(V, T, n, h, nrm=nrm)
    F = force.irrotational_force(H, V, np.full(len(V), 2.0 / 0.3), h, T)
    fmax = max(np.abs(c).max() for c in F)
    assert diag.curl_max(F) <= 1e-12 * fmax
    assert np.max(np.abs(diag.grid_force_sum(F, h))) < 1e-12 * fmax
