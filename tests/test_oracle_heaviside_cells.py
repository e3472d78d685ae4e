"""Oracle pin: the per-cell discrete Heaviside against an independent clipper.

The oracle computes H_c = sum_m dH_m |cell ∩ P_m| / h^dim (Section 3.2,
eqs new_hea and new_hea2; the three-polygon figure's caption H_ij = sum A_I H_I)
by column integrals of the offset boundaries. This file recomputes every cell
value by another route that shares nothing with it:

* offsets: 2D mitred offsets as the intersection of the two neighbouring
  edge lines moved by c along their inward normals (a 2 x 2 solve); 3D vertex
  normals as the angle-weighted sum of face normals, written here again;
* region increments dH_m from the closed-form profile evaluated here;
* overlaps: the offset polygon (polyhedron) is fanned into signed triangles
  (tetrahedra) from an interior point, each is clipped against the cell
  square (cube) by Sutherland-Hodgman, and the clipped area is the shoelace
  sum (the clipped volume the divergence-theorem sum over the clipped faces).

Cells are compared one by one to 1e-14. Cases reach the sloped pieces that
cross a cell partially, in both directions, and the 3D clip of a piece by the
cell's z-planes: a circle and a mode-2 curve in 2D, a seeded-rotation
level-2 icosphere in 3D, none axis-aligned.
"""
import math

import numpy as np
import pytest

from oracle import heaviside, kernel
from paper_1807_10504_amd import workloads as W


def _profile(q):
    return 0.5 + q / 4.0 + math.sin(math.pi * q / 2.0) / (2.0 * math.pi)


# region boundaries in grid units (negative = away from the drop) and the
# increments of the region values H(-2), H(-1), H(0), H(1), H(2) across them
BOUNDS = (-1.5, -0.5, 0.5, 1.5)
JUMPS = (_profile(-1.0) - 0.0, 0.5 - _profile(-1.0), _profile(1.0) - 0.5, 1.0 - _profile(1.0))


def test_region_constants_match_the_oracle():
    assert tuple(kernel.OFFSETS) == BOUNDS
    assert np.allclose(kernel.region_jumps(), JUMPS, rtol=0, atol=1e-16)


# ----------------------------------------------------------------------------
# 2D
def _mitred_offset(X, c):
    """Vertex k of the offset: the meeting point of edges (k-1, k) and (k, k+1)
    each moved by c along its left (inward for a counter-clockwise curve) normal."""
    N = len(X)
    out = np.empty_like(X)
    for k in range(N):
        p0, p1, p2 = X[k - 1], X[k], X[(k + 1) % N]
        ta, tb = p1 - p0, p2 - p1
        na = np.array([-ta[1], ta[0]]) / math.hypot(*ta)
        nb = np.array([-tb[1], tb[0]]) / math.hypot(*tb)
        # p1 + c na + s ta = p1 + c nb + t tb
        M = np.array([[ta[0], -tb[0]], [ta[1], -tb[1]]])
        s, _ = np.linalg.solve(M, c * (nb - na))
        out[k] = p1 + c * na + s * ta
    return out


def _clip2(poly, axis, value, keep_ge):
    out = []
    m = len(poly)
    for r in range(m):
        p, q = poly[r], poly[(r + 1) % m]
        dp = (p[axis] - value) if keep_ge else (value - p[axis])
        dq = (q[axis] - value) if keep_ge else (value - q[axis])
        if dp >= 0.0:
            out.append(p)
        if (dp >= 0.0) != (dq >= 0.0):
            t = dp / (dp - dq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def _shoelace(poly):
    s = 0.0
    for r in range(len(poly)):
        x0, y0 = poly[r]
        x1, y1 = poly[(r + 1) % len(poly)]
        s += x0 * y1 - x1 * y0
    return 0.5 * s


def _cell_areas_by_fan(P, n, h):
    """|cell ∩ P| for every cell: signed fan triangles from the vertex mean."""
    nx, ny = n
    A = np.zeros((ny, nx))
    o = tuple(P.mean(axis=0))
    for e in range(len(P)):
        a, b = tuple(P[e]), tuple(P[(e + 1) % len(P)])
        tri = [o, a, b]
        sign = 1.0 if _shoelace(tri) > 0 else -1.0
        xs = [o[0], a[0], b[0]]
        ys = [o[1], a[1], b[1]]
        for i in range(int(math.floor(min(xs) / h)), int(math.floor(max(xs) / h)) + 1):
            for j in range(int(math.floor(min(ys) / h)), int(math.floor(max(ys) / h)) + 1):
                # in coordinates local to the cell's corner (the shoelace terms
                # are then of the cell's size, not of the box's)
                x0, y0 = i * h, j * h
                poly = [(p[0] - x0, p[1] - y0) for p in tri]
                for axis, val, ge in ((0, 0.0, True), (0, h, False), (1, 0.0, True), (1, h, False)):
                    poly = _clip2(poly, axis, val, ge)
                    if len(poly) < 3:
                        break
                if len(poly) >= 3:
                    A[j, i] += sign * abs(_shoelace(poly))
    return A


def _h2d_by_fan(X, n, h):
    H = np.zeros((n[1], n[0]))
    for c, dH in zip(BOUNDS, JUMPS):
        H += dH * _cell_areas_by_fan(_mitred_offset(X, c * h), n, h) / (h * h)
    return H


@pytest.mark.parametrize("case", ["circle", "mode2"])
def test_h2d_per_cell_against_fan_clipper(case):
    n, h = (40, 40), 1.0 / 40
    if case == "circle":
        X = W.circle_markers(72, 0.27, centre=(0.503, 0.497))
    else:
        X = W.mode_shape(96, 0.26, 0.2)
    for c in BOUNDS:
        # the two constructions round differently; the solve for nearly parallel
        # neighbouring edges amplifies it by about 1 / sin(turning angle)
        assert np.max(np.abs(_mitred_offset(X, c * h) - heaviside.offset_polygon_2d(X, c * h))) <= 1e-14
    Ho = heaviside.heaviside_2d(X, n, h)
    Hf = _h2d_by_fan(X, n, h)
    band = (Hf > 1e-9) & (Hf < 1 - 1e-9)
    assert band.sum() > 100
    assert np.max(np.abs(Ho - Hf)) <= 1e-14


def test_h2d_per_cell_single_square_edge_cases():
    """A square of side 0.45 rotated by 31 degrees (its four corners as the
    markers): long sides of both slope signs cross many cells partially, and
    the mitred corners of the offsets stay sharp; against the fan clipper."""
    h = 1.0 / 24
    th = math.radians(31.0)
    X = np.array([[0.5 + 0.225 * (math.cos(th) * sx - math.sin(th) * sy),
                   0.5 + 0.225 * (math.sin(th) * sx + math.cos(th) * sy)]
                  for (sx, sy) in ((-1, -1), (1, -1), (1, 1), (-1, 1))])
    Ho = heaviside.heaviside_2d(X, (24, 24), h)
    Hf = _h2d_by_fan(X, (24, 24), h)
    assert np.max(np.abs(Ho - Hf)) <= 1e-14


# ----------------------------------------------------------------------------
# 3D (plain tuples: many small clips)
def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _normals(V, T):
    """Angle-weighted unit vertex normals toward the inside (triangles are
    outward counter-clockwise): the face normal weighted by the corner angle,
    negated."""
    acc = [[0.0, 0.0, 0.0] for _ in range(len(V))]
    P = [tuple(map(float, v)) for v in V]
    for t in T:
        ia, ib, ic = (int(x) for x in t)
        fn = _cross(_sub(P[ib], P[ia]), _sub(P[ic], P[ia]))
        fl = math.sqrt(_dot(fn, fn))
        for (i0, i1, i2) in ((ia, ib, ic), (ib, ic, ia), (ic, ia, ib)):
            u, v = _sub(P[i1], P[i0]), _sub(P[i2], P[i0])
            ang = math.acos(_dot(u, v) / math.sqrt(_dot(u, u) * _dot(v, v)))
            for d in range(3):
                acc[i0][d] -= ang * fn[d] / fl
    out = np.array(acc)
    return out / np.linalg.norm(out, axis=1, keepdims=True)


def _clip_polyhedron(faces, axis, value, keep_ge):
    """A convex polyhedron (faces: outward vertex loops) cut by the half-space
    coordinate[axis] >= value (or <=); the cap face on the plane closes it."""
    new, cut = [], []
    for f in faces:
        out = []
        m = len(f)
        for r in range(m):
            p, q = f[r], f[(r + 1) % m]
            dp = (p[axis] - value) if keep_ge else (value - p[axis])
            dq = (q[axis] - value) if keep_ge else (value - q[axis])
            if dp >= 0.0:
                out.append(p)
                if dp == 0.0:
                    cut.append(p)
            if (dp > 0.0 and dq < 0.0) or (dp < 0.0 and dq > 0.0):
                t = dp / (dp - dq)
                x = (p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]), p[2] + t * (q[2] - p[2]))
                out.append(x)
                cut.append(x)
        if len(out) >= 3:
            new.append(out)
    if len(cut) >= 3:
        u, v = (axis + 1) % 3, (axis + 2) % 3
        cu = sum(p[u] for p in cut) / len(cut)
        cv = sum(p[v] for p in cut) / len(cut)
        cap = sorted(cut, key=lambda p: math.atan2(p[v] - cv, p[u] - cu))
        # counter-clockwise about +e_axis; the outward normal of the cap is
        # -e_axis when the kept side is >=
        if keep_ge:
            cap = cap[::-1]
        new.append(cap)
    return new


def _volume(faces, o):
    """Divergence theorem about the point o: (1/6) sum over fan triangles of
    (a - o) . ((b - o) x (c - o))."""
    s = 0.0
    for f in faces:
        a = _sub(f[0], o)
        for r in range(1, len(f) - 1):
            s += _dot(a, _cross(_sub(f[r], o), _sub(f[r + 1], o)))
    return s / 6.0


def _span(faces, axis, h):
    vals = [p[axis] for f in faces for p in f]
    return range(int(math.floor(min(vals) / h)), int(math.floor(max(vals) / h)) + 1)


def _cell_volumes_by_fan(P, T, n, h):
    nx, ny, nz = n
    out = np.zeros((nz, ny, nx))
    Pt = [tuple(map(float, v)) for v in P]
    o = tuple(map(float, P.mean(axis=0)))
    for t in T:
        a, b, c = Pt[t[0]], Pt[t[1]], Pt[t[2]]
        sign = 1.0 if _dot(_sub(a, o), _cross(_sub(b, o), _sub(c, o))) > 0 else -1.0
        # outward faces of the tetrahedron o, a, b, c
        if sign > 0:
            tet = [[a, b, c], [o, b, a], [o, c, b], [o, a, c]]
        else:
            tet = [[a, c, b], [o, a, b], [o, b, c], [o, c, a]]
        # slabs in x, then columns in y, then cells in z
        for i in _span(tet, 0, h):
            fx = _clip_polyhedron(_clip_polyhedron(tet, 0, i * h, True), 0, (i + 1) * h, False)
            if len(fx) < 4:
                continue
            for j in _span(fx, 1, h):
                fy = _clip_polyhedron(_clip_polyhedron(fx, 1, j * h, True), 1, (j + 1) * h, False)
                if len(fy) < 4:
                    continue
                for k in _span(fy, 2, h):
                    fz = _clip_polyhedron(_clip_polyhedron(fy, 2, k * h, True), 2, (k + 1) * h, False)
                    if len(fz) >= 4:
                        out[k, j, i] += sign * abs(_volume(fz, (i * h, j * h, k * h)))
    return out


def test_fan_clipper_on_a_cube_by_hand():
    """The 3D clipper alone: the unit cube [0.1, 0.7]^3 fanned from its centre
    on an h = 0.25 grid; each cell's overlap is the product of its three
    interval overlaps."""
    lo, hi, h = 0.1, 0.7, 0.25
    c = [(x, y, z) for z in (lo, hi) for y in (lo, hi) for x in (lo, hi)]
    V = np.array(c)
    # 12 outward counter-clockwise triangles
    T = np.array([[0, 2, 3], [0, 3, 1], [4, 5, 7], [4, 7, 6], [0, 1, 5], [0, 5, 4],
                  [2, 6, 7], [2, 7, 3], [0, 4, 6], [0, 6, 2], [1, 3, 7], [1, 7, 5]])
    vol = _cell_volumes_by_fan(V, T, (4, 4, 4), h)

    def ov(i):
        return max(0.0, min(hi, (i + 1) * h) - max(lo, i * h))

    ref = np.array([[[ov(i) * ov(j) * ov(k) for i in range(4)] for j in range(4)] for k in range(4)])
    assert np.max(np.abs(vol - ref)) <= 1e-16
    assert abs(heaviside.mesh_volume(V, T) - 0.6 ** 3) <= 1e-15


@pytest.mark.slow
def test_h3d_per_cell_against_fan_clipper():
    n, h = (16, 16, 16), 1.0 / 16
    V, T = W.sphere_mesh(2, 0.31, centre=(0.507, 0.493, 0.501), seed=11)
    nrm = _normals(V, T)
    assert np.max(np.abs(nrm - heaviside.vertex_normals(V, T))) <= 1e-14
    Ho = heaviside.heaviside_3d(V, T, n, h, nrm=nrm)
    Hf = np.zeros_like(Ho)
    for c, dH in zip(BOUNDS, JUMPS):
        Hf += dH * _cell_volumes_by_fan(V + c * h * nrm, T, n, h) / h ** 3
    band = (Hf > 1e-9) & (Hf < 1 - 1e-9)
    assert band.sum() > 300
    assert np.max(np.abs(Ho - Hf)) <= 1e-14
