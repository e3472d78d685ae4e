"""Discrete Heaviside from the interface polygons (oracle), Section 3.2.

Construction (eqs new_hea, new_hea2; captions of the polygon figures): around
the interface, the plane is split into five regions by the distance r to the
interface (positive toward the drop) with boundaries r = -1.5h, -0.5h, 0.5h,
1.5h; each region carries H at its sample point q = -2..2. Equivalently
H^(x) = sum_m dH_m 1[x in P_m], where P_m is the interface offset inward by
c_m in {-1.5h, -0.5h, 0.5h, 1.5h} and dH_m are the increments between region
values. The cell value sums the overlap areas times the region value (caption
of the three-polygon figure), H_c = sum_m dH_m |cell ∩ P_m| / h^dim.

2D offsets are mitred (each offset edge lies at exactly c from its segment);
3D offsets move each vertex by c along its unit angle-weighted normal.

Overlaps are computed column by column. For a closed, outward-oriented
boundary, the measure of (P ∩ column ∩ {coordinate > c}) equals
W(c) = sum over boundary pieces of (signed projected size) * integral of
max(height - c, 0); the cell measure is W(bottom) - W(top).
"""
import math

import numpy as np

from .kernel import OFFSETS, region_jumps


# ----------------------------------------------------------------------------
# 2D
# ----------------------------------------------------------------------------
def offset_polygon_2d(X, c):
    """Mitred offset of a closed counter-clockwise polyline, c > 0 inward."""
    X = np.asarray(X, dtype=np.float64)
    N = len(X)
    out = np.empty_like(X)
    for k in range(N):
        a = X[k] - X[k - 1]
        b = X[(k + 1) % N] - X[k]
        na = np.array([-a[1], a[0]]) / math.hypot(a[0], a[1])
        nb = np.array([-b[1], b[0]]) / math.hypot(b[0], b[1])
        m = (na + nb) / (1.0 + na @ nb)
        out[k] = X[k] + c * m
    return out


def _g_segment(xa, ya, xb, yb, c):
    """-(integral over x from xa to xb of max(y(x) - c, 0)) for a straight piece."""
    c = np.asarray(c, dtype=np.float64)
    dx = xb - xa
    g = np.zeros_like(c)
    both = (ya >= c) & (yb >= c)
    g = np.where(both, -dx * (0.5 * (ya + yb) - c), g)
    if ya != yb:
        t1 = (ya - c) / (ya - yb)
        m1 = (ya >= c) & (yb < c)
        g = np.where(m1, -(t1 * dx) * (0.5 * (ya - c)), g)
        t2 = (yb - c) / (yb - ya)
        m2 = (yb >= c) & (ya < c)
        g = np.where(m2, -(t2 * dx) * (0.5 * (yb - c)), g)
    return g


def polygon_cell_areas(P, n, h):
    """|cell ∩ P| for every cell of an (ny, nx) grid; P closed counter-clockwise."""
    nx, ny = n[0], n[1]
    A = np.zeros((ny, nx))
    yb = np.arange(ny) * h
    N = len(P)
    for e in range(N):
        xa, ya = P[e]
        xb, yb_ = P[(e + 1) % N]
        if xa == xb:
            continue
        lo, hi = min(xa, xb), max(xa, xb)
        for i in range(int(math.floor(lo / h)), int(math.floor(hi / h)) + 1):
            x0, x1 = i * h, (i + 1) * h
            t0 = (x0 - xa) / (xb - xa)
            t1 = (x1 - xa) / (xb - xa)
            ta, tb = max(0.0, min(t0, t1)), min(1.0, max(t0, t1))
            if tb <= ta:
                continue
            pxa, pya = xa + ta * (xb - xa), ya + ta * (yb_ - ya)
            pxb, pyb = xa + tb * (xb - xa), ya + tb * (yb_ - ya)
            if pxa == pxb:
                continue
            A[:, i] += _g_segment(pxa, pya, pxb, pyb, yb) - _g_segment(pxa, pya, pxb, pyb, yb + h)
    return A


def heaviside_2d(X, n, h):
    H = np.zeros((n[1], n[0]))
    for c, dH in zip(OFFSETS, region_jumps()):
        P = offset_polygon_2d(X, c * h)
        H += dH * polygon_cell_areas(P, n, h) / (h * h)
    return H


def shoelace(P):
    x, y = P[:, 0], P[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


# ----------------------------------------------------------------------------
# 3D
# ----------------------------------------------------------------------------
def vertex_normals(V, T):
    """Unit angle-weighted vertex normals pointing into the enclosed volume."""
    V = np.asarray(V, dtype=np.float64)
    acc = np.zeros_like(V)
    for t in T:
        for r in range(3):
            a, b, c = V[t[r]], V[t[(r + 1) % 3]], V[t[(r + 2) % 3]]
            e1, e2 = b - a, c - a
            ang = math.atan2(np.linalg.norm(np.cross(e1, e2)), float(e1 @ e2))
            nt = np.cross(V[t[1]] - V[t[0]], V[t[2]] - V[t[0]])
            nt = nt / np.linalg.norm(nt)
            acc[t[r]] += ang * nt
    acc = -acc  # triangles are outward counter-clockwise; inward is the negative
    return acc / np.linalg.norm(acc, axis=1, keepdims=True)


def offset_mesh(V, nrm, c):
    return np.asarray(V) + c * np.asarray(nrm)


def _clip(poly, axis, value, keep_ge):
    """Sutherland-Hodgman clip of a 3D polygon by coordinate[axis] >= / <= value."""
    out = []
    m = len(poly)
    for r in range(m):
        p, q = poly[r], poly[(r + 1) % m]
        sp = p[axis] - value if keep_ge else value - p[axis]
        sq = q[axis] - value if keep_ge else value - q[axis]
        if sp >= 0:
            out.append(p)
        if (sp >= 0) != (sq >= 0):
            t = sp / (sp - sq)
            out.append(p + t * (q - p))
    return out


def _g_poly(poly, c):
    """integral over the xy-projection (signed) of max(z - c, 0)."""
    q = _clip(poly, 2, c, True)
    if len(q) < 3:
        return 0.0
    s = 0.0
    p0 = q[0]
    for r in range(1, len(q) - 1):
        a, b = q[r] - p0, q[r + 1] - p0
        area = 0.5 * (a[0] * b[1] - a[1] * b[0])
        s += area * ((p0[2] + q[r][2] + q[r + 1][2]) / 3.0 - c)
    return s


def _column_piece(tri, i, j, h):
    poly = [tri[0], tri[1], tri[2]]
    poly = _clip(poly, 0, i * h, True)
    if len(poly) < 3:
        return None
    poly = _clip(poly, 0, (i + 1) * h, False)
    if len(poly) < 3:
        return None
    poly = _clip(poly, 1, j * h, True)
    if len(poly) < 3:
        return None
    poly = _clip(poly, 1, (j + 1) * h, False)
    if len(poly) < 3:
        return None
    return poly


def _projected_area(poly):
    s = 0.0
    p0 = poly[0]
    for r in range(1, len(poly) - 1):
        a, b = poly[r] - p0, poly[r + 1] - p0
        s += 0.5 * (a[0] * b[1] - a[1] * b[0])
    return s


def mesh_column_volumes(P, T, n, h, columns=None):
    """Cell volumes |cell ∩ P| for a closed outward mesh; returns a dict
    (i, j) -> array over k when ``columns`` is given, else the full array."""
    nx, ny, nz = n
    P = np.asarray(P, dtype=np.float64)
    tri_pts = P[T]                                  # (M, 3, 3)
    lo = tri_pts.min(axis=1)
    hi = tri_pts.max(axis=1)
    full = columns is None
    if full:
        out = np.zeros((nz, ny, nx))
        cand = range(len(T))
    else:
        out = {c: np.zeros(nz) for c in columns}
    zb = np.arange(nz) * h

    def add_piece(tri, i, j, target):
        piece = _column_piece(tri, i, j, h)
        if piece is None:
            return
        zs = [p[2] for p in piece]
        kmin = int(math.floor(min(zs) / h))
        kmax = int(math.floor(max(zs) / h))
        area = _projected_area(piece)
        # cells entirely below the piece: full height h
        if kmin > 0:
            target[:kmin] += area * h
        for k in range(max(kmin, 0), min(kmax, nz - 1) + 1):
            target[k] += _g_poly(piece, zb[k]) - _g_poly(piece, zb[k] + h)

    if full:
        for t in range(len(T)):
            tri = [tri_pts[t, 0], tri_pts[t, 1], tri_pts[t, 2]]
            for i in range(int(math.floor(lo[t, 0] / h)), int(math.floor(hi[t, 0] / h)) + 1):
                for j in range(int(math.floor(lo[t, 1] / h)), int(math.floor(hi[t, 1] / h)) + 1):
                    add_piece(tri, i, j, out[:, j, i])
    else:
        for (i, j) in columns:
            sel = np.nonzero((lo[:, 0] < (i + 1) * h) & (hi[:, 0] > i * h) &
                             (lo[:, 1] < (j + 1) * h) & (hi[:, 1] > j * h))[0]
            for t in sel:
                tri = [tri_pts[t, 0], tri_pts[t, 1], tri_pts[t, 2]]
                add_piece(tri, i, j, out[(i, j)])
    return out


def heaviside_3d(V, T, n, h, nrm=None, columns=None):
    if nrm is None:
        nrm = vertex_normals(V, T)
    jumps = region_jumps()
    if columns is None:
        H = np.zeros((n[2], n[1], n[0]))
        for c, dH in zip(OFFSETS, jumps):
            H += dH * mesh_column_volumes(offset_mesh(V, nrm, c * h), T, n, h) / h ** 3
        return H
    H = {col: np.zeros(n[2]) for col in columns}
    for c, dH in zip(OFFSETS, jumps):
        vols = mesh_column_volumes(offset_mesh(V, nrm, c * h), T, n, h, columns=columns)
        for col in columns:
            H[col] += dH * vols[col] / h ** 3
    return H


def mesh_volume(P, T):
    """Enclosed volume by the divergence theorem (outward triangles)."""
    P = np.asarray(P)
    a, b, c = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    return float(np.sum(np.einsum("ij,ij->i", a, np.cross(b, c)))) / 6.0
