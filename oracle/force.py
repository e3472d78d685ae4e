"""Face surface tension and the irrotational delta vector (oracle).

eq delta_hea_xy (Section 3.2): on the face between cells c - e_d and c,
F_d = f_face * (H_c - H_{c-e_d}) / h. The difference of the cell-centred
Heaviside is the discrete gradient, so for a constant f the field is curl-free
in index form. (The paper writes the difference without 1/h; the 1/h makes F
a force density, which does not change its curl.)

The paper defers the face value f to a later section that never gives it.
Reading used here: f_face is sigma*kappa at the foot of the perpendicular from
the face centre to the nearest interface segment (2D) or triangle (3D), with
sigma*kappa interpolated linearly (2D) or barycentrically (3D) from the end
markers / vertices; exact distance ties go to the lower element index.
f is only evaluated on faces where the Heaviside difference is nonzero.
In exact arithmetic H is exactly 0 or 1 away from the interface; the overlap
sums leave rounding noise of order 1e-16 there, so a face counts as an
interface face when |H_c - H_{c-e_d}| > DH_EPS = 1e-13 and carries F = 0
otherwise (well above the noise, and a legitimate difference that small
would change F by less than 1e-13 of its scale).
"""
import numpy as np

DH_EPS = 1e-13


def _face_centres(dim, d, idx, h):
    """Coordinates (M x dim) of faces of orientation d at array indices idx."""
    pts = np.empty((len(idx[0]), dim))
    for e in range(dim):
        ie = idx[dim - 1 - e]
        pts[:, e] = (ie + (0.0 if e == d else 0.5)) * h
    return pts


def nearest_on_polyline(p, X, fs):
    """sigma*kappa at the foot point on the nearest segment of the closed polyline."""
    A = X
    B = np.roll(X, -1, axis=0)
    AB = B - A
    t = np.einsum("ij,ij->i", p[None, :] - A, AB) / np.einsum("ij,ij->i", AB, AB)
    t = np.clip(t, 0.0, 1.0)
    Q = A + t[:, None] * AB
    d2 = np.sum((Q - p[None, :]) ** 2, axis=1)
    k = int(np.argmin(d2))  # first occurrence = lowest index on ties
    return (1.0 - t[k]) * fs[k] + t[k] * fs[(k + 1) % len(X)]


def _closest_on_segment(p, a, b):
    ab = b - a
    t = np.einsum("ij,ij->i", p - a, ab) / np.einsum("ij,ij->i", ab, ab)
    t = np.clip(t, 0.0, 1.0)
    return a + t[:, None] * ab, t


def nearest_on_mesh(p, V, T, fs):
    """sigma*kappa at the closest point of the nearest triangle (barycentric)."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    M = len(T)
    P = np.broadcast_to(p, (M, 3))
    # candidate 1: projection onto the plane when it falls inside the triangle
    n = np.cross(b - a, c - a)
    nn = np.einsum("ij,ij->i", n, n)
    w = P - a
    # barycentric coordinates of the projection
    l1 = np.einsum("ij,ij->i", np.cross(w, c - a), n) / nn   # weight of b
    l2 = np.einsum("ij,ij->i", np.cross(b - a, w), n) / nn   # weight of c
    l0 = 1.0 - l1 - l2
    inside = (l0 >= 0) & (l1 >= 0) & (l2 >= 0)
    proj = a + l1[:, None] * (b - a) + l2[:, None] * (c - a)
    best_d2 = np.where(inside, np.sum((proj - P) ** 2, axis=1), np.inf)
    bary = np.stack([l0, l1, l2], axis=1)
    # candidates 2-4: the three edges
    for (u, v, iu, iv) in ((a, b, 0, 1), (b, c, 1, 2), (c, a, 2, 0)):
        q, t = _closest_on_segment(P, u, v)
        d2 = np.sum((q - P) ** 2, axis=1)
        better = d2 < best_d2
        best_d2 = np.where(better, d2, best_d2)
        nb = np.zeros((M, 3))
        nb[np.arange(M), iu] = 1.0 - t
        nb[np.arange(M), iv] = t
        bary = np.where(better[:, None], nb, bary)
    k = int(np.argmin(best_d2))
    return float(bary[k] @ fs[T[k]])


def irrotational_force(H, X, fs, h, tris=None):
    """Face force F_d = f_face (H_c - H_{c-e_d}) / h for every orientation d."""
    dim = H.ndim
    F = []
    for d in range(dim):
        ax = dim - 1 - d
        dH = H - np.roll(H, 1, axis=ax)
        Fd = np.zeros_like(H)
        idx = np.nonzero(np.abs(dH) > DH_EPS)
        pts = _face_centres(dim, d, idx, h)
        for m in range(len(pts)):
            if dim == 2:
                f = nearest_on_polyline(pts[m], X, fs)
            else:
                f = nearest_on_mesh(pts[m], X, tris, fs)
            Fd[tuple(ix[m] for ix in idx)] = f * dH[tuple(ix[m] for ix in idx)] / h
        F.append(Fd)
    return F


def face_force_at(H_lo, H_hi, pt, X, fs, h, tris=None):
    """F at one face from the two adjacent cell values (for sampled checks)."""
    dH = H_hi - H_lo
    if abs(dH) <= DH_EPS:
        return 0.0
    f = nearest_on_polyline(pt, X, fs) if tris is None else nearest_on_mesh(pt, X, tris, fs)
    return f * dH / h
