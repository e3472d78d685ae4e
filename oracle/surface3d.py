"""Curvature force on a closed triangulated surface (oracle; builder's 3D
extension: the paper reconstructs only curves and leaves closed surfaces in
3D to future work, Sections 4 and 6).

Markers are the mesh vertices. The surface-tension force on vertex v is
minus sigma times the gradient of the total area with respect to X_v, written
with the cotangent formula of the discrete Laplace-Beltrami operator:
  F_v = (sigma / 2) sum_{w ~ v} (cot a_vw + cot b_vw) (X_w - X_v),
where a_vw, b_vw are the angles opposite the edge vw. With the vertex area
A_v = (1/3) sum of adjacent triangle areas and the unit inward
angle-weighted normal n_v:
  fs_v = (F_v . n_v) / A_v  (sigma times the sum of principal curvatures),
  ds_v = A_v.
"""
import numpy as np

from .heaviside import vertex_normals


def cotangent_forces(V, T, sigma):
    V = np.asarray(V, dtype=np.float64)
    F = np.zeros_like(V)
    for t in T:
        for r in range(3):
            o = t[r]                       # vertex opposite edge (p, q)
            p, q = t[(r + 1) % 3], t[(r + 2) % 3]
            e1 = V[p] - V[o]
            e2 = V[q] - V[o]
            cot = float(e1 @ e2) / np.linalg.norm(np.cross(e1, e2))
            F[p] += 0.5 * sigma * cot * (V[q] - V[p])
            F[q] += 0.5 * sigma * cot * (V[p] - V[q])
    return F


def vertex_areas(V, T):
    V = np.asarray(V, dtype=np.float64)
    A = np.zeros(len(V))
    for t in T:
        a = 0.5 * np.linalg.norm(np.cross(V[t[1]] - V[t[0]], V[t[2]] - V[t[0]]))
        for r in range(3):
            A[t[r]] += a / 3.0
    return A


def surface_geometry(V, T, sigma):
    """(fs, ds, nrm) per vertex."""
    F = cotangent_forces(V, T, sigma)
    A = vertex_areas(V, T)
    nrm = vertex_normals(V, T)
    fs = np.einsum("ij,ij->i", F, nrm) / A
    return fs, A, nrm, F


# ----------------------------------------------------------------------------
# Local least-squares reconstruction of a moving surface (the 3D counterpart
# of the least-squares B-spline of Section 4, which the paper leaves to future
# work for surfaces).
#
# Per vertex v: a frame (t1, t2, n) with n the inward angle-weighted normal,
# t1 the unit projection on the tangent plane of the coordinate axis least
# aligned with n, t2 = n x t1; the points of the vertex's two-ring (v itself
# included) in local coordinates scaled by L, their mean distance from v; the
# least-squares quadric z = g + d x + e y + a x^2 + b x y + c y^2. Then
#   X'_v  = X_v + g L n                        (the vertex on the fitted surface),
#   n'_v  = (n - d t1 - e t2) / sqrt(1 + d^2 + e^2),
#   kappa = [(1 + e^2) 2a - 2 d e b + (1 + d^2) 2c] / (L (1 + d^2 + e^2)^(3/2))
# (the sum of the principal curvatures of the graph at the vertex, positive
# for a convex drop), fs = sigma kappa, ds = the vertex area (a third of the
# adjacent triangles' areas) of the moved mesh.
# ----------------------------------------------------------------------------
def two_rings(nv, T):
    nb = [set() for _ in range(nv)]
    for t in T:
        for r in range(3):
            nb[t[r]].update((t[(r + 1) % 3], t[(r + 2) % 3]))
    rings = []
    for v in range(nv):
        ring = set(nb[v])
        for w in nb[v]:
            ring |= nb[w]
        ring.add(v)
        rings.append(sorted(ring))
    return rings


def local_frame(n):
    axis = int(np.argmin(np.abs(n)))
    e = np.zeros(3)
    e[axis] = 1.0
    t1 = e - (e @ n) * n
    t1 = t1 / np.linalg.norm(t1)
    return t1, np.cross(n, t1)


def lsq_reconstruct(V, T, sigma):
    """(V', fs, ds, nrm) of the local least-squares quadric reconstruction."""
    V = np.asarray(V, dtype=np.float64)
    nrm0 = vertex_normals(V, T)
    rings = two_rings(len(V), T)
    Vn = V.copy()
    fs = np.zeros(len(V))
    nrm = np.zeros_like(V)
    for v, ring in enumerate(rings):
        n = nrm0[v]
        t1, t2 = local_frame(n)
        P = V[ring] - V[v]
        L = np.mean(np.linalg.norm(P, axis=1)) * len(ring) / (len(ring) - 1)
        x, y, z = P @ t1 / L, P @ t2 / L, P @ n / L
        A = np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], axis=1)
        g, d, e, a, b, c = np.linalg.lstsq(A, z, rcond=None)[0]
        Vn[v] = V[v] + g * L * n
        w = 1.0 + d * d + e * e
        nrm[v] = (n - d * t1 - e * t2) / np.sqrt(w)
        fs[v] = sigma * ((1 + e * e) * 2 * a - 2 * d * e * b + (1 + d * d) * 2 * c) / (L * w ** 1.5)
    return Vn, fs, vertex_areas(Vn, T), nrm
