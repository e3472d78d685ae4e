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
