"""Diagnostics of the projection step (oracle), Section 5.

eq sd_pres_diff: Delta P = mean(p inside) - mean(p outside), interface cells
excluded (inside = H >= 1 - 1e-12, outside = H <= 1e-12).
eq tke: TKE = sum (u^2 + v^2 [+ w^2]) dV, exactly as printed (no 1/2, no rho);
the staggered components are summed face by face.
Force ratio (caption of the large-deformation figure): |sum_grid F dV| over
sum_s |F_s|.
Discrete curl in index form (Section 3.2, the identity after eq delta_hea_xy):
for the (a, b) plane, (F_b[c] - F_b[c - e_a]) - (F_a[c] - F_a[c - e_b]).
"""
import numpy as np


def pressure_jump(p, H):
    inside = H >= 1.0 - 1e-12
    outside = H <= 1e-12
    return float(p[inside].mean() - p[outside].mean())


def tke(u, h):
    dim = len(u)
    return float(sum(np.sum(c * c) for c in u) * h ** dim)


def force_ratio(F, Fs, h):
    dim = len(F)
    tot = np.array([np.sum(F[d]) for d in range(dim)]) * h ** dim
    return float(np.linalg.norm(tot) / np.sum(np.linalg.norm(Fs, axis=1)))


def grid_force_sum(F, h):
    dim = len(F)
    return np.array([np.sum(F[d]) for d in range(dim)]) * h ** dim


def curl_max(F):
    """Maximum |index-form curl| over all nodes (2D) / edges (3D)."""
    dim = len(F)
    m = 0.0
    planes = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (2, 0)]
    for (a, b) in planes:
        axa, axb = dim - 1 - a, dim - 1 - b
        c = (F[b] - np.roll(F[b], 1, axis=axa)) - (F[a] - np.roll(F[a], 1, axis=axb))
        m = max(m, float(np.max(np.abs(c))))
    return m
