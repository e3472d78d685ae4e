"""Gravity, the non-inertial frame and the mass correction of the free-fall
runs (oracle; test infrastructure only).

Section 2.1 (non-inertial frame, eqs non-inertial, fictitious, fic_1, fic_2;
conservation of mass) and Section 5.3 (free-fall drop).

Readings (the paper is silent or its printed forms are ambiguous):
  * the box is periodic along the vertical axis, where a uniform rho g cannot
    be balanced by a periodic pressure; the weight enters as the force density
    (rho - rho_mean) g with rho_mean the volume mean of the density (no net
    force on the box: the drop falls through the fluid, which rises);
  * the frame acceleration of eq fictitious acts as a restoring control on the
    drop's centre of mass COM (c1 = c2 = 0.1 as printed):
        a = -c1 (COM_n - COM_0) / dt - c2 (COM_n - COM_{n-1}) / dt,
    added per unit mass (force density rho a) along the vertical axis; the
    printed signs mix a restoring and an amplifying term, and only this
    combination keeps the drop in place;
  * mass correction: every `every` steps the enclosed area (2D) or volume of
    revolution (axisymmetric) is compared with the initial one; when the
    relative difference exceeds 1e-6 all markers move by one distance delta
    along their unit normals toward the drop, delta found by bisection until
    the relative difference is below 1e-12.
"""
import numpy as np


def polygon_area_centroid(X):
    """Signed area and centroid (x, y) of the closed polygon X (counter-clockwise)."""
    x, y = X[:, 0], X[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = 0.5 * np.sum(cr)
    cx = np.sum((x + xn) * cr) / (6 * A)
    cy = np.sum((y + yn) * cr) / (6 * A)
    return A, cx, cy


def revolution_volume_centroid(X, axis_x):
    """Volume of revolution about x = axis_x of the region that the closed
    mirrored meridian curve X encloses on the side x >= axis_x, and the axial
    (y) coordinate of its centroid. Green's theorem on the right half:
    V = pi * sum over segments of int r^2 dz, V z_c = pi * sum int z r^2 dz,
    exact for straight segments (segments with an end left of the axis skip)."""
    r = X[:, 0] - axis_x
    z = X[:, 1]
    rn, zn = np.roll(r, -1), np.roll(z, -1)
    keep = (r >= -1e-12) & (rn >= -1e-12)
    A, B = np.maximum(r, 0.0), np.maximum(rn, 0.0) - np.maximum(r, 0.0)
    C, D = z, zn - z
    i_r2 = D * (A * A + A * B + B * B / 3.0)
    i_zr2 = D * (C * (A * A + A * B + B * B / 3.0) + D * (A * A / 2.0 + 2.0 * A * B / 3.0 + B * B / 4.0))
    V = np.pi * np.sum(np.where(keep, i_r2, 0.0))
    zc = np.pi * np.sum(np.where(keep, i_zr2, 0.0)) / V
    return V, zc


def mesh_volume_centroid(V, T):
    """Volume enclosed by the closed triangulated surface (V, T outward counter-
    clockwise) and the y coordinate of its centroid (the vertical axis of the 3D
    runs): the divergence theorem over the tetrahedra (origin, a, b, c), each of
    volume a . (b x c) / 6 and centroid (a + b + c) / 4."""
    V = np.asarray(V, dtype=np.float64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    vt = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    vol = float(np.sum(vt))
    cy = float(np.sum(vt * (a[:, 1] + b[:, 1] + c[:, 1]) / 4.0)) / vol
    return vol, cy


def measure(X, axis_x=None, T=None):
    """(enclosed area, volume of revolution or mesh volume; vertical centroid)."""
    if T is not None:
        return mesh_volume_centroid(X, T)
    if axis_x is None:
        A, _, cy = polygon_area_centroid(X)
        return A, cy
    return revolution_volume_centroid(X, axis_x)


def mass_correct(X, nrm, target, axis_x=None, h=1.0, trigger=1e-6, tol=1e-12, T=None):
    """Move the markers (mesh vertices when T is given) along their normals
    (toward the drop for delta > 0) so that the enclosed area / volume returns
    to target; unchanged when the relative difference is at most `trigger`."""
    v0, _ = measure(X, axis_x, T)
    if abs(v0 - target) <= trigger * abs(target):
        return X, 0.0
    lo, hi = -h, h          # volume decreases with delta
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        v, _ = measure(X + mid * nrm, axis_x, T)
        if abs(v - target) <= tol * abs(target):
            break
        if v > target:
            lo = mid
        else:
            hi = mid
    return X + mid * nrm, mid


def frame_acceleration(com0, com_prev, com_n, dt, c1=0.1, c2=0.1):
    """Restoring frame acceleration along the vertical axis (reading above)."""
    return -c1 * (com_n - com0) / dt - c2 * (com_n - com_prev) / dt


def body_force(rho_face, rho_mean, g, a):
    """Force density on the vertical faces: (rho - rho_mean) g + rho a."""
    return (rho_face - rho_mean) * g + rho_face * a
