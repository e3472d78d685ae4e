"""Velocity interpolation and conventional force spreading (oracle).

Grid convention (Section 2.1, staggered MAC grid): cell (i, j[, k]) has centre
((i+1/2)h, (j+1/2)h[, (k+1/2)h]); the velocity component along axis d lives on
the face at the low side of the cell along d, e.g. u[k, j, i] at
(i h, (j+1/2)h, (k+1/2)h). Arrays have shape (nz, ny, nx) in 3D and (ny, nx)
in 2D (x fastest). The box is periodic; kernel offsets use the minimum image.

eq jump_condu: U(X_s) = sum over faces of u(x_f) delta_h(x_f - X_s) h^dim.
eq delta_vec / eq delta: F(x_f) = sum over markers of F_s delta_h(x_f - X_s),
with F_s the force carried by marker s (force per unit length/area times its
arc length/area, times its unit normal).
"""
import itertools

import numpy as np

from .kernel import phi


def _axis(dim: int, e: int) -> int:
    """Array axis of spatial direction e (x fastest = last axis)."""
    return dim - 1 - e


def _taps(X, h, d, e):
    """4 face indices and kernel weights along direction e for component d."""
    off = 0.0 if e == d else 0.5
    s = X[:, e] / h - off
    base = np.floor(s).astype(np.int64) - 1
    idx = base[:, None] + np.arange(4)[None, :]
    w = phi(idx + off - X[:, e:e + 1] / h)
    return idx, w


def interp(u, X, h):
    """U (N x dim): kernel-weighted sum over the 4^dim faces around each marker."""
    X = np.asarray(X, dtype=np.float64)
    N, dim = X.shape
    shape = u[0].shape
    n = shape[::-1]
    U = np.zeros((N, dim))
    for d in range(dim):
        taps = [_taps(X, h, d, e) for e in range(dim)]
        for combo in itertools.product(range(4), repeat=dim):
            w = np.ones(N)
            index = [None] * dim
            for e in range(dim):
                idx, we = taps[e]
                w = w * we[:, combo[e]]
                index[_axis(dim, e)] = np.mod(idx[:, combo[e]], n[e])
            U[:, d] += w * u[d][tuple(index)]
    return U


def interp_bruteforce(u, X, h):
    """Same sum over every face of the grid (minimum-image offsets); tiny grids."""
    X = np.asarray(X, dtype=np.float64)
    N, dim = X.shape
    shape = u[0].shape
    n = shape[::-1]
    L = [n[e] * h for e in range(dim)]
    U = np.zeros((N, dim))
    for d in range(dim):
        for s in range(N):
            acc = 0.0
            for index in np.ndindex(*shape):
                w = 1.0
                for e in range(dim):
                    ie = index[_axis(dim, e)]
                    xf = (ie + (0.0 if e == d else 0.5)) * h
                    dx = xf - X[s, e]
                    dx -= L[e] * np.round(dx / L[e])
                    w *= phi(dx / h)
                    if w == 0.0:
                        break
                acc += w * u[d][index]
            U[s, d] = acc
    return U


def marker_normals_2d(X):
    """Unit normal toward the interior of a counter-clockwise closed polyline:
    the left perpendicular of the central chord X_{k+1} - X_{k-1}."""
    t = np.roll(X, -1, axis=0) - np.roll(X, 1, axis=0)
    nrm = np.stack([-t[:, 1], t[:, 0]], axis=1)
    return nrm / np.linalg.norm(nrm, axis=1, keepdims=True)


def marker_forces(fs, ds, nrm):
    """F_s = (sigma kappa)_s * ds_s * n_s."""
    return (np.asarray(fs) * np.asarray(ds))[:, None] * np.asarray(nrm)


def spread_delta(Fs, X, n, h):
    """Conventional spreading: each face receives sum_s F_s,d delta_h(x_f - X_s)."""
    X = np.asarray(X, dtype=np.float64)
    N, dim = X.shape
    shape = tuple(reversed(n[:dim]))
    F = [np.zeros(shape) for _ in range(dim)]
    inv = 1.0 / h ** dim
    for d in range(dim):
        taps = [_taps(X, h, d, e) for e in range(dim)]
        for combo in itertools.product(range(4), repeat=dim):
            w = np.ones(N)
            index = [None] * dim
            for e in range(dim):
                idx, we = taps[e]
                w = w * we[:, combo[e]]
                index[_axis(dim, e)] = np.mod(idx[:, combo[e]], n[e])
            np.add.at(F[d], tuple(index), w * Fs[:, d] * inv)
    return F
