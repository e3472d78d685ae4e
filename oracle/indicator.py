"""Indicator function of the conventional scheme (oracle; test infrastructure
only -- the product path never imports this package).

Section 2.2, eqs indicator and ind_psn: the properties follow an indicator I,
psi = psi_1 + (psi_2 - psi_1) I, that solves
    div grad I = div delta_vec,
delta_vec the discrete delta vector of eq delta_vec: the unit normals (toward
the drop) times the arc elements, spread to the faces by the discrete delta
function (the conventional spreading). Section 3.1 discusses the same Poisson
problem (eq poisson_delta): the split delta vector is not curl-free, so its
solution is not a perfect Heaviside function and converges at first order.

Readings (the paper is silent): the periodic solution is fixed up to a
constant; the constant makes the integral of I equal to the area the markers
enclose (the integral a Heaviside function has), I = P + A / |Omega| with P
the zero-mean solution. The discrete operators are those of the projection
(faces on the low side of each cell, the 5-point Laplacian); the solve is the
exact periodic one (discrete Fourier diagonalisation).
"""
import numpy as np

from . import heaviside, poisson, transfer


def delta_vector(X, ds, nrm, n, h):
    """Face components of sum_k n_k ds_k delta_h(x - X_k) (eq delta_vec with the
    unit normal as the force, eq delta for the spreading)."""
    return transfer.spread_delta(np.asarray(nrm) * np.asarray(ds)[:, None], X, n, h)


def indicator_from_faces(F, area, h):
    """I of eq ind_psn for a given face vector field F and enclosed area."""
    b = poisson.divergence(F, h)
    P = poisson.fft_solve(b - b.mean(), 1.0, h)
    P = P - P.mean()
    return P + area / (P.size * h ** P.ndim)


def indicator(X, ds, nrm, n, h):
    """I of the conventional scheme for the closed curve X (counter-clockwise)."""
    F = delta_vector(X, ds, nrm, n, h)
    return indicator_from_faces(F, heaviside.shoelace(np.asarray(X)), h)
