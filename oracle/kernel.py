"""Cosine kernel of the discrete delta function and its integral (oracle).

Section 2.2, eqs delta and cherby: delta_h(x - X) = prod_d phi(dx_d / h) / h^dim
with phi(q) = (1 + cos(pi q / 2)) / 4 for |q| < 2 and 0 otherwise (q in grid
units; eq cherby carries 1/(4 ds) and eq delta divides by the cell size, so the
consistent reading takes ds = 1 grid unit inside eq delta).

Section 3.2, eq new_hea: the discrete Heaviside profile is the integral of the
same kernel along the interface normal, H(q) = 1/2 + q/4 + sin(pi q/2)/(2 pi)
for q in [-2, 2] (the printed closed form is garbled; this is the integral of
eq cherby, which reproduces the printed region values 0.5 and 0.909).
eq new_hea2: the region values are H at q = -2, -1, 0, 1, 2, i.e.
0, 0.0908, 0.5, 0.9092, 1 (the printed 0.409 for region II is the increment
H(0) - H(-1); by the symmetry H(-q) = 1 - H(q) the value is 0.0908).
"""
import math

import numpy as np


def phi(q):
    q = np.asarray(q, dtype=np.float64)
    return np.where(np.abs(q) < 2.0, 0.25 * (1.0 + np.cos(0.5 * np.pi * q)), 0.0)


def phi_scalar(q: float) -> float:
    if abs(q) < 2.0:
        return 0.25 * (1.0 + math.cos(0.5 * math.pi * q))
    return 0.0


def heaviside_profile(q):
    """Integral of phi from -2 to q: 0 below the support, 1 (its total mass) above."""
    q = np.asarray(q, dtype=np.float64)
    inner = 0.5 + 0.25 * q + np.sin(0.5 * np.pi * q) / (2.0 * np.pi)
    return np.where(q <= -2.0, 0.0, np.where(q >= 2.0, 1.0, inner))


# Region boundaries of the per-segment polygons, in grid units, positive toward
# the drop: each region collects the points whose normal distance rounds to its
# sample point q in {-2, -1, 0, 1, 2}.
OFFSETS = (-1.5, -0.5, 0.5, 1.5)


def region_values():
    return [float(heaviside_profile(q)) for q in (-2.0, -1.0, 0.0, 1.0, 2.0)]


def region_jumps():
    """Increments Delta H_m between consecutive regions (sum = 1)."""
    v = region_values()
    return [v[m + 1] - v[m] for m in range(4)]
