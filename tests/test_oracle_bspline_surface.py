"""Oracle pins: B-spline relocation (Section 4) and 3D surface curvature.

Pins: the Cox-de Boor recursion against the closed-form uniform cubic
polynomials and partition of unity; the Gauss-Legendre rule against exact
polynomial integrals (the least-squares solve itself is pinned in
test_oracle_pins_hand.py); circle curvature 1/R; constant marker spacing after
relocation; the curvature-noise illustration of eq interpol_cir; sphere
mean curvature 2/R and translation invariance of the cotangent force.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import bspline, surface3d
from paper_1807_10504_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("u", [0.0, 0.1, 0.37, 0.5, 0.83, 0.999])
def test_cox_de_boor_uniform_closed_form(u):
    B3, B2 = bspline.cox_de_boor(u)
    ref3 = [(1 - u) ** 3 / 6, (3 * u ** 3 - 6 * u ** 2 + 4) / 6,
            (-3 * u ** 3 + 3 * u ** 2 + 3 * u + 1) / 6, u ** 3 / 6]
    ref2 = [(1 - u) ** 2 / 2, (-2 * u ** 2 + 2 * u + 1) / 2, u ** 2 / 2]
    assert max(abs(a - b) for a, b in zip(B3, ref3)) < 1e-15
    assert max(abs(a - b) for a, b in zip(B2, ref2)) < 1e-15
    assert abs(sum(B3) - 1.0) < 1e-15


def test_gauss_legendre_rule():
    assert abs(sum(bspline.GL_W) - 2.0) < 1e-15
    for p in range(0, 16):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        got = sum(w * x ** p for w, x in zip(bspline.GL_W, bspline.GL_X))
        assert abs(got - exact) < 1e-14


@pytest.mark.parametrize("n,R,h", [(128, 0.25, 1 / 64), (1024, 0.2, 1 / 512)])
def test_circle_curvature_and_spacing(n, R, h):
    X = W.circle_markers(n, R)
    Xn, fs, ds, nrm = bspline.relocate([tuple(x) for x in X], [(0.0, 0.0)] * n, 0.0, h, 1.0)
    fs = np.array(fs)
    assert np.max(np.abs(fs - 1.0 / R)) < 1e-3 / R
    Xn = np.array(Xn)
    ch = np.hypot(*(np.roll(Xn, -1, 0) - Xn).T)
    assert ch.max() - ch.min() < 1e-6 * h
    # the first marker stays where the old first marker was on the curve
    assert np.hypot(*(Xn[0] - X[0])) < 1e-6 * R
    nrm = np.array(nrm)
    inward = (np.array([0.5, 0.5]) - Xn) / R
    assert np.max(np.abs(nrm - inward)) < 1e-3


def test_curvature_noise_illustration():
    g = GOLD["curvature_noise"]
    X = W.perturbed_circle(g["n"], g["g"])
    # three-point circle through raw neighbours: strongly fluctuating
    a, c = np.roll(X, 1, 0), np.roll(X, -1, 0)
    ab = np.linalg.norm(X - a, axis=1)
    bc = np.linalg.norm(c - X, axis=1)
    ca = np.linalg.norm(a - c, axis=1)
    cr = np.abs((X - a)[:, 0] * (c - a)[:, 1] - (X - a)[:, 1] * (c - a)[:, 0])
    k3 = 2 * cr / (ab * bc * ca)
    assert k3.max() - k3.min() > 3.5
    # the least-squares B-spline removes it (knot spacing 1.5h, 1.9 markers/span)
    _, fs, _, _ = bspline.relocate([tuple(x) for x in X], [(0.0, 0.0)] * len(X), 0.0, 1 / 32, 1.0)
    assert max(abs(f - g["kappa_exact"]) for f in fs) < 0.05


def test_schoenberg_whitney_violation_raises():
    X = W.circle_markers(20, 0.3)
    with pytest.raises(bspline.BSplineError):
        bspline.relocate([tuple(x) for x in X], [(0.0, 0.0)] * 20, 0.0, 1 / 256, 1.0)


def test_advance_moves_markers():
    X = W.circle_markers(128, 0.25)
    U = [(1.0, -0.5)] * 128
    Xn, _, _, _ = bspline.relocate([tuple(x) for x in X], U, 1e-3, 1 / 64, 1.0)
    Xn = np.array(Xn)
    c = Xn.mean(axis=0)
    assert abs(c[0] - 0.501) < 1e-9 and abs(c[1] - 0.4995) < 1e-9


def test_sphere_mean_curvature_and_translation_invariance():
    V, T = W.sphere_mesh(4, 0.25, seed=3)
    fs, A, nrm, F = surface3d.surface_geometry(V, T, 1.0)
    assert abs(np.mean(fs) - 8.0) < 0.005 * 8.0
    # barycentric vertex areas overestimate curvature at the 12 valence-5 vertices
    assert np.percentile(np.abs(fs - 8.0), 99) < 0.01 * 8.0
    assert np.max(np.abs(fs - 8.0)) < 0.2 * 8.0
    assert np.max(np.abs(F.sum(axis=0))) < 1e-13 * np.abs(F).sum()
    assert abs(A.sum() - 4 * math.pi * 0.25 ** 2) < 0.01 * 4 * math.pi * 0.25 ** 2
    # normals point to the centre
    c = (np.array([0.5, 0.5, 0.5]) - V) / 0.25
    assert np.max(np.linalg.norm(nrm - c, axis=1)) < 0.02
