"""Oracle pins: cosine kernel, Heaviside profile, interpolation and spreading.

Every check here fixes the oracle against something other than itself: the
closed-form identities of the kernel, a numerical integral of it, the
paper's printed region values, brute force over all faces, and the
adjoint/partition-of-unity identities of the transfer operators.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import kernel, transfer
from paper_1807_10504_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_kernel_partition_of_unity_and_parity_sums():
    # Section 2.2: "the sum over all grid points must be equal to one"
    q = np.linspace(-3.0, 3.0, 2001)
    s = sum(kernel.phi(q - j) for j in range(-6, 7))
    se = sum(kernel.phi(q - j) for j in range(-6, 7, 2))
    assert np.max(np.abs(s - 1.0)) < 1e-15
    assert np.max(np.abs(se - 0.5)) < 1e-15


def test_kernel_support_strict():
    assert kernel.phi(2.0) == 0.0 and kernel.phi(-2.0) == 0.0
    assert kernel.phi(1.9999999) > 0.0
    assert kernel.phi(0.0) == 0.5


def test_heaviside_profile_is_integral_of_kernel():
    for q in (-2.0, -1.3, -1.0, -0.2, 0.0, 0.7, 1.0, 1.8, 2.0):
        ref, _ = quad(lambda r: float(kernel.phi(r)), -2.0, q, epsabs=1e-15, epsrel=1e-13, limit=200)
        assert abs(float(kernel.heaviside_profile(q)) - ref) < 1e-13


def test_region_values_match_paper():
    g = GOLD["heaviside_region_values"]
    v = kernel.region_values()
    assert v[0] == 0.0 and abs(v[4] - 1.0) < 1e-15
    assert round(v[2], 3) == g["region_III"]
    assert round(v[3], 3) == g["region_IV"]
    # symmetry H(-q) = 1 - H(q) fixes region II
    assert abs(v[1] - (1.0 - v[3])) < 1e-15
    assert abs(v[3] - (0.75 + 1.0 / (2.0 * math.pi))) < 1e-15
    assert abs(sum(kernel.region_jumps()) - 1.0) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_matches_bruteforce(dim):
    n = (8, 8) if dim == 2 else (6, 6, 6)
    h = 1.0 / n[0]
    rng = np.random.default_rng(11)
    # markers anywhere, including next to the periodic seam
    X = rng.uniform(0.0, 1.0, size=(5, dim))
    X[0, 0] = 0.01
    X[1, 1] = 0.995
    u = W.random_faces(n, dim, 1.0, seed=4)
    U = transfer.interp(u, X, h)
    Ub = transfer.interp_bruteforce(u, X, h)
    assert np.max(np.abs(U - Ub)) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_constant_field_exact(dim):
    n = (16,) * dim
    h = 1.0 / 16
    X = np.random.default_rng(3).uniform(0, 1, size=(40, dim))
    u = [np.full(tuple(reversed(n)), 1.0 + d) for d in range(dim)]
    U = transfer.interp(u, X, h)
    for d in range(dim):
        assert np.max(np.abs(U[:, d] - (1.0 + d))) < 1e-14


def test_interp_not_exact_for_linear_fields():
    # the first moment of the cosine kernel is not zero: a linear field is
    # not reproduced exactly (a plausible "symmetric kernel" mistake would be)
    q = 0.3
    m1 = sum((q - j) * kernel.phi(q - j) for j in range(-3, 4))
    assert abs(m1) > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_spread_total_and_adjoint(dim):
    n = (16,) * dim
    h = 1.0 / 16
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, size=(30, dim))
    Fs = rng.standard_normal((30, dim))
    F = transfer.spread_delta(Fs, X, n, h)
    tot = np.array([F[d].sum() for d in range(dim)]) * h ** dim
    assert np.max(np.abs(tot - Fs.sum(axis=0))) < 1e-12 * np.abs(Fs).sum()
    u = W.random_faces(n, dim, 1.0, seed=9)
    U = transfer.interp(u, X, h)
    lhs = float(np.sum(U * Fs))
    rhs = float(sum(np.sum(u[d] * F[d]) for d in range(dim)) * h ** dim)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_spread_bruteforce_tiny():
    n = (8, 8)
    h = 1.0 / 8
    X = np.array([[0.31, 0.77], [0.02, 0.5]])
    Fs = np.array([[1.0, -2.0], [0.5, 0.25]])
    F = transfer.spread_delta(Fs, X, n, h)
    for d in range(2):
        for j in range(8):
            for i in range(8):
                xf = np.array([(i + (0.0 if d == 0 else 0.5)) * h, (j + (0.0 if d == 1 else 0.5)) * h])
                acc = 0.0
                for s in range(2):
                    dx = xf - X[s]
                    dx -= np.round(dx)
                    acc += Fs[s, d] * float(kernel.phi(dx[0] / h) * kernel.phi(dx[1] / h)) / h ** 2
                assert abs(F[d][j, i] - acc) < 1e-12
