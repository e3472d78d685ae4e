"""Seeded synthetic inputs for the immersed-boundary projection step.

This module only builds input data: marker sets on analytic droplet shapes,
icosphere triangulations, seeded rotations and seeded velocity fields. It
holds none of the method's arithmetic (no kernels, no Heaviside, no
curvature, no solver), so both the HIP path and the CPU oracle draw their
inputs from it.

Geometry recipes (Section 5 of the paper and the workloads derived from it):
  * static circular drop: markers equispaced in angle, counter-clockwise
    (interior on the left), drop = heavy phase;
  * jittered circle: radius R(1 + a*xi_k), xi_k ~ U(-1, 1) from PCG64(seed);
  * mode-2 drop: r(theta) = R(1 + eps*cos(2 theta)) (oscillating-drop shape,
    Section 5.2), optional seeded modes 3..6;
  * the perturbed circle of the curvature-noise illustration (Section 2.2,
    eq interpol_cir): radius 0.5(1 +/- g), sign alternating with i;
  * level-L icosphere (10*4^L + 2 vertices), projected to radius R, rotated
    by a seeded uniform rotation and translated to the box centre; triangles
    are counter-clockwise seen from outside.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# 2D marker sets (closed, counter-clockwise polylines)
# ----------------------------------------------------------------------------
def circle_markers(n: int, R: float, centre=(0.5, 0.5)) -> np.ndarray:
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([centre[0] + R * np.cos(th), centre[1] + R * np.sin(th)], axis=1)


def jittered_circle(n: int, R: float, amp: float, seed: int, centre=(0.5, 0.5)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=n)
    th = 2.0 * np.pi * np.arange(n) / n
    r = R * (1.0 + amp * xi)
    return np.stack([centre[0] + r * np.cos(th), centre[1] + r * np.sin(th)], axis=1)


def axis_symmetric_shape(n: int, R: float, amp: float, seed: int, centre, modes=range(2, 7)) -> np.ndarray:
    """Markers on the meridian curve of a body of revolution about the axis
    x = centre[0]: r(psi) = R(1 + sum_m a_m cos(m psi)), psi the angle from the
    axis direction, a_m uniform in (-amp, amp) from PCG64(seed) for the modes
    given (even in psi, so the curve is mirror-symmetric about the axis)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-amp, amp, size=len(list(modes)))
    th = 2.0 * np.pi * np.arange(n) / n
    psi = th - 0.5 * np.pi
    r = np.ones(n)
    for am, m in zip(a, modes):
        r = r + am * np.cos(m * psi)
    r = R * r
    return np.stack([centre[0] + r * np.cos(th), centre[1] + r * np.sin(th)], axis=1)


def mode_shape(n: int, R: float, eps: float = 0.1, centre=(0.5, 0.5), seed: int | None = None,
               extra_amp: float = 0.0) -> np.ndarray:
    """r(theta) = R(1 + eps cos 2theta [+ sum_m a_m cos(m theta + phi_m), m = 3..6])."""
    th = 2.0 * np.pi * np.arange(n) / n
    r = 1.0 + eps * np.cos(2.0 * th)
    if seed is not None and extra_amp > 0.0:
        rng = np.random.default_rng(seed)
        for m in range(3, 7):
            a = rng.uniform(-extra_amp, extra_amp)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            r = r + a * np.cos(m * th + ph)
    r = R * r
    return np.stack([centre[0] + r * np.cos(th), centre[1] + r * np.sin(th)], axis=1)


def ellipse_markers(n: int, R: float, beta: float, centre=(0.5, 0.5)) -> np.ndarray:
    """eq osc: x = x' + R cos(theta) beta, y = y' + R sin(theta) / beta."""
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([centre[0] + R * np.cos(th) * beta, centre[1] + R * np.sin(th) / beta], axis=1)


def rotated_square_markers(h: float, angle_deg: float, L: float = 0.5, centre=(0.5, 0.5)):
    """Markers 0.5 h apart on the sides of a square of side L rotated by angle_deg
    about `centre`, counter-clockwise, with the inward unit normals of the sides
    and the arc element of each marker: (X, nrm, ds)."""
    th = np.deg2rad(angle_deg)
    m = int(round(L / (0.5 * h)))
    s = (np.arange(m) + 0.5) / m * L - L / 2
    rot = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    pts, nv = [], []
    for a, n in (((0, -1), (0, 1)), ((1, 0), (-1, 0)), ((0, 1), (0, -1)), ((-1, 0), (1, 0))):
        c = np.array(a, dtype=float) * L / 2
        t = np.array([-a[1], a[0]], dtype=float)
        pts.append(c + s[:, None] * t)
        nv.append(np.tile(n, (m, 1)).astype(float))
    X = np.concatenate(pts) @ rot.T + np.asarray(centre, dtype=float)
    nrm = np.concatenate(nv) @ rot.T
    return X, nrm, np.full(len(X), L / m)


def perturbed_circle(n: int = 126, g: float = 1e-3) -> np.ndarray:
    """Markers of the curvature-sensitivity illustration (eq interpol_cir).

    x_i = 0.5 + 0.5(1 +/- g) sin(2 pi i/n), y_i = 0.5 + 0.5(1 +/- g) cos(2 pi i/n),
    '+' for odd i and '-' for even i. As printed the points run clockwise; they
    are returned in reversed order so that the curve is counter-clockwise.
    """
    i = np.arange(n)
    sgn = np.where(i % 2 == 1, 1.0, -1.0)
    r = 0.5 * (1.0 + sgn * g)
    X = np.stack([0.5 + r * np.sin(2 * np.pi * i / n), 0.5 + r * np.cos(2 * np.pi * i / n)], axis=1)
    return np.ascontiguousarray(X[::-1])


# ----------------------------------------------------------------------------
# 3D triangulated spheres
# ----------------------------------------------------------------------------
def icosphere(level: int):
    """Unit icosphere: (V, T) with T counter-clockwise seen from outside."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    T = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        T2 = []
        for (a, b, c) in T:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            T2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        T = T2
    Vn = np.array(V)
    Tn = np.array(T, dtype=np.int32)
    # enforce outward counter-clockwise orientation
    a, b, c = Vn[Tn[:, 0]], Vn[Tn[:, 1]], Vn[Tn[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    Tn[flip] = Tn[flip][:, [0, 2, 1]]
    return Vn, Tn


def seeded_rotation(seed: int) -> np.ndarray:
    """Uniform random rotation: QR of a Gaussian matrix with sign fix, det = +1."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    Q, Rm = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(Rm))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def sphere_mesh(level: int, R: float, centre=(0.5, 0.5, 0.5), seed: int | None = 3):
    V, T = icosphere(level)
    if seed is not None:
        V = V @ seeded_rotation(seed).T
    V = np.asarray(centre, dtype=np.float64) + R * V
    return np.ascontiguousarray(V), np.ascontiguousarray(T)


def perturbed_sphere_mesh(level: int, R: float, amp: float, seed: int, centre=(0.5, 0.5, 0.5)):
    """Icosphere of mean radius R whose vertex radii carry a seeded smooth
    perturbation: r(v) = R (1 + amp * sum_k c_k P(v . a_k)), a_k three seeded
    unit axes, c_k ~ U(-1, 1), P(s) = (3 s^2 - 1) / 2 (an axisymmetric l = 2
    mode about each axis); with amp = 0 it is the sphere of sphere_mesh(seed)."""
    rng = np.random.default_rng(seed)
    V, T = icosphere(level)
    V = V @ seeded_rotation(seed).T
    axes = rng.standard_normal((3, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    c = rng.uniform(-1.0, 1.0, size=3)
    s = V @ axes.T
    r = R * (1.0 + amp * ((3.0 * s * s - 1.0) * 0.5) @ c)
    V = np.asarray(centre, dtype=np.float64) + r[:, None] * V
    return np.ascontiguousarray(V), np.ascontiguousarray(T)


# ----------------------------------------------------------------------------
# Fields
# ----------------------------------------------------------------------------
def random_faces(n, dim: int, scale: float, seed: int):
    """Seeded N(0, scale^2) MAC velocity components, each of cell-array shape (z,y,x)."""
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n[:dim]))
    return [scale * rng.standard_normal(shape) for _ in range(dim)]


def random_cells(n, dim: int, scale: float, seed: int):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(tuple(reversed(n[:dim])))


def network_init(seed: int, dim: int = 2, channels=(3, 32, 32, 32, 32, 32, 1)) -> np.ndarray:
    """He-normal initial weights (zero biases) of the warm-start network in the
    ABI's flat float32 layout: per layer W[co][ci][taps] then b[co], taps 3^dim."""
    rng = np.random.default_rng(seed)
    parts = []
    taps = 3 ** dim
    for l in range(6):
        ci, co = channels[l], channels[l + 1]
        std = np.sqrt(2.0 / (ci * taps)) if l < 5 else 0.1 * np.sqrt(1.0 / (ci * taps))
        parts.append((rng.standard_normal(co * ci * taps) * std).astype(np.float32))
        parts.append(np.zeros(co, dtype=np.float32))
    return np.concatenate(parts)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    dim: int
    n: tuple
    h: float
    rho_in: float
    rho_out: float
    sigma: float
    dt: float
    steps: int
    X: np.ndarray                      # markers (N x dim)
    tris: np.ndarray | None = None     # 3D triangles (M x 3), outward CCW
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(np.prod(self.n[: self.dim]))


def static_drop_2d_64() -> Workload:
    """64^2 unit periodic box, R = 0.25 centred, 128 equispaced markers."""
    n = (64, 64)
    return Workload("static_drop_2d_64", 2, n, 1.0 / 64, 1.0, 1e-3, 1.0, 1e-4, 10,
                    circle_markers(128, 0.25))


def static_drop_2d_512() -> Workload:
    """512^2, R = 0.2, 1024 markers with seeded 1e-3 R radial jitter (seed 2)."""
    n = (512, 512)
    return Workload("static_drop_2d_512", 2, n, 1.0 / 512, 1.0, 1e-3, 1.0, 2e-5, 200,
                    jittered_circle(1024, 0.2, 1e-3, seed=2))


def static_drop_3d(nc: int = 256, level: int = 6, seed: int = 3) -> Workload:
    """nc^3 periodic unit box, sphere R = 0.25 from a seeded-rotation icosphere."""
    V, T = sphere_mesh(level, 0.25, seed=seed)
    return Workload(f"static_drop_3d_{nc}", 3, (nc, nc, nc), 1.0 / nc, 1.0, 1e-3, 1.0, 5e-5, 100,
                    V, T)


def oscillating_drop_2d_512(seed: int | None = None) -> Workload:
    n = (512, 512)
    return Workload("oscillating_drop_2d_512", 2, n, 1.0 / 512, 1.0, 1e-3, 1.0, 2e-5, 1000,
                    mode_shape(1024, 0.2, 0.1, seed=seed, extra_amp=0.02 if seed is not None else 0.0))


def oscillating_drop_2d_osc(n: int = 256, h: float = 0.01, beta: float = 1.03,
                            markers: int = 256) -> Workload:
    """The free oscillation of Section 5 (Table osc): a drop of R = 0.2 stretched by
    beta (eq osc), densities 1 / 0.01, viscosities 0.01 / 1e-5, sigma = 1, on an
    n^2 periodic box of spacing h, centred; dt = 1e-4."""
    c = 0.5 * n * h
    return Workload(f"oscillating_drop_2d_{n}_h{h:g}", 2, (n, n), h, 1.0, 0.01, 1.0, 1e-4, 2600,
                    ellipse_markers(markers, 0.2, beta, centre=(c, c)),
                    extra=dict(mu_in=0.01, mu_out=1e-5, beta=beta, R=0.2))
