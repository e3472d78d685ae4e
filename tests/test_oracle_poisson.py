"""Oracle pins: operator, multigrid, mixed precision, right side and update.

Pins: dense direct solve of the bordered system on 16^2 and 8^3 at density
ratio 1000; diagonalisation (FFT) for constant coefficients; a discrete
manufactured solution; second-order convergence for a continuous one;
symmetry of A; divergence-free corrected velocity (the projection property).
Flexible CG: finite termination with the identity preconditioner (plain CG),
one iteration with the exact inverse, the dense direct solve and FFT solve
when converged, and fewer V-cycles than plain multigrid on a drop.
"""
import numpy as np
import pytest

from oracle import poisson
from paper_1807_10504_amd import workloads as W


def _drop_beta(shape, ratio=1000.0):
    dim = len(shape)
    n = shape[0]
    g = np.indices(shape)
    r2 = sum(((g[a] + 0.5) / n - 0.5) ** 2 for a in range(dim))
    H = (r2 < 0.3 ** 2).astype(float)
    return poisson.face_beta(poisson.density(H, 1.0, 1.0 / ratio))


@pytest.mark.parametrize("shape", [(16, 16), (8, 8, 8)])
def test_multigrid_matches_dense_direct(shape):
    beta = _drop_beta(shape)
    h = 1.0 / shape[0]
    b = W.random_cells(tuple(reversed(shape)), len(shape), 1.0, seed=21)
    b -= b.mean()
    pd = poisson.direct_solve(b, beta, h)
    pm, cyc, hist = poisson.mg_solve(b, beta, h, rtol=1e-13)
    assert hist[-1] <= 1e-13
    assert np.max(np.abs(pm - pd)) <= 1e-10 * np.max(np.abs(pd))
    assert abs(pm.mean()) < 1e-14 * np.max(np.abs(pd))


@pytest.mark.parametrize("shape", [(32, 32), (16, 16, 16)])
def test_constant_coefficient_fft(shape):
    dim = len(shape)
    h = 1.0 / shape[0]
    beta = [np.full(shape, 0.7) for _ in range(dim)]
    b = W.random_cells(tuple(reversed(shape)), dim, 1.0, seed=5)
    b -= b.mean()
    pf = poisson.fft_solve(b, 0.7, h)
    pm, _, _ = poisson.mg_solve(b, beta, h, rtol=1e-13)
    assert np.max(np.abs(pm - pf)) <= 1e-10 * np.max(np.abs(pf))


def test_discrete_manufactured_solution_ratio_1000():
    shape = (64, 64)
    h = 1.0 / 64
    beta = _drop_beta(shape)
    pex = W.random_cells(shape, 2, 1.0, seed=8)
    pex -= pex.mean()
    b = poisson.apply_A(pex, beta, h)
    p, cyc, hist = poisson.mg_solve(b, beta, h, rtol=1e-13)
    assert np.linalg.norm(p - pex) <= 1e-9 * np.linalg.norm(pex)


def test_continuous_manufactured_second_order():
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(x, x, indexing="xy")
        xf = np.arange(n) * h
        # beta(x, y) = 2 + sin(2 pi x) sampled on faces
        bx = 2.0 + np.sin(2 * np.pi * xf)[None, :] * np.ones((n, 1))
        by = 2.0 + np.sin(2 * np.pi * X)
        pex = np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        # div(beta grad p) with beta = 2 + sin(2 pi x)
        px = -2 * np.pi * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        pxx = -4 * np.pi ** 2 * pex
        pyy = -4 * np.pi ** 2 * pex
        beta_c = 2.0 + np.sin(2 * np.pi * X)
        f = beta_c * (pxx + pyy) + 2 * np.pi * np.cos(2 * np.pi * X) * px
        f -= f.mean()
        p, _, _ = poisson.mg_solve(f, [bx, by], h, rtol=1e-12)
        errs.append(np.max(np.abs(p - (pex - pex.mean()))))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4)])
def test_operator_symmetric_and_null_space(shape):
    beta = _drop_beta(shape)
    h = 1.0 / shape[0]
    A = poisson.dense_matrix(beta, h)
    assert np.max(np.abs(A - A.T)) <= 1e-12 * np.max(np.abs(A))
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) <= 1e-12 * np.max(np.abs(A))


def test_restriction_prolongation_transfer_constants():
    e = np.full((4, 4, 4), 3.0)
    assert np.max(np.abs(poisson.prolong(e) - 3.0)) == 0.0
    r = W.random_cells((8, 8, 8), 3, 1.0, seed=1)
    assert abs(poisson.restrict(r).sum() * 8 - r.sum()) < 1e-12
    # linear in x along one axis: interior fine values follow the line exactly
    x = np.arange(8, dtype=float)
    e1 = np.tile(x, (8, 1))
    f = poisson.prolong(e1)
    xf = (np.arange(16) + 0.5) / 2 - 0.5
    assert np.max(np.abs(f[3, 1:15] - xf[1:15])) < 1e-14


def test_coarsen_beta_means_fine_faces():
    b = [W.random_cells((8, 8), 2, 1.0, seed=s) for s in (1, 2)]
    c = poisson.coarsen_beta(b)
    assert abs(c[0][1, 2] - 0.5 * (b[0][2, 4] + b[0][3, 4])) < 1e-15
    assert abs(c[1][1, 2] - 0.5 * (b[1][2, 4] + b[1][2, 5])) < 1e-15


@pytest.mark.parametrize("shape", [(64, 64), (16, 16, 16)])
def test_mixed_precision_reaches_fp64_tolerance(shape):
    beta = _drop_beta(shape)
    h = 1.0 / shape[0]
    b = W.random_cells(tuple(reversed(shape)), len(shape), 1.0, seed=31)
    b -= b.mean()
    p64, c64, h64 = poisson.mg_solve(b, beta, h, rtol=1e-10)
    p32, c32, h32 = poisson.mg_solve_mixed(b, beta, h, rtol=1e-10)
    assert h32[-1] <= 1e-10
    assert c32 <= c64 + 2
    pt, _, _ = poisson.mg_solve(b, beta, h, rtol=1e-14, max_cycles=200)
    assert np.linalg.norm(p32 - pt) <= 1e-7 * np.linalg.norm(pt)


def test_mixed_precision_from_float32_densities():
    """The float32 cycle whose finest coefficients are formed in float32 from
    float32 densities: uniform density gives exactly 1/fl32(rho) on every face,
    a face across a jump is 2 / (fl32(rho_L) + fl32(rho_R)) rounded once, and
    the defect correction still reaches 1e-10 with an answer within the FP64
    error bound."""
    r = np.full((4, 4), 0.3)
    for f in poisson.face_beta_f32(r):
        assert f.dtype == np.float32
        assert np.all(f == np.float32(1.0) / np.float32(0.3))
    r[1, 2] = 1e-3
    fx = poisson.face_beta_f32(r)[0]
    assert fx[1, 2] == np.float32(2.0) / np.float32(np.float32(1e-3) + np.float32(0.3))
    shape = (32, 32, 32)
    g = np.indices(shape)
    rr = np.sqrt(sum(((g[a] + 0.5) / 32 - 0.5) ** 2 for a in range(3)))
    rho = poisson.density(np.clip((0.3 - rr) * 32 / 3 + 0.5, 0.0, 1.0), 1.0, 1e-3)
    beta = poisson.face_beta(rho)
    h = 1.0 / 32
    b = W.random_cells(shape, 3, 1.0, seed=33)
    b -= b.mean()
    pt, _, _ = poisson.mg_solve(b, beta, h, rtol=1e-14, max_cycles=200)
    p32, c32, h32 = poisson.mg_solve_mixed(b, beta, h, rtol=1e-10, rho=rho)
    assert h32[-1] <= 1e-10
    assert np.linalg.norm(p32 - pt) <= 1e-7 * np.linalg.norm(pt)
    pk, ck, hk = poisson.mg_pcg(b, beta, h, rtol=1e-10, mixed=True, rho=rho)
    assert hk[-1] <= 1e-10 and ck < c32
    assert np.linalg.norm(pk - pt) <= 1e-7 * np.linalg.norm(pt)


def test_projection_makes_velocity_divergence_free():
    shape = (32, 32)
    h = 1.0 / 32
    beta = _drop_beta(shape)
    us = W.random_faces((32, 32), 2, 1.0, seed=3)
    F = W.random_faces((32, 32), 2, 5.0, seed=4)
    dt = 1e-3
    b = poisson.rhs(us, F, beta, dt, h)
    assert abs(b.sum()) < 1e-9 * np.abs(b).sum()
    p, _, _ = poisson.mg_solve(b, beta, h, rtol=1e-13)
    u = poisson.velocity_update(us, F, beta, p, dt, h)
    div = poisson.divergence(u, h)
    assert np.max(np.abs(div)) <= 1e-9 * np.max(np.abs(poisson.divergence(us, h)))


# ----------------------------------------------------------------------------
# flexible CG preconditioned by multigrid
def test_fcg_finite_termination_identity_preconditioner():
    """With M = I the method is plain CG: on an SPD matrix with m distinct
    eigenvalues it reaches the solution in at most m iterations (exact
    arithmetic; here to ~1e-12). A wrong alpha or beta breaks this."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.repeat([1.0, 2.0, 5.0, 11.0, 30.0], [3, 3, 2, 2, 2])
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(12)
    x, it, hist = poisson.fcg(lambda v: A @ v, lambda r: r.copy(), b, rtol=1e-12, max_iter=50)
    assert it <= 5
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_fcg_exact_preconditioner_one_iteration():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((10, 10))
    A = M @ M.T + 10 * np.eye(10)
    Ainv = np.linalg.inv(A)
    b = rng.standard_normal(10)
    x, it, hist = poisson.fcg(lambda v: A @ v, lambda r: Ainv @ r, b, rtol=1e-12)
    assert it == 1
    assert np.linalg.norm(x - Ainv @ b) <= 1e-12 * np.linalg.norm(Ainv @ b)


@pytest.mark.parametrize("shape", [(16, 16), (8, 8, 8)])
def test_mg_pcg_matches_dense_direct(shape):
    beta = _drop_beta(shape)
    h = 1.0 / shape[0]
    b = W.random_cells(tuple(reversed(shape)), len(shape), 1.0, seed=22)
    b -= b.mean()
    pd = poisson.direct_solve(b, beta, h)
    p, it, hist = poisson.mg_pcg(b, beta, h, rtol=1e-13)
    assert hist[-1] <= 1e-13
    assert np.max(np.abs(p - pd)) <= 1e-10 * np.max(np.abs(pd))
    # the recursive residual tracks the true one
    true = np.linalg.norm(b - poisson.apply_A(p, beta, h)) / np.linalg.norm(b)
    assert true <= 1e-12


def test_mg_pcg_constant_coefficient_fft():
    shape = (16, 16, 16)
    h = 1.0 / 16
    beta = [np.full(shape, 0.7) for _ in range(3)]
    b = W.random_cells(shape, 3, 1.0, seed=6)
    b -= b.mean()
    p, _, _ = poisson.mg_pcg(b, beta, h, rtol=1e-13)
    pf = poisson.fft_solve(b, 0.7, h)
    assert np.max(np.abs(p - pf)) <= 1e-10 * np.max(np.abs(pf))


def test_mg_pcg_fewer_iterations_than_vcycles_and_mixed():
    """Drop at density ratio 1000 on 32^3: the Krylov wrapper needs fewer
    V-cycles than plain multigrid for the same stopping test, and the mixed
    (float32 preconditioner) variant converges to the same answer."""
    shape = (32, 32, 32)
    beta = _drop_beta(shape)
    h = 1.0 / 32
    b = W.random_cells(shape, 3, 1.0, seed=23)
    b -= b.mean()
    pm, cyc, _ = poisson.mg_solve(b, beta, h, rtol=1e-10)
    p, it, hist = poisson.mg_pcg(b, beta, h, rtol=1e-10)
    p32, it32, _ = poisson.mg_pcg(b, beta, h, rtol=1e-10, mixed=True)
    assert it < cyc
    assert np.linalg.norm(p - pm) <= 1e-8 * np.linalg.norm(pm)
    assert np.linalg.norm(p32 - p) <= 1e-8 * np.linalg.norm(p)
