"""Oracle pins for the momentum predictor (eqs ns1_new, ad_bf, cr_ni).

* advection of a uniform flow at uniform density vanishes; the surface sum
  conserves momentum (C / rho_f sums to zero over a periodic box, and C
  itself at uniform density);
* advection converges at second order to rho div(u u) = rho (u . grad) u
  (eq ns_1) for a Taylor-Green field with a smooth variable density (closed
  form);
* the viscous operator at constant mu has the discrete Fourier symbol
  mu sum_e (2 cos(2 pi k_e h) - 2)/h^2; with variable mu it is symmetric,
  negative semi-definite, kills constants and converges at second order to
  div(mu grad u_d);
* the predictor reduces to explicit Euler without viscosity (and Adams-
  Bashforth with a constant history to the same), and a single shear mode
  without advection is multiplied by the Crank-Nicolson factor
  (1 + dt lam / (2 rho)) / (1 - dt lam / (2 rho)).
"""
import numpy as np
import pytest

from oracle import flow


def _faces(n, d):
    """Face coordinates (x, y) of component d on an n x n unit periodic grid."""
    h = 1.0 / n
    j, i = np.indices((n, n))
    x = (i + (0.0 if d == 0 else 0.5)) * h
    y = (j + (0.0 if d == 1 else 0.5)) * h
    return x, y


def _cells(n):
    h = 1.0 / n
    j, i = np.indices((n, n))
    return (i + 0.5) * h, (j + 0.5) * h


def test_advection_uniform_flow_uniform_density_is_zero():
    n = 16
    u = [np.full((n, n), 0.7), np.full((n, n), -1.3)]
    C = flow.advection(u, np.full((n, n), 2.5), 1.0 / n)
    assert all(np.all(c == 0.0) for c in C)
    u3 = [np.full((4, 6, 8), v) for v in (0.3, -0.2, 0.9)]
    C3 = flow.advection(u3, np.full((4, 6, 8), 1.7), 0.125)
    assert all(np.all(c == 0.0) for c in C3)
    # a drop carried by a uniform flow is not accelerated (eq ns_1: rho div(u u)),
    # whatever the density field; the density inside the flux would add u u . grad rho
    rho = 0.01 + np.random.default_rng(2).random((n, n))
    C = flow.advection(u, rho, 1.0 / n)
    assert all(np.all(c == 0.0) for c in C)


@pytest.mark.parametrize("shape", [(12, 16), (6, 8, 10)])
def test_advection_conserves_momentum(shape):
    rng = np.random.default_rng(4)
    dim = len(shape)
    u = [rng.standard_normal(shape) for _ in range(dim)]
    rho = 0.1 + rng.random(shape)
    C = flow.advection(u, rho, 0.1)
    for d, c in enumerate(C):
        q = c / flow.face_density(rho, dim, d)
        assert abs(q.sum()) <= 1e-12 * np.abs(q).sum()
    C = flow.advection(u, np.full(shape, 0.6), 0.1)
    for c in C:
        assert abs(c.sum()) <= 1e-12 * np.abs(c).sum()


def _tg_error(n):
    h = 1.0 / n
    tp = 2 * np.pi
    u, exact = [], []
    xc, yc = _cells(n)
    rho = 1.0 + 0.5 * np.sin(tp * xc) * np.sin(tp * yc)
    for d in range(2):
        x, y = _faces(n, d)
        U = np.sin(tp * x) * np.cos(tp * y)
        V = -np.cos(tp * x) * np.sin(tp * y)
        r = 1.0 + 0.5 * np.sin(tp * x) * np.sin(tp * y)
        # rho div(u u) = rho (u . grad) u   (div u = 0);
        # (u . grad) u = (pi sin 4 pi x, pi sin 4 pi y) for this field
        conv = np.pi * np.sin(2 * tp * (x if d == 0 else y))
        exact.append(r * conv)
        u.append(U if d == 0 else V)
    C = flow.advection(u, rho, h)
    return max(np.abs(C[d] - exact[d]).max() for d in range(2))


def test_advection_second_order_taylor_green():
    e1, e2 = _tg_error(32), _tg_error(64)
    rate = e1 / e2
    assert e2 < 5e-2     # of a field of size ~10
    assert 3.6 < rate < 4.4, rate


def test_viscous_fourier_symbol():
    n = 16
    h = 1.0 / n
    mu = 0.37
    for d in range(2):
        x, y = _faces(n, d)
        k = (2, 3)
        ud = np.cos(2 * np.pi * (k[0] * x + k[1] * y))
        u = [ud if e == d else np.zeros_like(ud) for e in range(2)]
        D = flow.viscous(u, np.full((n, n), mu), h)
        lam = mu * sum((2 * np.cos(2 * np.pi * ke * h) - 2) / (h * h) for ke in k)
        assert np.abs(D[d] - lam * ud).max() <= 1e-11 * abs(lam)
        assert np.all(D[1 - d] == 0.0)


@pytest.mark.parametrize("shape", [(8, 12), (4, 6, 8)])
def test_viscous_symmetric_negative(shape):
    rng = np.random.default_rng(5)
    dim = len(shape)
    mu = 0.01 + rng.random(shape)
    u = [rng.standard_normal(shape) for _ in range(dim)]
    w = [rng.standard_normal(shape) for _ in range(dim)]
    h = 0.2
    Du, Dw = flow.viscous(u, mu, h), flow.viscous(w, mu, h)
    lhs = sum(np.sum(a * b) for a, b in zip(Du, w))
    rhs = sum(np.sum(a * b) for a, b in zip(u, Dw))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    assert sum(np.sum(a * b) for a, b in zip(Du, u)) < 0.0
    Dc = flow.viscous([np.full(shape, 3.0) for _ in range(dim)], mu, h)
    assert all(np.abs(c).max() <= 1e-12 for c in Dc)
    for d in range(dim):
        M = flow.viscous_matrix(mu, h, d, dim)
        assert abs(M - M.T).max() <= 1e-12 * abs(M).max()
        assert np.allclose(M @ u[d].ravel(), Du[d].ravel(), rtol=0, atol=1e-10 * np.abs(Du[d]).max())


def _visc_error(n):
    h = 1.0 / n
    tp = 2 * np.pi
    xc, yc = _cells(n)
    mu = 1.0 + 0.5 * np.cos(tp * xc) * np.sin(tp * yc)
    err = 0.0
    for d in range(2):
        x, y = _faces(n, d)
        f = np.sin(tp * x) * np.sin(2 * tp * y)
        fx, fy = tp * np.cos(tp * x) * np.sin(2 * tp * y), 2 * tp * np.sin(tp * x) * np.cos(2 * tp * y)
        fxx, fyy = -tp * tp * f, -4 * tp * tp * f
        m = 1.0 + 0.5 * np.cos(tp * x) * np.sin(tp * y)
        mx, my = -0.5 * tp * np.sin(tp * x) * np.sin(tp * y), 0.5 * tp * np.cos(tp * x) * np.cos(tp * y)
        exact = m * (fxx + fyy) + mx * fx + my * fy
        u = [f if e == d else np.zeros_like(f) for e in range(2)]
        err = max(err, np.abs(flow.viscous(u, mu, h)[d] - exact).max())
    return err


def test_viscous_second_order_variable_mu():
    e1, e2 = _visc_error(32), _visc_error(64)
    assert 3.6 < e1 / e2 < 4.4, e1 / e2


def test_predictor_reduces_to_euler_without_viscosity():
    rng = np.random.default_rng(6)
    shape = (8, 10)
    u = [rng.standard_normal(shape) for _ in range(2)]
    rho_n = 0.5 + rng.random(shape)
    rho1 = 0.5 + rng.random(shape)
    dt, h = 1e-3, 0.1
    zero = np.zeros(shape)
    us, adv = flow.predict(u, rho_n, rho1, zero, dt, h)
    us2, _ = flow.predict(u, rho_n, rho1, zero, dt, h, adv_prev=adv)
    for d in range(2):
        rf = 0.5 * (rho1 + np.roll(rho1, 1, axis=1 - d))
        euler = u[d] - dt * adv[d] / rf
        assert np.abs(us[d] - euler).max() <= 1e-14 * np.abs(u[d]).max()
        assert np.abs(us2[d] - euler).max() <= 1e-14 * np.abs(u[d]).max()


def test_predictor_crank_nicolson_factor():
    n = 16
    h = 1.0 / n
    rho, mu, dt = 0.8, 0.05, 0.02
    x, y = _faces(n, 0)
    ud = np.cos(2 * np.pi * y)          # a shear mode: no advection
    u = [ud, np.zeros_like(ud)]
    us, adv = flow.predict(u, np.full((n, n), rho), np.full((n, n), rho), np.full((n, n), mu), dt, h)
    assert np.abs(adv[0]).max() <= 1e-14 and np.abs(adv[1]).max() <= 1e-14
    lam = mu * (2 * np.cos(2 * np.pi * h) - 2) / (h * h)
    g = (1 + 0.5 * dt * lam / rho) / (1 - 0.5 * dt * lam / rho)
    assert np.abs(us[0] - g * ud).max() <= 1e-13
    assert np.abs(us[1]).max() <= 1e-14


def test_oscillation_period_formulas_match_printed_values():
    """eqs osc_p and aosc_p with n = 2, r = 0.2, sigma = 1 give the printed
    periods for drop density 1 and ambient 0.01 (the reading of the garbled
    parameter sentence of Section 5.2 that the flow tests use)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    n, r, sigma, rd, ra = 2, 0.2, 1.0, 1.0, 0.01
    t2 = 2 * np.pi * np.sqrt((rd + ra) * r ** 3 / ((n ** 3 - n) * sigma))
    tax = 2 * np.pi * np.sqrt(((n + 1) * rd + n * ra) * r ** 3 / (n * (n - 1) * (n + 1) * (n + 2) * sigma))
    assert abs(t2 - gold["oscillation_periods"]["period_2d"]) < 5e-6
    assert abs(tax - gold["oscillation_periods"]["period_axisymmetric"]) < 5e-6
    tab = gold["oscillation_period_table_2d"]
    for T, pct in zip(tab["period_new"], tab["discrepancy_new_percent"]):
        assert abs(100 * abs(T - t2) / t2 - pct) < 0.02


def test_table_osc_axis_rows_match_eq_aosc_p():
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    T = gold["oscillation_periods"]["period_axisymmetric"]
    tab = gold["oscillation_period_table_axis"]
    for Tn, pct in zip(tab["period_new"], tab["discrepancy_new_percent"]):
        assert abs(100 * abs(Tn - T) / T - pct) < 0.02
