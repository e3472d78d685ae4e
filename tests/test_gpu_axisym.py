"""The axisymmetric projection step on the GPU against oracle.axisym.

* the static drop of Table staticdrop_axis (D = 0.4 on the axis, dx = 0.02,
  rho 1 / 0.01, one step of 1e-3): markers, sigma kappa (with the azimuthal
  term), H, F, p and u against the oracle, and the pressure jump within the
  band of the paper's errors;
* a moving case (seeded velocities, the mirrored interpolation and the
  relocation of moving markers): the same comparisons;
* the projected velocity has zero annular divergence;
* argument errors.
"""
import json
import os

import numpy as np
import pytest

from oracle import axisym as oaxi
from oracle import diag
from paper_1807_10504_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ib():
    from paper_1807_10504_amd import ibproj
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ibproj.load()
    return ibproj


def _run(ib, nr, nz, h, Xd, u, dt, rho_out=0.01, conventional=False):
    ax = ib.Axisym(nr, nz, h, max_markers=len(Xd))
    mg = ib.Multigrid(2, (nr, nz), h)
    prm = dict(rho_in=1.0, rho_out=rho_out, sigma=1.0, dt=dt, rtol=1e-12, warm_start=ib.WS_ZERO,
               spread_mode=ib.IB_SPREAD_DELTA if conventional else ib.IB_SPREAD_IRROT)
    X = Xd.copy()
    out = {"H": torch.empty((nz, nr), dtype=torch.float64, device="cuda"),
           "F": [torch.empty((nz, nr), dtype=torch.float64, device="cuda") for _ in range(2)],
           "fs_host": np.zeros(len(Xd))}
    out = ax.project_step(mg, prm, [dev(a) for a in u], X, out=out)
    ref = oaxi.project_step(nr, nz, h, 1.0, rho_out, 1.0, dt, u, Xd, rtol=1e-12, conventional=conventional)
    return X, out, ref


def _compare(X, out, ref):
    ex = np.abs(X - ref["X"]).max()
    efs = np.abs(out["fs_host"] - ref["fs"]).max() / np.abs(ref["fs"]).max()
    eH = np.abs(host(out["H"]) - ref["H"]).max()
    eF = max(np.abs(host(out["F"][d]) - ref["F"][d]).max() for d in range(2)) / \
        max(np.abs(f).max() for f in ref["F"])
    p = host(out["p"])
    ep = np.linalg.norm(p - ref["p"]) / np.linalg.norm(ref["p"])
    u = [host(c) for c in out["u"]]
    scale = max(max(np.abs(c).max() for c in ref["u"]), 1e-30)
    eu = max(np.abs(u[d] - ref["u"][d]).max() for d in range(2))
    print(f"X {ex:.1e}, sigma kappa {efs:.1e}, H {eH:.1e}, F {eF:.1e}, p {ep:.1e}, "
          f"u {eu:.1e} (max|u| {scale:.1e}); cycles {out['stats']['cycles']} / {ref['cycles']}")
    assert ex <= 1e-13 and efs <= 1e-13 and eH <= 1e-13 and eF <= 1e-11
    assert ep <= 1e-10
    return p, u, eu, scale


def test_static_drop_axis_parity_and_table(ib):
    g = GOLD["static_drop_axis_table"]
    h = g["dx"][0]
    nr, nz = 32, 64
    n = int(round(2 * np.pi * 0.2 / (0.63 * h))) // 4 * 4
    Xd = W.circle_markers(n, 0.2, centre=(nr * h, 0.5 * nz * h))
    zero = [np.zeros((nz, nr)), np.zeros((nz, nr))]
    X, out, ref = _run(ib, nr, nz, h, Xd, zero, 1e-3)
    p, u, eu, scale = _compare(X, out, ref)
    assert eu <= 1e-9 * max(scale, 1e-3)
    dp = diag.pressure_jump(p, host(out["H"]))
    err = abs(dp - 10.0)
    print(f"axisymmetric static drop, dx = {h}: dP = {dp:.6f}, |dP - 10| = {err:.3e} "
          f"(paper: new {g['new'][0]}, conventional {g['conventional'][0]})")
    assert err < 5.0 * max(g["conventional"])
    assert np.all(u[0][:, 0] == 0.0)


def test_static_drop_axis_conventional_parity(ib):
    """The conventional spreading on the meridian plane against the oracle; its
    pressure jump error at dx = 0.02 is of the size of the paper's conventional
    column."""
    g = GOLD["static_drop_axis_table"]
    h = g["dx"][0]
    nr, nz = 32, 64
    n = int(round(2 * np.pi * 0.2 / (0.63 * h))) // 4 * 4
    Xd = W.circle_markers(n, 0.2, centre=(nr * h, 0.5 * nz * h))
    zero = [np.zeros((nz, nr)), np.zeros((nz, nr))]
    X, out, ref = _run(ib, nr, nz, h, Xd, zero, 1e-3, conventional=True)
    p, u, eu, scale = _compare(X, out, ref)
    assert eu <= 1e-9 * max(scale, 1e-3)
    err = abs(diag.pressure_jump(p, host(out["H"])) - 10.0)
    print(f"conventional axisymmetric static drop, dx = {h}: |dP - 10| = {err:.3e} "
          f"(paper: conventional {g['conventional'][0]})")
    assert err < 5.0 * max(g["conventional"])


def test_moving_axis_parity_and_divergence(ib):
    nr, nz, h = 32, 32, 1.0 / 32
    rng = np.random.default_rng(91)
    u = [0.05 * rng.standard_normal((nz, nr)), 0.05 * rng.standard_normal((nz, nr))]
    u[0][:, 0] = 0.0
    Xd = W.circle_markers(96, 0.25, centre=(nr * h, 0.5))
    X, out, ref = _run(ib, nr, nz, h, Xd, u, 2e-3, rho_out=1e-3)
    eU = np.abs(host(out["U"]) - ref["U"]).max()
    assert eU <= 1e-14
    p, ug, eu, scale = _compare(X, out, ref)
    assert eu <= 1e-10 * scale
    div0 = np.abs(oaxi.divergence(u, h)).max()
    div1 = np.abs(oaxi.divergence(ug, h)).max()
    print(f"annular divergence {div0:.2e} -> {div1:.2e}")
    assert div1 <= 1e-8 * div0


def test_axis_errors(ib):
    import ctypes as C
    handle = C.c_void_p()
    g3 = ib.make_grid(3, (16, 16, 16), 1 / 16)
    assert ib.load().ib_axi_create(C.byref(g3), 64, C.byref(handle)) == ib.IB_EINVAL
    ax = ib.Axisym(16, 32, 1 / 16, 64)
    mg = ib.Multigrid(2, (16, 32), 1 / 16)
    u = [torch.zeros((32, 16), dtype=torch.float64, device="cuda") for _ in range(2)]
    X = W.circle_markers(32, 0.25, centre=(1.0, 1.0))
    for bad in (dict(spread_mode=7), dict(warm_start=ib.WS_NN)):
        prm = dict(rho_in=1.0, rho_out=0.01, dt=1e-3, **bad)
        with pytest.raises(ib.IbError):
            ax.project_step(mg, prm, u, X.copy())


# ---------------------------------------------------------------------------
# momentum predictor and full steps on the meridian plane
# ---------------------------------------------------------------------------
def _axi_fields(nr, nz, h, seed):
    rng = np.random.default_rng(seed)
    u = [rng.standard_normal((nz, nr)), rng.standard_normal((nz, nr))]
    u[0][:, 0] = 0.0
    k, i = np.indices((nz, nr))
    d = np.sqrt(((i + 0.5) * h) ** 2 + ((k + 0.5) * h - 0.5 * nz * h) ** 2)
    H = np.clip((0.3 - d) / (3 * h) + 0.5, 0.0, 1.0)
    from oracle import poisson
    return u, H, poisson.density(H, 1.0, 1e-3), poisson.density(H, 1e-2, 1e-4)


def test_axi_predict_parity_two_steps(ib):
    nr, nz = 32, 48
    h = 1.0 / 32
    dt = 2e-4
    u, H, rho, mu = _axi_fields(nr, nz, h, 93)
    from oracle import poisson
    rho1 = poisson.density(np.clip(H * 1.02, 0, 1), 1.0, 1e-3)
    ax = ib.Axisym(nr, nz, h, max_markers=16)
    us, st = ax.predict([dev(a) for a in u], dev(rho), dev(rho1), dev(mu), dt, rtol=1e-13)
    uo, adv = oaxi.predict(u, rho, rho1, mu, dt, h)
    errs = [np.linalg.norm(host(us[d]) - uo[d]) / np.linalg.norm(uo[d]) for d in range(2)]
    rng = np.random.default_rng(94)
    u2 = [a + 0.1 * rng.standard_normal((nz, nr)) for a in uo]
    u2[0][:, 0] = 0.0
    us2, st2 = ax.predict([dev(a) for a in u2], dev(rho1), dev(rho), dev(mu), dt, rtol=1e-13)
    uo2, _ = oaxi.predict(u2, rho1, rho, mu, dt, h, adv_prev=adv)
    errs += [np.linalg.norm(host(us2[d]) - uo2[d]) / np.linalg.norm(uo2[d]) for d in range(2)]
    print(f"meridian predictor: sweeps {st['sweeps']}, {st2['sweeps']}; rel L2 vs oracle {max(errs):.2e}")
    assert st["first_step"] == 1 and st2["first_step"] == 0
    assert max(errs) <= 1e-11
    assert np.all(host(us2[0])[:, 0] == 0.0)


def test_axi_flow_step_parity(ib):
    nr, nz = 32, 64
    h = 1.0 / 32
    prm = dict(rho_in=1.0, rho_out=1e-3, mu_in=1e-2, mu_out=1e-4, sigma=1.0, dt=1e-4, rtol=1e-12,
               pred_rtol=1e-13, warm_start=ib.WS_PREV)
    X0 = W.ellipse_markers(128, 0.25, 1.1, centre=(nr * h, 1.0))
    ax = ib.Axisym(nr, nz, h, max_markers=256)
    mg = ib.Multigrid(2, (nr, nz), h)
    u = [torch.zeros((nz, nr), dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros((nz, nr), dtype=torch.float64, device="cuda")
    Xg = X0.copy()
    from oracle import heaviside
    uo = [np.zeros((nz, nr)), np.zeros((nz, nr))]
    Xo = X0.copy()
    Ho = heaviside.heaviside_2d(Xo, (2 * nr, nz), h)[:, nr:]
    advo, po = None, None
    for step in range(3):
        out = ax.flow_step(mg, prm, u, Xg, p_prev=p, out={"p": p, "u": u})
        r = oaxi.flow_step(nr, nz, h, 1.0, 1e-3, 1e-2, 1e-4, 1.0, 1e-4, uo, Xo, Ho, adv_prev=advo,
                           p_prev=po, rtol=1e-12)
        uo, Xo, Ho, advo, po = r["u"], r["X"], r["H"], r["adv"], r["p"]
        eu = max(np.abs(host(u[d]) - uo[d]).max() for d in range(2)) / max(np.abs(a).max() for a in uo)
        ep = np.linalg.norm(host(p) - po) / np.linalg.norm(po)
        ex = np.abs(Xg - Xo).max()
        print(f"step {step}: sweeps {out['flow']['sweeps']}, cycles {out['stats']['cycles']} "
              f"(oracle {r['cycles']}); |du|/|u| {eu:.1e}, p {ep:.1e}, X {ex:.1e}", flush=True)
        assert eu <= 1e-9 and ep <= 1e-10 and ex <= 1e-12


def test_axi_flow_step_freefall_parity(ib):
    """Weight, restoring frame and mass correction (a volume 2e-4 above the
    initial one) on the meridian plane over three steps against the oracle."""
    from oracle import dynamics, heaviside
    nr, nz = 32, 64
    h = 1.0 / 32
    dt = 1e-4
    axis = nr * h
    X0 = W.ellipse_markers(128, 0.25, 1.1, centre=(axis, 1.0))
    V0, c0 = dynamics.measure(X0, axis)
    target = V0 * (1 + 2e-4)
    prm = dict(rho_in=1.0, rho_out=1e-3, mu_in=1e-2, mu_out=1e-4, sigma=1.0, dt=dt, rtol=1e-12,
               pred_rtol=1e-13, warm_start=ib.WS_PREV, gravity=-5.0, frame=True, mass_every=1,
               mass_target=target)
    ax = ib.Axisym(nr, nz, h, max_markers=256)
    mg = ib.Multigrid(2, (nr, nz), h)
    u = [torch.zeros((nz, nr), dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros((nz, nr), dtype=torch.float64, device="cuda")
    Xg = X0.copy()
    uo = [np.zeros((nz, nr)), np.zeros((nz, nr))]
    Xo = X0.copy()
    Ho = heaviside.heaviside_2d(Xo, (2 * nr, nz), h)[:, nr:]
    advo, po, c_prev = None, None, c0
    for step in range(3):
        _, c = dynamics.measure(Xo, axis)
        a = dynamics.frame_acceleration(c0, c_prev, c, dt)
        c_prev = c
        out = ax.flow_step(mg, prm, u, Xg, p_prev=p, out={"p": p, "u": u})
        r = oaxi.flow_step(nr, nz, h, 1.0, 1e-3, 1e-2, 1e-4, 1.0, dt, uo, Xo, Ho, adv_prev=advo,
                           p_prev=po, rtol=1e-12, gravity=-5.0, frame_a=a, mass_target=target)
        uo, Xo, Ho, advo, po = r["u"], r["X"], r["H"], r["adv"], r["p"]
        f = out["flow"]
        eu = max(np.abs(host(u[d]) - uo[d]).max() for d in range(2)) / max(np.abs(x).max() for x in uo)
        ep = np.linalg.norm(host(p) - po) / np.linalg.norm(po)
        ex = np.abs(Xg - Xo).max()
        print(f"step {step}: frame a {f['frame_a']:.3e} (oracle {a:.3e}), mass delta {f['mass_delta']:.2e}, "
              f"|du|/|u| {eu:.1e}, p {ep:.1e}, X {ex:.1e}", flush=True)
        assert abs(f["frame_a"] - a) <= 1e-7 and abs(f["com"] - c) <= 1e-12
        assert (f["mass_delta"] != 0.0) == (step == 0)
        # restored to 1e-12 by the correction, then within its trigger (1e-6)
        assert abs(dynamics.measure(Xg, axis)[0] - target) <= (2e-12 if step == 0 else 1e-6) * target
        assert eu <= 1e-9 and ep <= 1e-10 and ex <= 1e-12


def test_axi_oscillating_drop_period(ib):
    """Table osc, axisymmetric rows: the drop on the axis stretched by 1.03
    along r (eq osc), h = 0.01, rho 1 / 0.01, mu 0.01 / 1e-5; the first-cycle
    period within 5 % of eq aosc_p -- the largest discrepancy Table osc reports
    for the axisymmetric drop (4.84 %, new scheme at h = 0.02; 1.53 % at
    h = 0.01). The run differs from the paper's in its box (periodic along the
    axis, outer wall at r = 2.56) and in the first-order accuracy of the
    annular fluxes beside the axis."""
    nr, nz, h, dt = 256, 256, 0.01, 1e-4
    X = W.ellipse_markers(256, 0.2, 1.03, centre=(nr * h, 0.5 * nz * h))
    prm = dict(rho_in=1.0, rho_out=0.01, mu_in=0.01, mu_out=1e-5, sigma=1.0, dt=dt, rtol=1e-10,
               pred_rtol=1e-12, warm_start=ib.WS_PREV)
    ax = ib.Axisym(nr, nz, h, max_markers=len(X))
    mg = ib.Multigrid(2, (nr, nz), h, krylov=1)
    u = [torch.zeros((nz, nr), dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros((nz, nr), dtype=torch.float64, device="cuda")
    diam = [np.ptp(X[:, 0])]
    out = {"p": p, "u": u}
    for step in range(2300):
        out = ax.flow_step(mg, prm, u, X, p_prev=p, out=out)
        diam.append(np.ptp(X[:, 0]))
        if step % 500 == 0:
            print(f"step {step}: r-diameter {diam[-1]:.5f}, sweeps {out['flow']['sweeps']}, "
                  f"cycles {out['stats']['cycles']}", flush=True)
    d = np.array(diam)
    kmin = int(np.argmin(d[: len(d) // 2 + 200]))
    kmax = kmin + int(np.argmax(d[kmin:]))
    assert 0 < kmin < kmax < len(d) - 1, (kmin, kmax)
    y0, y1, y2 = d[kmax - 1], d[kmax], d[kmax + 1]
    T = (kmax + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt
    T_exact = GOLD["oscillation_periods"]["period_axisymmetric"]
    err = abs(T - T_exact) / T_exact
    T_paper = GOLD["oscillation_period_table_axis"]["period_new"][1]
    print(f"axisymmetric first-cycle period {T:.4f} (eq aosc_p {T_exact}, {100 * err:.2f} %; the paper's "
          f"new scheme at h = 0.01: {T_paper})")
    assert err <= 0.05
