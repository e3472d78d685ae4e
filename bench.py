"""Projection-step throughput on one MI355X.

Workload (the headline configuration): static spherical drop in a 256^3
periodic unit box, sphere R = 0.25 from a level-6 icosphere (40,962 markers,
81,920 triangles) under a seeded rotation, density ratio 1000, sigma = 1,
dt = 5e-5, multigrid to ||r||/||b|| <= 1e-10. A step is one full pass of the
hot path through the C ABI (project_step): interpolation, spreading with the
irrotational delta vector (offset-polyhedron Heaviside + face force),
coefficients, right side, multigrid solve warm-started from the previous
pressure, velocity update; the next step starts from the updated velocity.

Every step solves from p = 0 ("cold"): a static drop warm-started from the
previous pressure already meets the 1e-10 test after the first step, so a
warm-started step would measure no multigrid at all. The warm-started
variant is reported beside it.

Variants: plain FP64 multigrid (the JSON `value`), float32 V-cycles inside
FP64 defect correction (same stopping test), each cold and warm.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "projection steps/s @256³, ρ ratio 1000, resid≤1e-10; FP64 vs mixed+NN"
HBM_PEAK_GBS = 8000.0
# one red-black sweep reads p, b and three face coefficients and writes p:
# 6 x 8 bytes per cell (float64); one launch updates one colour = half a sweep.
# This per-cell figure is the algorithmic traffic of the sweep the roofline
# reports. The sweep that forms the coefficients from cell densities moves
# less: it reads p, b, rho and writes p, 4 x 8 bytes per cell (reported beside).
SWEEP_BYTES_F64 = 48.0
SWEEP_BYTES_F64_RHO = 32.0
SWEEP_BYTES_F32 = 24.0
# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000, the factors an elementwise copy of
# known size reads), recorded with the kernel they were taken on; any other
# kernel reports null
TRAFFIC = {"k_rbgs_fused_rho<32,16,512>": (707.4e6, "profiles/rbgs_fused_rho_256cube_hbm_counters.txt")}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_variant(ib, torch, wl, geo, precision, steps, warmup, profile, warm=False, krylov=0, nn=None):
    n, h = wl.n, wl.h
    shape = tuple(reversed(n))
    V, T = wl.X, wl.tris
    fs, ds, nrm = geo
    Vd = torch.from_numpy(V).cuda()
    Td = torch.from_numpy(T.astype(np.int32)).cuda()
    fsd, dsd, nd = (torch.from_numpy(a).cuda() for a in (fs, ds, nrm))
    surf = ib.make_surface(Vd, elems=Td, nrm=nd, fs=fsd, ds=dsd)
    ctx = ib.Context(3, n, h, max_markers=len(V), max_elems=len(T))
    mg = ib.Multigrid(3, n, h, precision=precision, krylov=krylov)
    params = dict(rho_in=wl.rho_in, rho_out=wl.rho_out, sigma=wl.sigma, dt=wl.dt, rtol=1e-10,
                  max_cycles=100, warm_start=ib.WS_PREV if warm else ib.WS_ZERO)
    if nn is not None:
        # cold start from the network's guess (from b and 1/rho alone)
        params["warm_start"] = ib.WS_NN
    u = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    bufs = [dict(p=torch.empty(shape, dtype=torch.float64, device="cuda"),
                 u=[torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(3)],
                 U=torch.empty((len(V), 3), dtype=torch.float64, device="cuda"))
            for _ in range(2)]
    p_prev = None
    cycles = []
    res = []
    first = None

    accepted = []

    def one(k):
        nonlocal u, p_prev
        out = bufs[k % 2]
        out = ctx.project_step(mg, params, u, p_prev=None if nn is not None else p_prev, surf=surf,
                               out=out, nn=nn)
        u, p_prev = out["u"], out["p"]
        if nn is not None:
            accepted.append(out["guess"]["accepted"])
        return out["stats"]

    for k in range(warmup):
        st = one(k)
        if first is None:
            first = st
    torch.cuda.synchronize()
    if profile:
        ib.profile_reset()
        ib.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(steps):
        st = one(warmup + k)
        cycles.append(st["cycles"])
        res.append(st["rel_res"])
        if (k + 1) % max(1, steps // 4) == 0:
            log(f"  step {k + 1}/{steps}: cycles={st['cycles']} rel_res={st['rel_res']:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        ib.profile_enable(False)
        prof = ib.profile_read()
    d = ctx.diagnostics(p=p_prev, u=u)
    ctx.close()
    mg.close()
    return dict(seconds=t1 - t0, steps=steps, cycles=cycles, rel_res=res, first=first, prof=prof,
                dP=d["dP"], tke=d["tke"], accepted=accepted)


def precision_errors(ib, torch, wl, geo):
    """p of the first step's right side from each solver against a tightly
    converged FP64 solve (relative L2): what the 1e-10 stopping test and the
    float32 V-cycles leave in the answer."""
    n, h = wl.n, wl.h
    shape = tuple(reversed(n))
    fs, ds, nrm = geo
    keep = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
            for a in (wl.X, wl.tris.astype(np.int32), nrm, fs, ds)]
    surf = ib.make_surface(keep[0], elems=keep[1], nrm=keep[2], fs=keep[3], ds=keep[4])
    ctx = ib.Context(3, n, h, max_markers=len(wl.X), max_elems=len(wl.tris))
    mg = ib.Multigrid(3, n, h, krylov=1)
    u0 = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    out = dict(b=torch.empty(shape, dtype=torch.float64, device="cuda"),
               H=torch.empty(shape, dtype=torch.float64, device="cuda"))
    prm = dict(rho_in=wl.rho_in, rho_out=wl.rho_out, sigma=wl.sigma, dt=wl.dt, rtol=1e-10,
               warm_start=ib.WS_ZERO)
    out = ctx.project_step(mg, prm, u0, surf=surf, out=out)
    b = out["b"]
    rho = ctx.density(out["H"], wl.rho_in, wl.rho_out)
    mg.close()
    res = {}
    ref = None
    for name, prec, kry, rtol in (("fp64_tight", ib.MG_FP64, 1, 1e-13), ("fp64_fcg", ib.MG_FP64, 1, 1e-10),
                                  ("mixed_fcg", ib.MG_MIXED, 1, 1e-10), ("fp64_vcycle", ib.MG_FP64, 0, 1e-10),
                                  ("mixed_vcycle", ib.MG_MIXED, 0, 1e-10)):
        m = ib.Multigrid(3, n, h, precision=prec, krylov=kry)
        m.update_density(rho)
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        st = m.solve(b, p, rtol=rtol, max_cycles=60, allow_notconv=True)
        true = m.residual_norm(b, p)
        m.close()
        if ref is None:
            ref = p
            res[name] = dict(cycles=st["cycles"], true_rel_res=true)
            continue
        err = ((p - ref).norm() / ref.norm()).item()
        res[name] = dict(cycles=st["cycles"], true_rel_res=true, p_rel_l2_vs_fp64_tight=err)
    ctx.close()
    return res


def bench_3d_nn(ib, torch, wl, geo, steps, warmup, sps64, pairs=24, train_iters=60):
    """Learned warm start at the full 3D size: the 3D network is trained on cold FP64
    solutions of perturbed spheres (random radius 0.2-0.3, l = 2 modes of amplitude
    0.15; not the benchmark sphere) and then gives the cold-start guess of the
    benchmark step, evaluated by flexible CG in FP64 and mixed precision."""
    from paper_1807_10504_amd import workloads as W
    n, h = wl.n, wl.h
    shape = tuple(reversed(n))
    V0, T0 = wl.X, wl.tris
    ctx = ib.Context(3, n, h, max_markers=len(V0), max_elems=len(T0))
    mg = ib.Multigrid(3, n, h, krylov=1)
    prm = dict(rho_in=wl.rho_in, rho_out=wl.rho_out, sigma=wl.sigma, dt=wl.dt, rtol=1e-10,
               warm_start=ib.WS_ZERO)
    t0 = time.perf_counter()
    samples = []
    for s in range(pairs):
        seed = 1000 + s
        R = 0.2 + 0.1 * np.random.default_rng(seed).uniform()
        V, T = W.perturbed_sphere_mesh(6, R, 0.15, seed)
        fs, ds, nrm = ib.surface_geometry_3d(V, T, wl.sigma)
        keep = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (V, T.astype(np.int32), nrm, fs, ds)]
        surf = ib.make_surface(keep[0], elems=keep[1], nrm=keep[2], fs=keep[3], ds=keep[4])
        u0 = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        o = dict(b=torch.empty(shape, dtype=torch.float64, device="cuda"),
                 H=torch.empty(shape, dtype=torch.float64, device="cuda"))
        o = ctx.project_step(mg, prm, u0, surf=surf, out=o)
        samples.append((o["b"], o["H"], None, o["p"].clone()))
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    ctx.close()
    mg.close()
    net = ib.Network(n, h)
    net.set_params(W.network_init(1, dim=3))
    rng = np.random.default_rng(3)
    losses = []
    t0 = time.perf_counter()
    for it in range(train_iters):
        idx = rng.choice(pairs, size=4, replace=False)
        losses.append(net.train_step([samples[i] for i in idx], wl.rho_in, wl.rho_out, 2e-3))
        if (it + 1) % max(1, train_iters // 4) == 0:
            log(f"  training {it + 1}/{train_iters}: loss {losses[-1]:.3e}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    b, H = samples[0][0], samples[0][1]
    g = net.predict(b, H, None, wl.rho_in, wl.rho_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        net.predict(b, H, None, wl.rho_in, wl.rho_out, p0=g)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / 5
    del samples, b, H, g
    out = dict(workload=f"{pairs} perturbed spheres at {n[0]}^3 (level-6 meshes, R 0.2-0.3, l=2 modes of "
                        f"amplitude 0.15) -> training pairs from cold FP64 solves; evaluated on the benchmark "
                        f"sphere (not in the training set)",
               pairs_s=round(t_pairs, 2), train_iters=train_iters, train_s=round(t_train, 2),
               loss_first=float(np.mean(losses[:5])), loss_last=float(np.mean(losses[-10:])),
               inference_ms=round(1e3 * t_inf, 3))
    # useful work of one inference: 2 x 27 taps x c_in x c_out per voxel and layer
    # (channels 3 -> 32 x 5 -> 1), against the dense bf16 matrix-core peak
    chans = (3, 32, 32, 32, 32, 32, 1)
    flop = 2.0 * 27 * sum(a * b for a, b in zip(chans[:-1], chans[1:])) * n[0] * n[1] * n[2]
    out["inference_tflops"] = round(flop / t_inf / 1e12, 1)
    out["inference_frac_bf16_peak"] = round(flop / t_inf / 2.5e15, 3)
    for name, prec in (("fp64", ib.MG_FP64), ("mixed", ib.MG_MIXED)):
        log(f"== {name} flexible CG from the 3D network's guess, cold every step")
        r = run_variant(ib, torch, wl, geo, prec, steps, warmup, profile=False, krylov=1, nn=net)
        sps = r["steps"] / r["seconds"]
        out[f"{name}_cold_fcg_nn"] = dict(
            steps_per_s=round(sps, 3), ms_per_step=round(1e3 * r["seconds"] / r["steps"], 3),
            mean_cycles=float(np.mean(r["cycles"])), max_rel_res=float(np.max(r["rel_res"])),
            guess_accepted=float(np.mean(r["accepted"])) if r["accepted"] else 0.0,
            speedup_vs_fp64_cold=round(sps / sps64, 3))
    net.close()
    return out


def bench_2d_c2(ib, torch, steps=200):
    """512^2 jittered static drop, warm-started steps: FP64 vs mixed multigrid."""
    from paper_1807_10504_amd import workloads as W
    wl = W.static_drop_2d_512()
    shape = tuple(reversed(wl.n))
    out = {}
    for name, prec in (("fp64", ib.MG_FP64), ("mixed", ib.MG_MIXED)):
        ctx = ib.Context(2, wl.n, wl.h, max_markers=len(wl.X))
        mg = ib.Multigrid(2, wl.n, wl.h, precision=prec)
        X = wl.X.copy()
        u = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(2)]
        p_prev = None
        prm = dict(rho_in=wl.rho_in, rho_out=wl.rho_out, sigma=wl.sigma, dt=wl.dt, rtol=1e-10)
        cyc = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            o = ctx.project_step(mg, prm, u, p_prev=p_prev, X_host=X)
            u, p_prev = o["u"], o["p"]
            cyc.append(o["stats"]["cycles"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        d = ctx.diagnostics(p=p_prev, u=u)
        out[name] = dict(steps_per_s=round(steps / dt, 2), mean_cycles=float(np.mean(cyc)),
                         tke=d["tke"], p=p_prev.cpu().numpy())
    diff = float(np.linalg.norm(out["mixed"].pop("p") - out["fp64"]["p"]) / np.linalg.norm(out["fp64"]["p"]))
    out["fp64"].pop("p")
    out["mixed_vs_fp64_p_rel_l2_after_steps"] = diff
    out["workload"] = (f"static_drop_2d_512: 512^2, R=0.2, 1024 markers with 1e-3 R seeded jitter, rho ratio "
                       f"1000, dt=2e-5, {steps} steps warm-started from p_prev, B-spline relocation each step")
    return out


def _osc_period(d, dt):
    """First return of the diameter signal to its maximum after its first minimum
    (parabola through the three samples around the discrete maximum)."""
    d = np.asarray(d)
    kmin = int(np.argmin(d[: len(d) // 2 + 200]))
    kmax = kmin + int(np.argmax(d[kmin:]))
    y0, y1, y2 = d[kmax - 1], d[kmax], d[kmax + 1]
    return float((kmax + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt)


def _osc_run(ib, torch, axis, n, h, dt, steps, markers, spread_mode=None):
    """Full flow steps of the Table osc drop (R = 0.2 stretched by 1.03, rho 1/0.01,
    mu 0.01/1e-5, sigma 1) on an n^2 periodic box (2D) or n x n meridian half plane."""
    from paper_1807_10504_amd import workloads as W
    prm = dict(rho_in=1.0, rho_out=0.01, mu_in=0.01, mu_out=1e-5, sigma=1.0, dt=dt, rtol=1e-10,
               pred_rtol=1e-12, warm_start=ib.WS_PREV,
               spread_mode=ib.IB_SPREAD_IRROT if spread_mode is None else spread_mode)
    mg = ib.Multigrid(2, (n, n), h, krylov=1)
    if axis:
        X = W.ellipse_markers(markers, 0.2, 1.03, centre=(n * h, 0.5 * n * h))
        solver = ib.Axisym(n, n, h, max_markers=markers)
        step = lambda u, p, out: solver.flow_step(mg, prm, u, X, p_prev=p, out=out)
    else:
        X = W.ellipse_markers(markers, 0.2, 1.03, centre=(0.5 * n * h, 0.5 * n * h))
        ctx = ib.Context(2, (n, n), h, max_markers=markers)
        fl = ib.Flow(2, (n, n), h)
        step = lambda u, p, out: ctx.flow_step(mg, fl, prm, u, X, p_prev=p, out=out)
    u = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    out = {"p": p, "u": u}
    diam = [float(np.ptp(X[:, 0]))]
    sweeps, cycles = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = step(u, p, out)
        diam.append(float(np.ptp(X[:, 0])))
        sweeps.append(out["flow"]["sweeps"])
        cycles.append(out["stats"]["cycles"])
        if k % 2000 == 1999:
            log(f"  {'axisymmetric' if axis else '2D'} h={h}: flow step {k + 1}/{steps}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return dict(period=round(_osc_period(diam, dt), 5), steps=steps, steps_per_s=round(steps / secs, 2),
                ms_per_step=round(1e3 * secs / steps, 3), mean_predictor_sweeps=round(float(np.mean(sweeps)), 2),
                mean_cycles=round(float(np.mean(cycles)), 2))


def _osc_history(ib, torch, spread_mode, beta, steps, every, n=256, h=0.01, dt=1e-4, markers=256,
                 indicator_density=False):
    """The Table osc drop (reading of Section 5.2: R = 0.2, rho 1/0.01, mu 0.01/1e-5,
    sigma 1) stretched by beta, full flow steps with the irrotational or the
    conventional spreading; every `every` steps: TKE (eq tke), the axis ratio, and
    |sum of the grid force| / sum over markers of |sigma kappa| ds."""
    from paper_1807_10504_amd import workloads as W
    prm = dict(rho_in=1.0, rho_out=0.01, mu_in=0.01, mu_out=1e-5, sigma=1.0, dt=dt, rtol=1e-10,
               pred_rtol=1e-12, warm_start=ib.WS_PREV, spread_mode=spread_mode,
               indicator_density=indicator_density)
    mg = ib.Multigrid(2, (n, n), h, krylov=1)
    X = W.ellipse_markers(markers, 0.2, beta, centre=(0.5 * n * h, 0.5 * n * h))
    ctx = ib.Context(2, (n, n), h, max_markers=markers)
    fl = ib.Flow(2, (n, n), h)
    u = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    F = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(2)]
    fs = np.zeros(markers)
    out = {"p": p, "u": u, "F": F, "fs_host": fs}
    hist = dict(t=[], tke=[], axis_ratio=[], force_ratio=[])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = ctx.flow_step(mg, fl, prm, u, X, p_prev=p, out=out)
        if (k + 1) % every == 0:
            d = ctx.diagnostics(u=u, F=F)
            edge = np.linalg.norm(np.roll(X, -1, 0) - X, axis=1)
            ds = 0.5 * (edge + np.roll(edge, 1))
            hist["t"].append(round((k + 1) * dt, 6))
            hist["tke"].append(float(f"{d['tke']:.4e}"))
            hist["axis_ratio"].append(round(float(np.ptp(X[:, 0]) / np.ptp(X[:, 1])), 5))
            hist["force_ratio"].append(float(f"{np.hypot(*d['force_sum'][:2]) / np.sum(np.abs(fs) * ds):.3e}"))
    torch.cuda.synchronize()
    hist["steps_per_s"] = round(steps / (time.perf_counter() - t0), 2)
    return hist


def bench_osc_energy(ib, torch, steps=10000, every=100):
    """Eq tke over the first second of the Table osc drop (h = 0.01) with the new and
    the conventional spreading (the paper's TKE figure: the new scheme's decays, the
    conventional one's is held up by parasitic currents), per 0.2 s window its mean
    and its floor (the minimum, where the oscillation's kinetic energy passes
    through zero); and the large deformation beta = 1.3 with its grid-force ratio
    (the paper: at most of order 1e-4)."""
    res = {}
    win = max(1, int(round(0.2 / (every * 1e-4))))
    for name, mode, ind in (("new", ib.IB_SPREAD_IRROT, False), ("conventional", ib.IB_SPREAD_DELTA, False),
                            ("conventional_indicator", ib.IB_SPREAD_DELTA, True)):
        r = _osc_history(ib, torch, mode, 1.03, steps, every, indicator_density=ind)
        tke = np.array(r["tke"])
        res[f"tke_{name}"] = dict(
            window_s=0.2, steps_per_s=r["steps_per_s"],
            mean=[float(f"{tke[k:k + win].mean():.3e}") for k in range(0, len(tke), win)],
            floor=[float(f"{tke[k:k + win].min():.3e}") for k in range(0, len(tke), win)],
            force_ratio_max=max(r["force_ratio"]))
        log(f"  TKE {name}: window means {res[f'tke_{name}']['mean']}, floors {res[f'tke_{name}']['floor']}, "
            f"{r['steps_per_s']} steps/s")
    res["floor_ratio_conventional_over_new"] = [round(c / n, 2) for c, n in
                                                zip(res["tke_conventional"]["floor"], res["tke_new"]["floor"])]
    r = _osc_history(ib, torch, ib.IB_SPREAD_IRROT, 1.3, 4000, 50)
    res["deform_beta1.3"] = dict(steps=4000, t_end=0.4, steps_per_s=r["steps_per_s"],
                                 axis_ratio_min=min(r["axis_ratio"]), axis_ratio_max=max(r["axis_ratio"]),
                                 force_ratio_max=max(r["force_ratio"]),
                                 force_ratio_mean=float(f"{np.mean(r['force_ratio']):.3e}"))
    log(f"  beta 1.3: axis ratio {min(r['axis_ratio'])} .. {max(r['axis_ratio'])}, force ratio max "
        f"{max(r['force_ratio']):.2e}")
    res["workload"] = ("Table osc drop (R=0.2, rho 1/0.01, mu 0.01/1e-5, sigma 1) at h=0.01 on 256^2, dt 1e-4, "
                       "256 markers: beta 1.03 for 1 s with the new and the conventional spreading (the latter "
                       "also with the properties from the indicator of eq ind_psn; eq tke every "
                       "0.01 s), beta 1.3 for 0.4 s (axis ratio; |sum of grid force| / sum |sigma kappa| ds "
                       "every 0.005 s)")
    return res


def bench_conventional(ib, torch):
    """Section 3.1's curl study and the conventional indicator (eq ind_psn): for a
    circle R = 0.2 with a unit inward force, max |index-form curl| / max |F| of the
    split (conventional) and irrotational delta vectors, and the indicator's L1
    distance to the smoothed Heaviside, h = 1/64 ... 1/1024; the indicator solve's
    time (flexible-CG multigrid to 1e-10)."""
    from paper_1807_10504_amd import workloads as W
    rows = []
    for nn in (64, 128, 256, 512, 1024):
        h = 1.0 / nn
        m = int(round(2 * np.pi * 0.2 / (0.5 * h)))
        X0 = W.circle_markers(m, 0.2)
        X, _, ds, nrm = ib.relocate_bspline(X0, np.zeros_like(X0), 0.0, h, 1.0)
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, np.ones(m), ds, nrm)]
        surf = ib.Surface()
        surf.n_markers, surf.X, surf.fs, surf.ds, surf.nrm = (m, t[0].data_ptr(), t[1].data_ptr(),
                                                              t[2].data_ptr(), t[3].data_ptr())
        ctx = ib.Context(2, (nn, nn), h, max_markers=m)
        F, H = ctx.spread(surf, ib.IB_SPREAD_IRROT)
        Fc, _ = ctx.spread(surf, ib.IB_SPREAD_DELTA, want_H=False)
        d, dc = ctx.diagnostics(F=F), ctx.diagnostics(F=Fc)
        ind = ib.Indicator((nn, nn), h, max_markers=m)
        I, st = ind.solve(ctx, t[0], t[3], t[2], rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            I, st = ind.solve(ctx, t[0], t[3], t[2], rtol=1e-10, I=I)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / 5
        l1 = float((I - H).abs().sum()) * h * h
        rows.append(dict(h=f"1/{nn}", curl_over_fmax_conventional=round(dc["curl_max"] / dc["f_max"], 5),
                         curl_over_fmax_irrotational=float(f"{d['curl_max'] / d['f_max']:.2e}"),
                         indicator_l1_vs_H=float(f"{l1:.4e}"), indicator_cg_iterations=st["cycles"],
                         indicator_ms=round(ms, 3)))
        log(f"  h=1/{nn}: curl/|F| conventional {rows[-1]['curl_over_fmax_conventional']}, irrotational "
            f"{rows[-1]['curl_over_fmax_irrotational']}; L1 |I - H| {l1:.3e}; indicator {ms:.2f} ms")
    for a, b in zip(rows, rows[1:]):
        b["l1_ratio"] = round(a["indicator_l1_vs_H"] / b["indicator_l1_vs_H"], 3)
    return dict(rows=rows, workload="circle R=0.2 centred in the unit periodic box, markers 0.5 h apart "
                                    "(B-spline relocation), unit force toward the drop")


def _osc3d_run(ib, torch, nn, level, dt, frac):
    """A drop R = 0.25 stretched by 1.1 along x (volume kept), rho 1/0.01, mu
    0.01/1e-5, sigma 1, on an nn^3 unit periodic box, level-`level` icosphere,
    moving-surface flow steps over `frac` of Lamb's l = 2 period: the time of
    the first minimum of the x-extent (parabola through the samples around it)."""
    from paper_1807_10504_amd import workloads as W
    R, beta = 0.25, 1.1
    h = 1.0 / nn
    V, T = W.sphere_mesh(level, R, seed=3)
    V = 0.5 + (V - 0.5) * np.array([beta, 1 / np.sqrt(beta), 1 / np.sqrt(beta)])
    prm = dict(rho_in=1.0, rho_out=0.01, mu_in=0.01, mu_out=1e-5, sigma=1.0, dt=dt, rtol=1e-10,
               pred_rtol=1e-12, warm_start=ib.WS_PREV)
    n = (nn, nn, nn)
    ctx = ib.Context(3, n, h, max_markers=len(V), max_elems=len(T))
    mg = ib.Multigrid(3, n, h, krylov=1)
    fl = ib.Flow(3, n, h)
    u = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    p = torch.zeros(n, dtype=torch.float64, device="cuda")
    T_lamb = 2 * np.pi * np.sqrt((3 * 1.0 + 2 * 0.01) * R ** 3 / 24.0)
    steps = int(frac * T_lamb / dt)
    ext = [float(np.ptp(V[:, 0]))]
    cycles, sweeps = [], []
    out = {"p": p, "u": u}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = ctx.flow_step(mg, fl, prm, u, V, p_prev=p, out=out, tris=T)
        ext.append(float(np.ptp(V[:, 0])))
        cycles.append(out["stats"]["cycles"])
        sweeps.append(out["flow"]["sweeps"])
        if k % 1000 == 999:
            log(f"  3D drop {nn}^3: step {k + 1}/{steps}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    d = np.array(ext)
    k = int(np.argmin(d))
    y0, y1, y2 = d[k - 1], d[k], d[k + 1]
    t_min = (k + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt
    return dict(vertices=len(V), triangles=len(T), steps=steps, steps_per_s=round(steps / secs, 2),
                ms_per_step=round(1e3 * secs / steps, 3), half_period=round(float(t_min), 5),
                lamb_half_period=round(0.5 * T_lamb, 5),
                discrepancy_percent=round(100 * abs(t_min - 0.5 * T_lamb) / (0.5 * T_lamb), 2),
                x_extent_start=round(d[0], 5), x_extent_min=round(float(d[k]), 5),
                mean_cycles=round(float(np.mean(cycles)), 2), mean_predictor_sweeps=round(float(np.mean(sweeps)), 2))


def bench_flow3d(ib, torch):
    """Moving 3D drops (local least-squares surface reconstruction): the first
    half-period of the l = 2 oscillation against Lamb's formula, and full steps/s,
    at h = 1/64 (level-4 icosphere) and 1/128 (level 5)."""
    res = {}
    for nn, level, dt in ((64, 4, 2e-4), (128, 5, 1e-4)):
        r = _osc3d_run(ib, torch, nn, level, dt, 0.62)
        res[f"h1_{nn}"] = r
        log(f"  3D drop {nn}^3: half period {r['half_period']} (Lamb {r['lamb_half_period']}, "
            f"{r['discrepancy_percent']} %), {r['steps_per_s']} steps/s")
    res["workload"] = ("drop R=0.25 stretched by 1.1 along x (volume kept), rho 1/0.01, mu 0.01/1e-5, sigma 1, "
                       "unit periodic box; 64^3 with a level-4 icosphere (2562 vertices), dt 2e-4; 128^3 with "
                       "level 5 (10242 vertices), dt 1e-4; 0.62 of Lamb's l = 2 period")
    return res


def bench_flow_osc(ib, torch):
    """Full flow steps (markers, H and force, momentum predictor, projection) on the
    free oscillation of Section 5.2 (Table osc), 2D and axisymmetric, at h = 0.01
    and 0.005: steps/s and the first-cycle period against eqs osc_p / aosc_p and
    the paper's new-scheme values."""
    T2 = 2 * np.pi * np.sqrt(1.01 * 0.2 ** 3 / 6.0)
    Ta = 2 * np.pi * np.sqrt((3 * 1.0 + 2 * 0.01) * 0.2 ** 3 / 24.0)
    res = {}
    for axis, T, paper in ((False, T2, {0.02: 0.2411, 0.01: 0.2346, 0.005: 0.2328}),
                           (True, Ta, {0.02: 0.2090, 0.01: 0.2024})):
        for h, n, dt, steps, nm in ((0.02, 128, 2e-4, 1300 if not axis else 1150, 128),
                                    (0.01, 256, 1e-4, 2600 if not axis else 2300, 256),
                                    (0.005, 512, 5e-5, 5200 if not axis else 4600, 512)):
            r = _osc_run(ib, torch, axis, n, h, dt, steps, nm)
            r["discrepancy_percent"] = round(100 * abs(r["period"] - T) / T, 2)
            r["exact_period"] = round(float(T), 5)
            if h in paper:
                r["paper_new_scheme"] = paper[h]
            res[f"{'axis' if axis else '2d'}_h{h:g}"] = r
            log(f"  {'axisymmetric' if axis else '2D'} h={h}: period {r['period']} ({r['discrepancy_percent']} %), "
                f"{r['steps_per_s']} steps/s")
    # the conventional spreading's periods (Table osc's other column)
    for axis, T, h, n, dt, steps, nm, paper in ((False, T2, 0.02, 128, 2e-4, 1300, 128, 0.2348),
                                                (False, T2, 0.01, 256, 1e-4, 2600, 256, 0.2334),
                                                (False, T2, 0.005, 512, 5e-5, 5200, 512, 0.2326),
                                                (True, Ta, 0.02, 128, 2e-4, 1150, 128, 0.2044),
                                                (True, Ta, 0.01, 256, 1e-4, 2300, 256, 0.2039)):
        r = _osc_run(ib, torch, axis, n, h, dt, steps, nm, spread_mode=ib.IB_SPREAD_DELTA)
        r["discrepancy_percent"] = round(100 * abs(r["period"] - T) / T, 2)
        r["exact_period"] = round(float(T), 5)
        r["paper_conventional"] = paper
        res[f"{'axis' if axis else '2d'}_conventional_h{h:g}"] = r
        log(f"  {'axisymmetric' if axis else '2D'} conventional h={h}: period {r['period']} "
            f"({r['discrepancy_percent']} %), {r['steps_per_s']} steps/s")
    res["workload"] = ("Table osc drop: R=0.2 stretched by 1.03 (eq osc), rho 1/0.01, mu 0.01/1e-5, sigma=1; "
                       "2D: n^2 periodic box; axisymmetric: n x n meridian half plane (axis, outer wall at "
                       "r = n h, periodic along the axis); n = 128 at h = 0.02 (dt 2e-4), 256 at h = 0.01 "
                       "(dt 1e-4), 512 at h = 0.005 "
                       "(dt 5e-5); AB2 advection, Crank-Nicolson viscosity, irrotational force, FCG projection "
                       "warm-started from p_prev; markers 0.5 h apart")
    return res


# Table afd_param sets 1 and 2 (D = 1, rho_ambient = 1, sigma = 1, d = v = 10):
# g from the Eotvos number, mu_ambient from the Morton number
AFD_SETS = {1: (0.3, 3.333e-4), 2: (9.0, 1.440e-2)}


def _free_fall_run(ib, torch, eo, mo, h=0.0125, nr=128, nz=256, dt=5e-4, steps=8000, markers=512):
    """Axisymmetric free fall of a D = 1 drop (Section 5.3, Table afd_param) in the
    restoring non-inertial frame (c1 = c2 = 0.1), weight (rho - rho_mean) g along -z,
    mass correction every 20 steps. Slip Reynolds number rho_a D |W_a - W_d| / mu_a
    from the r-weighted mean axial velocities of the ambient (H = 0) and drop (H = 1)
    cells."""
    from paper_1807_10504_amd import workloads as W
    rho_a, rho_d, sigma, D = 1.0, 10.0, 1.0, 1.0
    g = eo * sigma / ((rho_d - rho_a) * D * D)
    mu_a = (mo * rho_a ** 2 * sigma ** 3 / (g * (rho_d - rho_a))) ** 0.25
    prm = dict(rho_in=rho_d, rho_out=rho_a, mu_in=10 * mu_a, mu_out=mu_a, sigma=sigma, dt=dt, rtol=1e-10,
               pred_rtol=1e-12, warm_start=ib.WS_PREV, gravity=-g, frame=True, c1=0.1, c2=0.1,
               mass_every=20)
    mg = ib.Multigrid(2, (nr, nz), h, krylov=1)
    axis = nr * h
    X = W.circle_markers(markers, 0.5 * D, centre=(axis, 0.5 * nz * h))
    solver = ib.Axisym(nr, nz, h, max_markers=markers)
    u = [torch.zeros((nz, nr), dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros((nz, nr), dtype=torch.float64, device="cuda")
    H = torch.zeros((nz, nr), dtype=torch.float64, device="cuda")
    out = {"p": p, "u": u, "H": H}
    rc = ((torch.arange(nr, dtype=torch.float64, device="cuda") + 0.5) * h)[None, :]
    re_hist, com_hist, vol_hist, corrections = [], [], [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = solver.flow_step(mg, prm, u, X, p_prev=p, out=out)
        f = out["flow"]
        com_hist.append(f["com"])
        vol_hist.append(f["measure"])
        corrections += f["mass_delta"] != 0.0
        if k % 200 == 199:
            wz = 0.5 * (u[1] + torch.roll(u[1], -1, 0))      # cell-centred axial velocity
            wd = float((wz * H * rc).sum() / (H * rc).sum())
            wa = float((wz * (1 - H) * rc).sum() / ((1 - H) * rc).sum())
            re_hist.append(rho_a * D * abs(wa - wd) / mu_a)
        if k % 2000 == 1999:
            log(f"  free fall Eo={eo}: step {k + 1}/{steps}, Re {re_hist[-1]:.4f}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    v0 = vol_hist[0]
    return dict(eotvos=eo, morton=mo, g=round(g, 6), mu_ambient=round(mu_a, 6), steps=steps, t_end=steps * dt,
                steps_per_s=round(steps / secs, 2), ms_per_step=round(1e3 * secs / steps, 3),
                reynolds_end=round(re_hist[-1], 5),
                reynolds_change_last_10pct=round(abs(re_hist[-1] - re_hist[-len(re_hist) // 10 - 1]) /
                                                 re_hist[-1], 5),
                reynolds_every_0p1=[round(r, 4) for r in re_hist],
                com_drift_over_D=float(f"{abs(com_hist[-1] - com_hist[0]) / D:.3e}"),
                volume_rel_change_max=float(f"{max(abs(v - v0) for v in vol_hist) / v0:.3e}"),
                mass_corrections=int(corrections))


def bench_c5(ib, torch, steps=2000, train_steps=400, train_iters=600, nr=256, nz=1024):
    """Axisymmetric free-falling water drop in air, SI units: (r, z) meridian half
    plane of nr x nz cells, h = 31.25 um (8 mm x 32 mm), drop radius 1 mm on the
    axis, rho 1000 / 1.2 kg/m^3, mu 1e-3 / 1.8e-5 Pa s, sigma 0.072 N/m, g 9.81,
    512 contour markers on a shape with seeded modes 2..6 of amplitude <= 1 %
    (mirror-symmetric about the axis); restoring frame, weight, mass correction every 20 steps; multigrid in
    mixed precision (float32 V(2,2) cycles in float64 defect correction; the
    flexible CG loses positivity of (r, V r) on this r-weighted system, so the
    plain cycles are the solver here). Two runs from
    the same start: both take train_steps steps warm-started from p_prev, whose
    pairs (b, 1/rho, p_prev -> p) train the warm network; then one continues
    `steps` steps with the learned warm start (multigrid judging every guess),
    the other from p_prev."""
    from paper_1807_10504_amd import workloads as W
    h = 8e-3 / nr
    R = 1e-3
    # the capillary limit sqrt(rho_mean h^3 / (2 pi sigma)) is 5.8e-6 s; at 5e-6 s the
    # air flow (density ratio 833) grows unstable within ~800 steps, at 1e-6 s it
    # stays below 0.2 m/s
    dt = 1e-6
    prm = dict(rho_in=1000.0, rho_out=1.2, mu_in=1e-3, mu_out=1.8e-5, sigma=0.072, dt=dt, rtol=1e-10,
               pred_rtol=1e-12, warm_start=ib.WS_PREV, gravity=-9.81, frame=True, c1=0.1, c2=0.1,
               mass_every=20)
    axis = nr * h
    X0 = W.axis_symmetric_shape(512, R, 0.01, 5, (axis, 0.5 * nz * h))
    runs = {}
    net = ib.Network((nr, nz), h)
    net.set_params(W.network_init(3))
    shape = (nz, nr)
    for mode in ("nn", "prev"):
        mg = ib.Multigrid(2, (nr, nz), h, precision=ib.MG_MIXED, krylov=0)
        solver = ib.Axisym(nr, nz, h, max_markers=512)
        X = X0.copy()
        u = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(2)]
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        pairs = []
        for k in range(train_steps):
            pp = p.clone()
            out = dict(p=torch.empty(shape, dtype=torch.float64, device="cuda"),
                       u=[torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(2)],
                       b=torch.empty(shape, dtype=torch.float64, device="cuda"),
                       H=torch.empty(shape, dtype=torch.float64, device="cuda"))
            out = solver.flow_step(mg, prm, u, X, p_prev=p, out=out)
            if mode == "nn" and k >= 2:
                pairs.append((out["b"], out["H"], pp, out["p"]))
            u, p = out["u"], out["p"]
        if mode == "nn":
            rng = np.random.default_rng(5)
            t0 = time.perf_counter()
            losses = []
            for it in range(train_iters):
                idx = rng.choice(len(pairs), size=4, replace=False)
                losses.append(net.train_step([pairs[i] for i in idx], prm["rho_in"], prm["rho_out"], 2e-3))
            torch.cuda.synchronize()
            runs["train"] = dict(pairs=len(pairs), iters=train_iters, seconds=round(time.perf_counter() - t0, 2),
                                 loss_first=float(np.mean(losses[:10])), loss_last=float(np.mean(losses[-50:])))
            del pairs
        cycles, accepted = [], []
        bufs = [dict(p=torch.empty(shape, dtype=torch.float64, device="cuda"),
                     u=[torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(2)]) for _ in range(2)]
        p_cur = p.clone()
        prm_run = dict(prm, warm_start=ib.WS_NN if mode == "nn" else ib.WS_PREV)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            o = solver.flow_step(mg, prm_run, u, X, p_prev=p_cur, out=bufs[k % 2],
                                 nn=net if mode == "nn" else None)
            u, p_cur = o["u"], o["p"]
            cycles.append(o["stats"]["cycles"])
            accepted.append(o["guess"]["accepted"])
            if k % 1000 == 999:
                log(f"  C5 {mode}: step {k + 1}/{steps}, cycles {np.mean(cycles[-1000:]):.2f}")
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        runs[mode] = dict(steps=steps, steps_per_s=round(steps / secs, 2), ms_per_step=round(1e3 * secs / steps, 3),
                          mean_vcycles=float(np.mean(cycles)),
                          guess_accepted=float(np.mean(accepted)) if mode == "nn" else None,
                          p_final=p_cur)
        mg.close()
        solver.close()
    net.close()
    d = (runs["nn"].pop("p_final") - runs["prev"]["p_final"]).norm().item() / runs["prev"]["p_final"].norm().item()
    runs["prev"].pop("p_final")
    runs["p_rel_l2_nn_vs_prev_after_run"] = d
    runs["workload"] = (f"axisymmetric free-falling water drop in air: {nr} x {nz} meridian half plane, h = 31.25 um, "
                        f"R = 1 mm, rho 1000/1.2, mu 1e-3/1.8e-5, sigma 0.072, g 9.81, 512 markers, seeded shape "
                        f"modes 2-6 <= 1%, dt = 1e-6 s; mixed-precision V(2,2) cycles; {train_steps} steps from p_prev to train "
                        f"the warm network, then {steps} steps with it vs from p_prev")
    return runs


def bench_free_fall(ib, torch):
    """Free-fall drops of Table afd_param sets 1 and 2 at h = 0.0125 on the meridian
    plane: steps/s of the full step with weight, frame and mass correction, and
    the slip Reynolds number's history (the paper plots it; no value is printed)."""
    res = {}
    for k in (1, 2):
        r = _free_fall_run(ib, torch, *AFD_SETS[k])
        res[f"set{k}"] = r
        log(f"  free fall set {k}: Re {r['reynolds_end']} (last-10% change {r['reynolds_change_last_10pct']}), "
            f"COM drift {r['com_drift_over_D']} D, {r['steps_per_s']} steps/s")
    res["workload"] = ("Table afd_param sets 1-2: D=1 drop, rho 10/1, mu 10 mu_a/mu_a, sigma=1, g from Eo, "
                       "mu_a from Mo; 128 x 256 meridian half plane at h=0.0125 (r <= 1.6 D, periodic "
                       "z of 3.2 D), dt 5e-4, 8000 steps (t = 4), 512 markers; weight (rho - rho_mean) g, "
                       "restoring frame c1 = c2 = 0.1, mass correction every 20 steps")
    return res


def bench_static_tables(ib, torch, reps=3):
    """Tables staticdrop_2d and staticdrop_axis of Section 5.1: a drop of diameter 0.4
    (2D: box centre; axisymmetric: on the axis), rho 1 / 0.01, sigma = 1, one projection
    step of 1e-3 from rest, at dx = 0.02 ... 0.00125. Box 1.28 (2D) and 0.64 x 1.28
    (meridian half plane), periodic; markers about 0.63 dx apart. Reports |dP - exact|
    beside the paper's new-scheme column and the step time."""
    from paper_1807_10504_amd import workloads as W
    dxs = [0.02, 0.01, 0.005, 0.0025, 0.00125]
    paper_2d = [1.1082e-3, 4.1935e-4, 5.5086e-4, 2.2961e-4, 1.2822e-4]
    paper_ax = [4.0890e-3, 1.3275e-3, 1.2220e-3, 4.8848e-4, 2.2793e-4]
    paper_2d_conv = [1.6475e-3, 1.4186e-3, 1.1080e-3, 1.0822e-3, 1.0744e-3]
    paper_ax_conv = [5.0019e-3, 8.8084e-4, 8.6586e-4, 1.8752e-3, 2.3319e-3]
    rows = []
    for dx, p2, pa, pc, pac in zip(dxs, paper_2d, paper_ax, paper_2d_conv, paper_ax_conv):
        nm = int(round(2 * np.pi * 0.2 / (0.63 * dx))) // 4 * 4
        prm = dict(rho_in=1.0, rho_out=0.01, sigma=1.0, dt=1e-3, rtol=1e-10, warm_start=ib.WS_ZERO)
        # 2D
        n = int(round(1.28 / dx))
        ctx = ib.Context(2, (n, n), dx, max_markers=nm)
        mg = ib.Multigrid(2, (n, n), dx, krylov=1)
        zero = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(2)]
        times = []
        for _ in range(reps):
            X = W.circle_markers(nm, 0.2, centre=(0.64, 0.64))
            out = {"H": torch.empty((n, n), dtype=torch.float64, device="cuda")}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = ctx.project_step(mg, prm, zero, X_host=X, out=out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        e2 = abs(ctx.diagnostics(p=out["p"], H=out["H"])["dP"] - 5.0)
        ms2 = 1e3 * min(times)
        # the conventional spreading (delta function), same drop
        X = W.circle_markers(nm, 0.2, centre=(0.64, 0.64))
        out = {"H": torch.empty((n, n), dtype=torch.float64, device="cuda")}
        out = ctx.project_step(mg, dict(prm, spread_mode=ib.IB_SPREAD_DELTA), zero, X_host=X, out=out)
        e2c = abs(ctx.diagnostics(p=out["p"], H=out["H"])["dP"] - 5.0)
        ctx.close()
        mg.close()
        # axisymmetric
        nr = int(round(0.64 / dx))
        ax = ib.Axisym(nr, 2 * nr, dx, max_markers=nm)
        mg = ib.Multigrid(2, (nr, 2 * nr), dx, krylov=1)
        zero = [torch.zeros((2 * nr, nr), dtype=torch.float64, device="cuda") for _ in range(2)]
        times = []
        for _ in range(reps):
            X = W.circle_markers(nm, 0.2, centre=(nr * dx, nr * dx))
            out = {"H": torch.empty((2 * nr, nr), dtype=torch.float64, device="cuda")}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = ax.project_step(mg, prm, zero, X, out=out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        hc = ib.Context(2, (nr, 2 * nr), dx, max_markers=16)
        ea = abs(hc.diagnostics(p=out["p"], H=out["H"])["dP"] - 10.0)
        msa = 1e3 * min(times)
        X = W.circle_markers(nm, 0.2, centre=(nr * dx, nr * dx))
        out = {"H": torch.empty((2 * nr, nr), dtype=torch.float64, device="cuda")}
        out = ax.project_step(mg, dict(prm, spread_mode=ib.IB_SPREAD_DELTA), zero, X, out=out)
        eac = abs(hc.diagnostics(p=out["p"], H=out["H"])["dP"] - 10.0)
        ax.close()
        mg.close()
        hc.close()
        rows.append(dict(dx=dx, markers=nm, err_2d=float(f"{e2:.4e}"), paper_new_2d=p2, ms_2d=round(ms2, 3),
                         err_2d_conventional=float(f"{e2c:.4e}"), paper_conventional_2d=pc,
                         err_axis=float(f"{ea:.4e}"), paper_new_axis=pa, ms_axis=round(msa, 3),
                         err_axis_conventional=float(f"{eac:.4e}"), paper_conventional_axis=pac))
        log(f"  dx {dx}: 2D |dP-5| {e2:.3e} (paper {p2}; conventional {e2c:.3e}, paper {pc}), "
            f"axis |dP-10| {ea:.3e} (paper {pa}; conventional {eac:.3e}, paper {pac})")
    return dict(workload="Tables staticdrop_2d / staticdrop_axis: D = 0.4, rho 1/0.01, sigma 1, one step "
                         "of 1e-3 from rest; 2D box 1.28, axisymmetric half plane 0.64 x 1.28, periodic; "
                         "flexible-CG projection to 1e-10", rows=rows)


def bench_predictor_3d(ib, torch, nc=256, calls=5):
    """The momentum predictor alone at nc^3 (FP64): a smooth drop of radius 0.3 with
    densities 1/1e-3 and viscosities 1e-2/1e-4, seeded velocities of size 0.1,
    dt = 5e-5, Adams-Bashforth history present, system solved to 1e-12."""
    shape = (nc, nc, nc)
    h = 1.0 / nc
    z = (np.arange(nc) + 0.5) * h - 0.5
    r = np.sqrt(z[:, None, None] ** 2 + z[None, :, None] ** 2 + z[None, None, :] ** 2)
    H = torch.from_numpy(np.clip((0.3 - r) / (3 * h) + 0.5, 0.0, 1.0)).cuda()
    rho = 1e-3 + (1.0 - 1e-3) * H
    mu = 1e-4 + (1e-2 - 1e-4) * H
    g = torch.Generator(device="cpu").manual_seed(7)
    u = [(0.1 * torch.randn(shape, generator=g, dtype=torch.float64)).cuda() for _ in range(3)]
    us = [torch.empty_like(a) for a in u]
    fl = ib.Flow(3, (nc, nc, nc), h)
    fl.predict(u, rho, rho, mu, 5e-5, rtol=1e-12, u_star=us)      # fills the history
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sw, ck = [], []
    for _ in range(calls):
        _, st = fl.predict(u, rho, rho, mu, 5e-5, rtol=1e-12, u_star=us)
        sw.append(st["sweeps"])
        ck.append(st["checks"])
    torch.cuda.synchronize()
    secs = (time.perf_counter() - t0) / calls
    N = float(nc) ** 3
    s, c = float(np.mean(sw)), float(np.mean(ck))
    # copy u -> u* 48 B, right side 120 B, per sweep 88 B (x read and written, g, rho and mu read
    # once: what any full sweep must move), per residual check 64 B
    algo = (48 + 120 + s * 88 + c * 64) * N
    fl.close()
    return dict(workload=f"predictor_3d_{nc}: smooth drop, rho 1/1e-3, mu 1e-2/1e-4, dt 5e-5, rtol 1e-12",
                ms_per_call=round(1e3 * secs, 3), sweeps=s, residual_checks=c,
                algorithmic_bytes=algo, achieved_GBs=round(algo / secs / 1e9, 1),
                frac_hbm=round(algo / secs / 1e9 / HBM_PEAK_GBS, 4))


def bench_2d_c4_nn(ib, torch, n=512, trajectories=20, steps=100, train_iters=1500, evals=20):
    """Learned warm start on the oscillating-drop configuration: seeded
    trajectories of projection-only dynamics (u* = u^n) from r = R(1 + 0.1 cos 2theta
    + seeded modes 3..6 of amplitude <= 0.02), the pairs (b, 1/rho, p_prev -> p)
    the multigrid generates along them, the last trajectory held out. Two networks:
    cold (from b and 1/rho alone) and warm (with p_prev). Reported: V-cycles from
    the guesses against zero and against p_prev on held-out steps, the solve time
    with inference, and the converged pressure's error against the oracle's
    tightly converged solve of the same step."""
    from oracle import poisson
    from paper_1807_10504_amd import workloads as W
    h = 1.0 / n
    shape = (n, n)
    ctx = ib.Context(2, (n, n), h, max_markers=1024)
    mg = ib.Multigrid(2, (n, n), h)
    prm = dict(rho_in=1.0, rho_out=1e-3, sigma=1.0, dt=2e-5, rtol=1e-10, warm_start=ib.WS_PREV)
    trajs = []
    t0 = time.perf_counter()
    for tr in range(trajectories):
        X = W.mode_shape(1024, 0.2, 0.1, seed=100 + tr, extra_amp=0.02)
        u = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(2)]
        p_prev, pairs = None, []
        for s_ in range(steps):
            o = dict(b=torch.empty(shape, dtype=torch.float64, device="cuda"),
                     H=torch.empty(shape, dtype=torch.float64, device="cuda"))
            pp = p_prev.clone() if p_prev is not None else torch.zeros(shape, dtype=torch.float64, device="cuda")
            o = ctx.project_step(mg, prm, u, p_prev=p_prev, X_host=X, out=o)
            if s_ >= 2:
                pairs.append((o["b"], o["H"], pp, o["p"].clone()))
            u, p_prev = o["u"], o["p"]
        trajs.append(pairs)
        if (tr + 1) % 5 == 0:
            log(f"  trajectory {tr + 1}/{trajectories}")
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    train = [smp for tr in trajs[:-1] for smp in tr]
    held = trajs[-1]
    out = dict(workload=f"oscillating drop 2D {n}^2, r=R(1+0.1cos2theta+seeded modes 3-6 <=0.02), R=0.2, 1024 "
                        f"markers, rho ratio 1000, dt=2e-5; {trajectories} seeded trajectories x {steps} "
                        f"projection steps -> {len(train)} training pairs, the last trajectory "
                        f"({len(held)} steps) held out",
               pairs=len(train), pairs_s=round(t_pairs, 2))
    nets = {}
    for kind in ("cold", "warm"):
        net = ib.Network((n, n), h)
        net.set_params(W.network_init(1 if kind == "cold" else 2))
        rng = np.random.default_rng(1)
        t0 = time.perf_counter()
        losses = []
        for it in range(train_iters):
            idx = rng.choice(len(train), size=4, replace=False)
            batch = [(train[i][0], train[i][1], None if kind == "cold" else train[i][2], train[i][3]) for i in idx]
            losses.append(net.train_step(batch, 1.0, 1e-3, 2e-3))
        torch.cuda.synchronize()
        out[f"{kind}_train_s"] = round(time.perf_counter() - t0, 2)
        out[f"{kind}_loss_first"] = float(np.mean(losses[:10]))
        out[f"{kind}_loss_last"] = float(np.mean(losses[-50:]))
        nets[kind] = net
    sel = np.linspace(0, len(held) - 1, evals).astype(int)
    res = {k: [] for k in ("zero", "cold_nn", "prev", "warm_nn")}
    t = {k: 0.0 for k in res}
    finals = []
    for i in sel:
        b, H, pp, p = held[i]
        mg.update_coeffs(ctx.coefficients(H, 1.0, 1e-3))
        for key, start in (("zero", None), ("cold_nn", "cold"), ("prev", pp), ("warm_nn", "warm")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if key == "zero":
                x = torch.zeros_like(p)
            elif key == "prev":
                x = pp.clone()
            else:
                x = nets[start].predict(b, H, None if start == "cold" else pp, 1.0, 1e-3)
            st = mg.solve(b, x, rtol=1e-10)
            torch.cuda.synchronize()
            t[key] += time.perf_counter() - t0
            res[key].append(st["cycles"])
            if key == "cold_nn" and len(finals) < 3:
                finals.append((b.cpu().numpy(), H.cpu().numpy(), x.cpu().numpy()))
    for k in res:
        out[f"cycles_{k}"] = float(np.mean(res[k]))
        out[f"solve_ms_{k}"] = round(1e3 * t[k] / len(sel), 3)
    # the converged answer from the learned start against the oracle
    errs = []
    for (b, H, x) in finals:
        beta = poisson.face_beta(poisson.density(H, 1.0, 1e-3))
        po, _, _ = poisson.mg_pcg(b, beta, h, rtol=1e-13, max_iter=100)
        errs.append(float(np.linalg.norm(x - po) / np.linalg.norm(po)))
    out["cold_nn_p_rel_l2_vs_oracle_tight"] = max(errs)
    for net in nets.values():
        net.close()
    mg.close()
    ctx.close()
    return out


def cpu_baseline(wl, cycles_per_step, krylov):
    """The oracle on a bounded sample of the same 256^3 step, extrapolated to one step."""
    from oracle import heaviside, poisson
    n, h = wl.n, wl.h
    shape = tuple(reversed(n))
    rng = np.random.default_rng(1)
    t = {}
    # multigrid: one FP64 V-cycle at full size
    H = np.zeros(shape)
    g = np.indices(shape, sparse=True)
    r2 = sum(((g[a] + 0.5) * h - 0.5) ** 2 for a in range(3))
    H[r2 < 0.25 ** 2] = 1.0
    beta = poisson.face_beta(poisson.density(H, wl.rho_in, wl.rho_out))
    b = rng.standard_normal(shape)
    b -= b.mean()
    t0 = time.perf_counter()
    hier = poisson.Hierarchy(beta, h)
    t["setup"] = time.perf_counter() - t0
    p = np.zeros(shape)
    t0 = time.perf_counter()
    p = poisson.vcycle(hier, 0, p, b)
    t["vcycle"] = time.perf_counter() - t0
    if krylov:
        # the rest of one flexible-CG iteration of the oracle: q = A d, the
        # three inner products and the three vector updates
        d, r = p.copy(), b.copy()
        t0 = time.perf_counter()
        q = poisson.apply_A(d, beta, h)
        alpha = np.vdot(r, p) / np.vdot(d, q)
        p += alpha * d
        r -= alpha * q
        np.linalg.norm(r)
        bq = np.vdot(q, p)
        np.vdot(r, p)
        d = p + bq * d
        t["cg_vectors"] = time.perf_counter() - t0
        t["vcycle"] += t["cg_vectors"]
    # coefficients, right side, update at full size
    F = [np.zeros(shape) for _ in range(3)]
    u = [np.zeros(shape) for _ in range(3)]
    t0 = time.perf_counter()
    beta = poisson.face_beta(poisson.density(H, wl.rho_in, wl.rho_out))
    b = poisson.rhs(u, F, beta, wl.dt, h)
    poisson.velocity_update(u, F, beta, p, wl.dt, h)
    t["grid_ops"] = time.perf_counter() - t0
    # Heaviside on a sample of columns, scaled by the number of columns the
    # surface projects onto
    V, T = wl.X, wl.tris
    nrm = heaviside.vertex_normals(V, T)  # static surface: computed once, not timed
    cols = []
    for k in range(24):
        i = int(rng.integers(int(0.25 / h) + 2, int(0.75 / h) - 2))
        j = int(rng.integers(int(0.25 / h) + 2, int(0.75 / h) - 2))
        cols.append((i, j))
    t0 = time.perf_counter()
    heaviside.heaviside_3d(V, T, n, h, nrm=nrm, columns=cols)
    tH = time.perf_counter() - t0
    ncols = math.pi * (0.25 + 2 * h) ** 2 / h ** 2
    t["heaviside"] = tH / len(cols) * ncols
    # face force: nearest-element search for sampled faces next to the surface,
    # scaled by the faces of a shell of +-2.9h (where H differences live)
    from oracle import force, surface3d
    fs_o = surface3d.surface_geometry(V, T, wl.sigma)[0]
    dirs = rng.standard_normal((40, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = 0.5 + (0.25 + rng.uniform(-2.5, 2.5, size=(40, 1)) * h) * dirs
    t0 = time.perf_counter()
    for q in pts:
        force.nearest_on_mesh(q, V, T, fs_o)
    tF = time.perf_counter() - t0
    nfaces = 3 * 4 * math.pi * 0.25 ** 2 * 5.8 * h / h ** 3
    t["face_force"] = tF / len(pts) * nfaces
    per_step = t["grid_ops"] + t["heaviside"] + t["face_force"] + cycles_per_step * t["vcycle"]
    what = "flexible-CG iteration (V-cycle + vector work)" if krylov else "V-cycle"
    sample = (f"256^3 oracle: one FP64 {what} ({t['vcycle']:.1f} s) x {cycles_per_step:.1f} per step, "
              f"coefficients+rhs+update ({t['grid_ops']:.1f} s), Heaviside on {len(cols)} columns scaled to "
              f"{ncols:.0f} columns ({t['heaviside']:.0f} s), nearest-element face value on 40 faces scaled "
              f"to {nfaces:.0f} band faces ({t['face_force']:.0f} s)")
    # NumPy's element-wise work runs on one thread: the oracle used one core
    return dict(value=1.0 / per_step, unit="steps/s", cores=1, host_cpu_count=os.cpu_count(),
                kind="oracle", sample=sample, seconds_per_step=per_step,
                breakdown={k: round(v, 2) for k, v in t.items()})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--level", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solver", choices=("fcg", "vcycle"), default="fcg",
                    help="headline FP64 solver: flexible CG preconditioned by V(2,2), or V(2,2) cycles")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D workloads (C2, learned warm start)")
    ap.add_argument("--no-nn3d", action="store_true", help="skip the 3D learned warm start")
    ap.add_argument("--nn3d-iters", type=int, default=60, help="training iterations of the 3D network")
    ap.add_argument("--c5-steps", type=int, default=2000,
                    help="steps of the axisymmetric free-fall run with and without the learned warm start")
    ap.add_argument("--c4-steps", type=int, default=100,
                    help="projection steps per oscillating-drop trajectory (20 trajectories) for the 2D network")
    ap.add_argument("--no-flow", action="store_true",
                    help="skip the full 2D flow steps and the 3D momentum predictor")
    ap.add_argument("--section", default=None,
                    choices=("flow_osc", "static_tables", "conventional", "osc_energy", "flow3d", "free_fall",
                             "predictor_3d", "c5", "c4"),
                    help="run only this section of the flow measurements and print its JSON (for profiling)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MB (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1807_10504_amd import ibproj as ib
    from paper_1807_10504_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    ib.load()
    if args.section:
        run = {"flow_osc": bench_flow_osc, "static_tables": bench_static_tables, "conventional": bench_conventional,
               "osc_energy": bench_osc_energy, "flow3d": bench_flow3d, "free_fall": bench_free_fall,
               "predictor_3d": lambda ib_, t_: bench_predictor_3d(ib_, t_, args.size),
               "c5": lambda ib_, t_: bench_c5(ib_, t_, steps=args.c5_steps),
               "c4": lambda ib_, t_: bench_2d_c4_nn(ib_, t_, steps=args.c4_steps)}[args.section]
        print(json.dumps({args.section: run(ib, torch)}), flush=True)
        return
    wl = W.static_drop_3d(args.size, args.level, seed=3)
    log(f"workload {wl.name}: {len(wl.X)} markers, {len(wl.tris)} triangles")
    geo = ib.surface_geometry_3d(wl.X, wl.tris, wl.sigma)
    if args.copy_mb:
        # an elementwise kernel (not a DMA blit): reads 8 B and writes 8 B per element
        a = torch.ones(args.copy_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=c)
        torch.cuda.synchronize()
        del a, c

    def summary(r, ref=None):
        sps = r["steps"] / r["seconds"]
        out = dict(steps_per_s=round(sps, 3), ms_per_step=round(1e3 * r["seconds"] / r["steps"], 3),
                   mean_cycles=float(np.mean(r["cycles"])), max_rel_res=float(np.max(r["rel_res"])),
                   dP=r["dP"])
        if ref is not None:
            out["speedup_vs_fp64_cold"] = round(sps / ref, 3)
        return out

    # the headline solver: FP64 flexible CG preconditioned by one V(2,2) cycle
    # (--solver vcycle: plain V(2,2) cycles); the other one is reported beside it
    head_k = 1 if args.solver == "fcg" else 0
    names = {1: "fcg", 0: "vcycle"}
    log(f"== FP64 {names[head_k]}, cold start every step (headline)")
    r64 = run_variant(ib, torch, wl, geo, ib.MG_FP64, args.steps, args.warmup, profile=True,
                      krylov=head_k)
    sps64 = r64["steps"] / r64["seconds"]
    variants = {f"fp64_cold_{names[head_k]}": summary(r64)}
    log(f"== FP64 {names[1 - head_k]}, cold start every step")
    ro = run_variant(ib, torch, wl, geo, ib.MG_FP64, args.steps, args.warmup, profile=False,
                     krylov=1 - head_k)
    variants[f"fp64_cold_{names[1 - head_k]}"] = summary(ro, sps64)
    if not args.no_mixed:
        for kry in (head_k, 1 - head_k):
            log(f"== mixed FP32/FP64 {names[kry]}, cold start every step")
            rmx = run_variant(ib, torch, wl, geo, ib.MG_MIXED, args.steps, args.warmup,
                              profile=kry == head_k, krylov=kry)
            variants[f"mixed_cold_{names[kry]}"] = summary(rmx, sps64)
            if kry == head_k:
                variants[f"mixed_cold_{names[kry]}"]["kernels"] = {
                    k: dict(launches=v[0], avg_us=round(1e3 * v[1] / v[0], 2))
                    for k, v in rmx["prof"].items() if v[0]}
    log("== error of each solver's p against a tightly converged FP64 solve")
    variants["p_error_vs_fp64_tight"] = precision_errors(ib, torch, wl, geo)
    if not args.no_warm:
        log(f"== FP64 {names[head_k]}, warm start from the previous pressure")
        rw = run_variant(ib, torch, wl, geo, ib.MG_FP64, args.steps, args.warmup, profile=False,
                         warm=True, krylov=head_k)
        variants[f"fp64_warm_{names[head_k]}"] = summary(rw, sps64)
    # roofline of the dominant kernel: the finest-level FP64 smoother, either
    # one full single-pass sweep or one colour pass (half a sweep)
    N = float(np.prod(wl.n))
    min_bytes = None
    if r64["prof"]["sweep64_rho"][0]:
        nl, ms = r64["prof"]["sweep64_rho"]
        bytes_per_launch = SWEEP_BYTES_F64 * N
        min_bytes = SWEEP_BYTES_F64_RHO * N
        kname = "k_rbgs_fused_rho<32,16,512>"
    elif r64["prof"]["sweep64"][0]:
        nl, ms = r64["prof"]["sweep64"]
        bytes_per_launch = SWEEP_BYTES_F64 * N
        kname = "k_rbgs_fused<double>"
    else:
        nl, ms = r64["prof"]["smooth64"]
        bytes_per_launch = 0.5 * SWEEP_BYTES_F64 * N
        kname = "k_rbgs<double,3>"
    avg_s = ms / 1e3 / max(nl, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    prof_summary = {k: dict(launches=v[0], avg_us=round(1e3 * v[1] / v[0], 2))
                    for k, v in r64["prof"].items() if v[0]}
    traffic, source = TRAFFIC.get(kname, (None, None))
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=kname + " (finest-level single-pass red-black sweep)",
                bytes_per_launch=bytes_per_launch, bytes_per_cell=bytes_per_launch / N,
                avg_launch_us=round(avg_s * 1e6, 2), traffic_source=source)
    if min_bytes is not None:
        # the same launch time against the bytes this kernel must move (p, b, rho
        # read, p written) and against the bytes the counters saw
        roof["frac_min_bytes"] = round(min_bytes / avg_s / 1e9 / HBM_PEAK_GBS, 4)
        roof["min_bytes_per_cell"] = SWEEP_BYTES_F64_RHO
    if traffic is not None:
        roof["frac_counters"] = round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
    # all four forms of the finest density sweep together (per step: plain, with
    # the prolongation folded in, zero-start, with the CG inner products), each
    # against the bytes its form must move (the first iteration's inner-product
    # sweep reads no q: one launch in twelve counted 8 bytes per cell high)
    forms = {"sweep64_rho": SWEEP_BYTES_F64_RHO, "sweep_pro": SWEEP_BYTES_F64_RHO + 1.0,
             "sweep_zero": SWEEP_BYTES_F64_RHO - 8.0, "sweep_dots": SWEEP_BYTES_F64_RHO + 8.0}
    if all(r64["prof"].get(k, (0, 0))[0] for k in forms):
        tb = sum(r64["prof"][k][0] * b * N for k, b in forms.items())
        tt = sum(r64["prof"][k][1] for k in forms) / 1e3
        roof["all_sweep_forms"] = dict(launches=sum(r64["prof"][k][0] for k in forms),
                                       ms=round(1e3 * tt, 2), bytes=tb,
                                       frac_min_bytes=round(tb / tt / 1e9 / HBM_PEAK_GBS, 4),
                                       min_bytes_per_cell=forms)
    line = dict(metric=METRIC, value=round(sps64, 3), unit="steps/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(1e3 * r64["seconds"] / r64["steps"], 3),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
                data="synthetic",
                config=dict(workload=f"static_drop_3d_{args.size}: {args.size}^3 periodic box, sphere R=0.25 "
                                     f"(level-{args.level} icosphere, {len(wl.X)} markers, {len(wl.tris)} "
                                     f"triangles, seeded rotation 3), rho ratio 1000, sigma=1, dt=5e-5, "
                                     f"irrotational spreading, FP64 pressure solve from p=0 to 1e-10 every step by "
                                     + ("flexible CG preconditioned by one V(2,2) cycle" if head_k else
                                        "V(2,2) multigrid cycles"),
                            grid=list(wl.n), markers=len(wl.X), triangles=len(wl.tris)),
                variants=variants, roofline=roof, kernels_fp64=prof_summary)
    if not args.no_nn3d:
        log(f"== 3D learned warm start at {args.size}^3")
        line["nn_3d"] = bench_3d_nn(ib, torch, wl, geo, args.steps, args.warmup, sps64,
                                    train_iters=args.nn3d_iters)
    if not args.no_2d:
        log("== 2D 512^2 jittered drop: FP64 vs mixed, 200 steps")
        line["c2_2d"] = bench_2d_c2(ib, torch)
        log("== 2D 512^2 learned warm start (oscillating-drop trajectories)")
        line["nn_2d"] = bench_2d_c4_nn(ib, torch, steps=args.c4_steps)
    if not args.no_flow:
        log("== full flow steps: Table osc oscillating drops (2D and axisymmetric)")
        line["flow_osc"] = bench_flow_osc(ib, torch)
        log("== static drop tables (2D and axisymmetric)")
        line["static_tables"] = bench_static_tables(ib, torch)
        log("== conventional delta vector: curl versus h, indicator function")
        line["conventional"] = bench_conventional(ib, torch)
        log("== oscillating drop energy (new vs conventional) and large deformation")
        line["osc_energy"] = bench_osc_energy(ib, torch)
        log("== moving 3D drops (local least-squares surface)")
        line["flow3d"] = bench_flow3d(ib, torch)
        log("== free-fall drops (Table afd_param sets 1-2, axisymmetric)")
        line["free_fall"] = bench_free_fall(ib, torch)
        log("== axisymmetric free-falling water drop, 256 x 1024, mixed precision + learned warm start")
        line["c5_free_fall_nn"] = bench_c5(ib, torch, steps=args.c5_steps)
        log(f"== momentum predictor at {args.size}^3")
        line["predictor_3d"] = bench_predictor_3d(ib, torch, args.size)
    if not args.no_cpu_baseline:
        log("== CPU oracle baseline (bounded sample)")
        line["cpu_baseline"] = cpu_baseline(wl, variants[f"fp64_cold_{names[head_k]}"]["mean_cycles"],
                                            head_k)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
