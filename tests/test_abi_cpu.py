"""The C ABI library without a GPU: it loads, exports every declared entry
point, rejects bad arguments before touching the device, and its host FP64
geometry (B-spline relocation, sphere-mesh curvature) matches the oracle --
bit for bit for the relocation, to rounding for the mesh geometry."""
import os
import re

import numpy as np
import pytest

from oracle import bspline, surface3d
from paper_1807_10504_amd import ibproj
from paper_1807_10504_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ibproj.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b([a-z_0-9]+)\s*\(", txt))
    return {n for n in names if n.startswith(("ib_", "mg_", "project_", "flow_", "axi_"))}


def test_library_exports_every_declared_symbol():
    lib = ibproj.load()
    decl = _declared()
    assert len(decl) >= 17
    for name in decl:
        assert hasattr(lib, name), name
    assert set(ibproj.EXPORTS) == decl


def test_library_shares_torch_hip_runtime():
    """Loaded through the binding, the library binds to the HIP runtime torch
    brings: one runtime is mapped in a fresh process (loaded before torch, the
    library would pull in a second runtime, and its allocations fail)."""
    import subprocess
    import sys
    code = ("from paper_1807_10504_amd import ibproj; ibproj.load(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_invalid_arguments_rejected_without_device():
    import ctypes as C
    lib = ibproj.load()
    g = ibproj.make_grid(5, (16, 16, 16), 1 / 16)
    out = C.c_void_p()
    assert lib.ib_create(C.byref(g), 100, 0, C.byref(out)) == ibproj.IB_EINVAL
    assert b"dim" in lib.ib_last_error()
    g = ibproj.make_grid(2, (24, 20, 1), 1 / 16)
    o = ibproj.MgOpts(0, 2, 2, 4)
    assert lib.mg_setup(C.byref(g), C.byref(o), C.byref(out)) == ibproj.IB_EINVAL
    g = ibproj.make_grid(2, (64, 64, 1), 1 / 64)
    o = ibproj.MgOpts(7, 2, 2, 4)
    assert lib.mg_setup(C.byref(g), C.byref(o), C.byref(out)) == ibproj.IB_EINVAL


def test_noalloc_residual_norm_rejects_oversized_grid():
    """The allocation-free norm refuses grids beyond its 2^31 - 1 cells before
    any device work (the pointers are never dereferenced)."""
    import ctypes as C
    lib = ibproj.load()
    g = ibproj.make_grid(3, (2048, 2048, 1024), 1 / 2048)
    fake = C.c_void_p(4096)
    rc = lib.mg_residual_norm_noalloc(C.byref(g), fake, fake, fake, fake, None)
    assert rc == ibproj.IB_EINVAL
    assert b"maximum" in lib.ib_last_error()
    g = ibproj.make_grid(4, (16, 16, 16), 1 / 16)
    assert lib.mg_residual_norm_noalloc(C.byref(g), fake, fake, fake, fake, None) == ibproj.IB_EINVAL


@pytest.mark.parametrize("case", ["c1_static", "c1_moving", "c2_jitter", "interpol_cir", "mode2"])
def test_bspline_relocation_bit_exact(case):
    if case == "c1_static":
        X, h, dt = W.circle_markers(128, 0.25), 1 / 64, 1e-4
        U = np.zeros_like(X)
    elif case == "c1_moving":
        X, h, dt = W.circle_markers(128, 0.25), 1 / 64, 1e-3
        U = np.random.default_rng(5).standard_normal(X.shape) * 0.3
    elif case == "c2_jitter":
        X, h, dt = W.jittered_circle(1024, 0.2, 1e-3, seed=2), 1 / 512, 2e-5
        U = np.zeros_like(X)
    elif case == "interpol_cir":
        X, h, dt = W.perturbed_circle(126, 1e-3), 1 / 32, 0.0
        U = np.zeros_like(X)
    else:
        X, h, dt = W.mode_shape(256, 0.2, 0.1), 1 / 128, 1e-4
        U = np.random.default_rng(7).standard_normal(X.shape)
    Xo, fs, ds, nrm = ibproj.relocate_bspline(X, U, dt, h, 1.0)
    Xr, fr, dr, nr = bspline.relocate([tuple(x) for x in X], [tuple(u) for u in U], dt, h, 1.0)
    assert np.array_equal(Xo, np.array(Xr))
    assert np.array_equal(fs, np.array(fr))
    assert np.array_equal(ds, np.array(dr))
    assert np.array_equal(nrm, np.array(nr))


def test_bspline_relocation_reports_schoenberg_whitney():
    X = W.circle_markers(20, 0.3)
    with pytest.raises(ibproj.IbError) as e:
        ibproj.relocate_bspline(X, np.zeros_like(X), 0.0, 1 / 256, 1.0)
    assert e.value.code == ibproj.IB_EGEOM


@pytest.mark.parametrize("level", [2, 4])
def test_surface_geometry_3d_matches_oracle(level):
    V, T = W.sphere_mesh(level, 0.25, seed=3)
    fs, ds, nrm = ibproj.surface_geometry_3d(V, T, 1.0)
    fo, Ao, no, _ = surface3d.surface_geometry(V, T, 1.0)
    assert np.max(np.abs(fs - fo)) <= 1e-12 * np.max(np.abs(fo))
    assert np.max(np.abs(ds - Ao)) <= 1e-14 * np.max(Ao)
    assert np.max(np.abs(nrm - no)) <= 1e-13


@pytest.mark.parametrize("axis", [None, 0.5])
def test_enclosed_measure_matches_oracle(axis):
    from oracle import dynamics
    for X in (W.circle_markers(256, 0.25), W.mode_shape(256, 0.2, 0.1), W.ellipse_markers(200, 0.2, 1.1)):
        v, c = ibproj.enclosed_measure(X, axis)
        vo, co = dynamics.measure(X, axis)
        assert abs(v - vo) <= 1e-13 * abs(vo) and abs(c - co) <= 1e-13
    with pytest.raises(ibproj.IbError) as e:
        ibproj.enclosed_measure(np.zeros((2, 2)), axis)
    assert e.value.code == ibproj.IB_EINVAL


@pytest.mark.parametrize("axis", [None, 0.5])
def test_mass_correction_matches_oracle(axis):
    """The relocation's normals point into the drop, so a shrunk drop takes a
    negative displacement; the host correction agrees with the oracle's."""
    from oracle import dynamics
    X0 = W.circle_markers(256, 0.25)
    h = 1 / 64
    _, _, _, nrm = ibproj.relocate_bspline(X0, np.zeros_like(X0), 0.0, h, 1.0)
    assert np.all(np.sum(nrm * (np.array([0.5, 0.5]) - X0), axis=1) > 0)
    target, _ = dynamics.measure(X0, axis)
    for s in (2e-4, -1e-4):
        X = X0 + s * nrm
        Xc, d = ibproj.mass_correct(X, nrm, target, axis, h)
        Xo, do = dynamics.mass_correct(X, nrm, target, axis, h)
        assert abs(dynamics.measure(Xc, axis)[0] - target) <= 2e-12 * target
        assert abs(d - do) <= 1e-11 and abs(d + s) <= 1e-9
        assert np.max(np.abs(Xc - Xo)) <= 1e-11
    Xc, d = ibproj.mass_correct(X0 + 1e-10 * nrm, nrm, target, axis, h)
    assert d == 0.0
    with pytest.raises(ibproj.IbError):
        ibproj.mass_correct(X0, nrm, -1.0, axis, h)


def test_markers_add_delete_bit_exact():
    from oracle import markers
    h = 1 / 64
    cases = [W.circle_markers(n, 0.25) for n in (60, 100, 300, 700)]
    cases.append(W.jittered_circle(400, 0.25, 0.02, seed=4))
    rng = np.random.default_rng(9)
    th = np.sort(rng.uniform(0, 2 * np.pi, 250))
    cases.append(np.stack([0.5 + 0.3 * np.cos(th), 0.5 + 0.2 * np.sin(th)], axis=1))
    for X in cases:
        Y = ibproj.markers_add_delete(X, h)
        assert np.array_equal(Y, markers.add_delete(X, h))
    with pytest.raises(ibproj.IbError):
        ibproj.markers_add_delete(np.zeros((2, 2)), h)


@pytest.mark.parametrize("level", [2, 3])
def test_surface_lsq_3d_matches_oracle(level):
    V, T = W.sphere_mesh(level, 0.25, seed=3)
    rng = np.random.default_rng(level)
    V = V + 1e-3 * rng.uniform(-1, 1, V.shape)            # not on a sphere
    Vo, fs, ds, nrm = ibproj.surface_lsq_3d(V, T, 1.0)
    Vr, fr, dr, nr = surface3d.lsq_reconstruct(V, T, 1.0)
    assert np.abs(Vo - Vr).max() <= 1e-14
    assert np.abs(fs - fr).max() <= 1e-11 * np.abs(fr).max()
    assert np.abs(ds - dr).max() <= 1e-15 * dr.max() * 10
    assert np.abs(nrm - nr).max() <= 1e-12
    with pytest.raises(ibproj.IbError):
        ibproj.surface_lsq_3d(V, np.where(T == 0, len(V), T), 1.0)


def test_surface_lsq_3d_degenerate_neighbourhood():
    # a tetrahedron: every two-ring holds 4 vertices, too few for the quadric
    V = np.array([[0.5, 0.5, 0.7], [0.6, 0.45, 0.4], [0.4, 0.45, 0.4], [0.5, 0.62, 0.4]])
    T = np.array([[0, 1, 3], [0, 3, 2], [0, 2, 1], [1, 2, 3]], dtype=np.int32)
    with pytest.raises(ibproj.IbError) as e:
        ibproj.surface_lsq_3d(V, T, 1.0)
    assert e.value.code == ibproj.IB_EGEOM


def test_mesh_measure_and_correction_match_oracle():
    from oracle import dynamics, surface3d as s3
    V, T = W.sphere_mesh(3, 0.25, seed=3)
    V = 0.5 + (V - 0.5) * np.array([1.1, 0.95, 1.0])
    v, c = ibproj.mesh_measure(V, T)
    vo, co = dynamics.measure(V, T=T)
    assert abs(v - vo) <= 1e-13 * vo and abs(c - co) <= 1e-13
    nrm = s3.vertex_normals(V, T)
    for sft in (2e-4, -1e-4):
        Vc, d = ibproj.mesh_mass_correct(V + sft * nrm, nrm, T, vo, 1 / 64)
        Vr, dr = dynamics.mass_correct(V + sft * nrm, nrm, vo, None, 1 / 64, T=T)
        assert abs(d - dr) <= 1e-11 and np.abs(Vc - Vr).max() <= 1e-11
        assert abs(dynamics.measure(Vc, T=T)[0] - vo) <= 2e-12 * vo
    with pytest.raises(ibproj.IbError):
        ibproj.mesh_measure(V, np.where(T == 0, len(V), T))
