"""Multigrid from cell densities (mg_update_density) against the stored-face
hierarchy (mg_update_coeffs) and against the oracle.

* ib_density: rho bitwise the oracle's rho_out + (rho_in - rho_out) H (NumPy
  rounds the multiply and the add separately, as the library does), and
  2 / (rho_c + rho_{c-e_d}) bitwise the faces of ib_coefficients;
* equal fixed cycles: p of the density path against the stored-face path,
  bitwise on grids where the faces are formed into the handle (2D; 32^3; FP64
  and 2D mixed) and to 1e-13 where the kernels read rho directly (128^3;
  256 x 128 x 128: the sweep updates cells away from the interface without a
  division); the residual history to 1e-13 (the tiled density kernels sum
  their norms per tile);
* mixed precision where the kernels read rho directly: the float32 cycle
  forms its finest coefficients in float32 from float32 densities, against
  the oracle's mixed solver given the densities (and the stored-face path
  against it without them), 1e-8 after three cycles;
* the density path against the oracle's multigrid at equal cycles (1e-11).
"""
import numpy as np
import pytest

from oracle import poisson
from paper_1807_10504_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _drop_H(shape, seed):
    """A smooth drop (radius 0.3, 3-cell ramp) with seeded noise in the ramp."""
    g = np.indices(shape)
    r = np.sqrt(sum(((g[a] + 0.5) / shape[a] - 0.5) ** 2 for a in range(len(shape))))
    h = 1.0 / max(shape)
    H = np.clip((0.3 - r) / (3 * h) + 0.5, 0.0, 1.0)
    ramp = (H > 0) & (H < 1)
    H[ramp] += 0.01 * np.random.default_rng(seed).standard_normal(ramp.sum())
    return np.clip(H, 0.0, 1.0)


@pytest.mark.parametrize("shape", [(48, 64), (16, 16, 32)])
def test_density_bitwise(ib, shape):
    dim = len(shape)
    n = tuple(reversed(shape))
    H = _drop_H(shape, 1)
    ctx = ib.Context(dim, n, 1.0 / n[0], max_markers=16)
    rho = host(ctx.density(dev(H), 1.0, 1e-3))
    assert np.array_equal(rho, poisson.density(H, 1.0, 1e-3))
    beta = [host(x) for x in ctx.coefficients(dev(H), 1.0, 1e-3)]
    for d, bo in enumerate(poisson.face_beta(rho)):
        assert np.array_equal(beta[d], bo)


CASES = [
    ((64, 64), 4, "fp64"),
    ((32, 32, 32), 4, "fp64"),
    ((128, 128, 128), 4, "fp64"),
    ((128, 128, 256), 2, "fp64"),
    ((64, 64), 4, "mixed"),
]


@pytest.mark.parametrize("shape,nc,prec", CASES)
def test_density_path_bitwise_vs_faces(ib, shape, nc, prec):
    dim = len(shape)
    n = tuple(reversed(shape))
    h = 1.0 / max(shape)
    H = dev(_drop_H(shape, 2))
    b = W.random_cells(n, dim, 1.0, seed=61)
    b = dev(b - b.mean())
    ctx = ib.Context(dim, n, h, max_markers=16)
    rho = ctx.density(H, 1.0, 1e-3)
    beta = ctx.coefficients(H, 1.0, 1e-3)
    precision = ib.MG_MIXED if prec == "mixed" else ib.MG_FP64
    out = []
    for mode in ("faces", "density"):
        mg = ib.Multigrid(dim, n, h, precision=precision, n_coarsest=nc)
        if mode == "faces":
            mg.update_coeffs(beta)
        else:
            mg.update_density(rho)
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        st = mg.solve(b, p, fixed_cycles=3)
        out.append((host(p), st))
        r = mg.residual_norm(b, p)
        out[-1] += (r,)
        mg.close()
    (p0, s0, r0), (p1, s1, r1) = out
    diff = np.max(np.abs(p0 - p1))
    print(f"{shape} {prec}: max |p_faces - p_density| = {diff:.3e}, rel_res {s1['rel_res']:.3e}")
    if dim == 3 and min(shape) >= 128:
        # the tiled density sweep updates cells away from the interface
        # without a division, (sum of neighbours - h^2 b rho) / 6: equal to
        # the stored-face sweep to rounding
        assert np.linalg.norm(p0 - p1) <= 1e-13 * np.linalg.norm(p0)
    else:
        assert np.array_equal(p0, p1)
    # the norms of the tiled density kernels are summed per tile, those of the
    # stored-face kernels per grid-stride block: equal up to summation order
    assert np.allclose(s0["hist"], s1["hist"], rtol=1e-13, atol=0)
    assert abs(r0 - r1) <= 1e-13 * r0


def test_density_path_vs_oracle_128(ib):
    shape = (128, 128, 128)
    n = shape
    h = 1.0 / 128
    Hn = _drop_H(shape, 3)
    b = W.random_cells(n, 3, 1.0, seed=62)
    b -= b.mean()
    ctx = ib.Context(3, n, h, max_markers=16)
    rho = ctx.density(dev(Hn), 1.0, 1e-3)
    mg = ib.Multigrid(3, n, h)
    mg.update_density(rho)
    p = torch.zeros(shape, dtype=torch.float64, device="cuda")
    st = mg.solve(dev(b), p, fixed_cycles=3)
    beta_o = poisson.face_beta(poisson.density(Hn, 1.0, 1e-3))
    po, cyc, hist = poisson.mg_solve(b, beta_o, h, fixed_cycles=3)
    err = float(np.linalg.norm(host(p) - po) / np.linalg.norm(po))
    print(f"density path vs oracle at 128^3, 3 cycles: rel L2 {err:.2e}")
    assert err <= 1e-11
    assert abs(st["rel_res"] - hist[-1]) <= 1e-6 * hist[-1]


def test_density_path_mixed_vs_oracle_128(ib):
    shape = (128, 128, 128)
    n = shape
    h = 1.0 / 128
    Hn = _drop_H(shape, 4)
    b = W.random_cells(n, 3, 1.0, seed=63)
    b -= b.mean()
    ctx = ib.Context(3, n, h, max_markers=16)
    rho = ctx.density(dev(Hn), 1.0, 1e-3)
    beta = ctx.coefficients(dev(Hn), 1.0, 1e-3)
    rho_o = poisson.density(Hn, 1.0, 1e-3)
    beta_o = poisson.face_beta(rho_o)
    for mode in ("density", "faces"):
        mg = ib.Multigrid(3, n, h, precision=ib.MG_MIXED)
        if mode == "density":
            mg.update_density(rho)
        else:
            mg.update_coeffs(beta)
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        st = mg.solve(dev(b), p, fixed_cycles=3)
        mg.close()
        po, _, hist = poisson.mg_solve_mixed(b, beta_o, h, fixed_cycles=3,
                                             rho=rho_o if mode == "density" else None)
        err = float(np.linalg.norm(host(p) - po) / np.linalg.norm(po))
        print(f"mixed {mode} path vs oracle at 128^3, 3 cycles: rel L2 {err:.2e}")
        assert err <= 1e-8
        assert abs(st["rel_res"] - hist[-1]) <= 1e-3 * hist[-1]


def test_density_null_and_errors(ib):
    mg = ib.Multigrid(2, (16, 16), 1 / 16)
    with pytest.raises(ib.IbError):
        ib._check(mg.lib.mg_update_density(mg.ptr, None, None))
    # solving before any coefficients is an error, not a fault
    p = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(ib.IbError):
        mg.solve(p.clone(), p)
