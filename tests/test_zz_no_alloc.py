"""The allocation-free residual norm (mg_residual_norm_noalloc) through the C
ABI against mg_residual_norm on a handle given the same densities: two calls
in a row, the second on a smaller grid (the fixed device array keeps the first
call's contents), then a 2D grid. Same kernels and summation order, so the
values agree to rounding (observed: bit for bit)."""
import numpy as np
import pytest

from paper_1807_10504_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _drop_rho(shape, seed):
    g = np.indices(shape)
    r = np.sqrt(sum(((g[a] + 0.5) / shape[a] - 0.5) ** 2 for a in range(len(shape))))
    h = 1.0 / max(shape)
    H = np.clip((0.3 - r) / (3 * h) + 0.5, 0.0, 1.0)
    ramp = (H > 0) & (H < 1)
    H[ramp] += 0.01 * np.random.default_rng(seed).standard_normal(ramp.sum())
    return 1e-3 + (1.0 - 1e-3) * np.clip(H, 0.0, 1.0)


@pytest.fixture(scope="module")
def ib():
    from paper_1807_10504_amd import ibproj
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ibproj.load()
    return ibproj


def _case(ib, shape, seed):
    dim = len(shape)
    n = tuple(reversed(shape))
    h = 1.0 / n[0]
    rho = torch.from_numpy(_drop_rho(shape, seed)).cuda()
    b = W.random_cells(n, dim, 1.0, seed=seed + 1)
    b = torch.from_numpy(b - b.mean()).cuda()
    p = torch.from_numpy(W.random_cells(n, dim, 0.1, seed=seed + 2)).cuda()
    rel = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    ib.residual_norm_noalloc(dim, n, h, rho, b, p, rel)
    got = rel.item()
    mg = ib.Multigrid(dim, n, h)
    mg.update_density(rho)
    ref = mg.residual_norm(b, p)
    mg.close()
    print(f"{shape}: noalloc {got!r} vs mg_residual_norm {ref!r}")
    return got, ref


def test_noalloc_residual_norm_matches_handle_version(ib):
    cases = [((128, 128, 128), 11), ((32, 32, 32), 21), ((64, 96), 31)]
    for shape, seed in cases:
        got, ref = _case(ib, shape, seed)
        assert ref > 0.0
        assert abs(got - ref) <= 1e-14 * ref


def test_noalloc_zero_right_side_gives_zero(ib):
    shape = (32, 32, 64)
    n = tuple(reversed(shape))
    rho = torch.from_numpy(_drop_rho(shape, 41)).cuda()
    z = torch.zeros(shape, dtype=torch.float64, device="cuda")
    rel = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    ib.residual_norm_noalloc(3, n, 1.0 / n[0], rho, z, z, rel)
    assert rel.item() == 0.0
