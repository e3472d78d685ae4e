"""The fused phases of the cycle against the launch-per-phase cycle: the
persistent coarse-level kernel (one workgroup runs the sub-V-cycle of the
levels with at most 4096 cells) and, on 3D density levels (128^3 and up),
the prolongation folded into the first post-smoothing sweep. p and the
residual history bitwise equal, on 2D and 3D hierarchies, FP64 and mixed,
plain cycles and flexible CG, other smoothing counts, and the 256^3 flexible
CG of the headline step."""
import numpy as np
import pytest

from paper_1807_10504_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    from paper_1807_10504_amd import ibproj
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ibproj.load()
    return ibproj


def _H(shape):
    g = np.indices(shape)
    r = np.sqrt(sum(((g[a] + 0.5) / shape[a] - 0.5) ** 2 for a in range(len(shape))))
    return np.clip((0.3 - r) * max(shape) / 3 + 0.5, 0.0, 1.0)


CASES = [((512, 512), "fp64", 0, (2, 2)), ((128, 128, 128), "fp64", 0, (2, 2)),
         ((128, 128, 128), "mixed", 1, (2, 2)), ((32, 32, 32), "fp64", 1, (1, 1)),
         ((64, 64, 64), "mixed", 0, (2, 1)), ((256, 256), "mixed", 1, (2, 2)),
         ((128, 128, 128), "fp64", 1, (1, 3)), ((128, 128, 128), "mixed", 0, (2, 2)),
         ((256, 256, 256), "fp64", 1, (2, 2)), ((128, 128, 128), "fp64", 1, (0, 2)),
         ((256, 256), "mixed", 0, (0, 2))]


@pytest.mark.parametrize("shape,prec,krylov,nu", CASES)
def test_persistent_coarse_bitwise(ib, shape, prec, krylov, nu):
    dim = len(shape)
    n = tuple(reversed(shape))
    h = 1.0 / max(shape)
    H = torch.from_numpy(_H(shape)).cuda()
    b = W.random_cells(n, dim, 1.0, seed=81)
    b = torch.from_numpy(b - b.mean()).cuda()
    ctx = ib.Context(dim, n, h, max_markers=16)
    rho = ctx.density(H, 1.0, 1e-3)
    precision = ib.MG_MIXED if prec == "mixed" else ib.MG_FP64
    res = []
    for split in (1, 0):
        mg = ib.Multigrid(dim, n, h, precision=precision, krylov=krylov, nu1=nu[0], nu2=nu[1],
                          split_coarse=split)
        mg.update_density(rho)
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        st = mg.solve(b, p, fixed_cycles=4)
        torch.cuda.synchronize()
        res.append((p.cpu().numpy(), st["hist"]))
        mg.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]
