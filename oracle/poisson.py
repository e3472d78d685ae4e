"""Projection Poisson problem and its multigrid solution (oracle).

eq indicator: density rho = rho_out + (rho_in - rho_out) I with I = H (the
indicator Poisson equation, eq ind_psn, is solved exactly by H when the delta
vector is grad_h H). Face coefficient beta = 1/rho on faces, taken as
2 / (rho_L + rho_R) (arithmetic face density; the paper is silent).

eq ps with eq ns2_new (surface tension moved into the projection step):
  div(beta grad p) = div(u*/dt + beta F),
  u^{n+1} = u* + dt beta (F - grad p).
The Laplacian is the second-order centred finite-volume form (Section 2.1):
  (A p)_c = (1/h^2) sum over faces of beta_f (p_nb - p_c).
The box is periodic, so A is singular with the constants as null space; the
right side has its mean removed and the solution is normalised to zero mean.

Multigrid (the paper cites multigrid without settings): cell-centred V(nu1,
nu2) cycles, red-black Gauss-Seidel with red = (i+j+k) even swept first,
restriction = mean of the 2^dim children, prolongation = cell-centred
(bi/tri)linear with weights 3/4, 1/4 per axis, coarse face coefficient = mean
of the 2^(dim-1) fine faces on the coarse face, coarsest grid solved exactly
(bordered system with the zero-mean constraint), mean of p removed after every
cycle, stop when ||b - A p||_2 / ||b||_2 <= rtol.

Mixed precision: the same V-cycle in float32 (float32 coefficients, float32
right side and correction, coarsest level in float64) inside a float64
defect-correction loop r = b - A p (float64), p += V32(fl32(r)). The float32
coefficients are the float64 ones rounded, except on a finest level given by
its cell densities (rho passed): there the densities are rounded to float32
and each face coefficient is formed in float32, 2 / (fl32(rho_L) + fl32(rho_R)).

Krylov variant (an extension; the paper only names multigrid): flexible
conjugate gradients (the Polak-Ribiere form of the direction update, which
tolerates a preconditioner that is not exactly symmetric) preconditioned by
one V-cycle from a zero guess. The V-cycle here is not symmetric (mean
restriction with linear prolongation; red-then-black in both smoothing
passes), hence the flexible form. The recursively updated residual is
checked first; the stop is decided on the true residual b - A x (the
stopping test of the pressure solve is ||b - A p|| / ||b|| <= rtol).
"""
import numpy as np


# ----------------------------------------------------------------------------
# Coefficients, right side, update
# ----------------------------------------------------------------------------
def density(H, rho_in, rho_out):
    return rho_out + (rho_in - rho_out) * H


def face_beta(rho):
    dim = rho.ndim
    return [2.0 / (rho + np.roll(rho, 1, axis=dim - 1 - d)) for d in range(dim)]


def divergence(w, h):
    """(1/h) sum_d [w_d(c + e_d) - w_d(c)] with faces at the low side."""
    dim = w[0].ndim
    out = np.zeros_like(w[0])
    for d in range(dim):
        out += np.roll(w[d], -1, axis=dim - 1 - d) - w[d]
    return out / h


def gradient(p, h):
    dim = p.ndim
    return [(p - np.roll(p, 1, axis=dim - 1 - d)) / h for d in range(dim)]


def rhs(u_star, F, beta, dt, h):
    w = [u_star[d] / dt + beta[d] * F[d] for d in range(len(beta))]
    b = divergence(w, h)
    return b - b.mean()


def velocity_update(u_star, F, beta, p, dt, h):
    g = gradient(p, h)
    return [u_star[d] + dt * beta[d] * (F[d] - g[d]) for d in range(len(beta))]


# ----------------------------------------------------------------------------
# Operator and smoother
# ----------------------------------------------------------------------------
def apply_A(p, beta, h):
    dim = p.ndim
    out = np.zeros_like(p)
    for d in range(dim):
        ax = dim - 1 - d
        bl = beta[d]
        br = np.roll(beta[d], -1, axis=ax)
        out += br * (np.roll(p, -1, axis=ax) - p) - bl * (p - np.roll(p, 1, axis=ax))
    return out / (h * h)


def color_mask(shape, color):
    grids = np.indices(shape)
    return (grids.sum(axis=0) % 2) == color


def rbgs_sweep(p, b, beta, h):
    """One red-black Gauss-Seidel sweep in place: red (index sum even), then black."""
    dim = p.ndim
    for color in (0, 1):
        num = np.zeros_like(p)
        diag = np.zeros_like(p)
        for d in range(dim):
            ax = dim - 1 - d
            bl = beta[d]
            br = np.roll(beta[d], -1, axis=ax)
            num += br * np.roll(p, -1, axis=ax) + bl * np.roll(p, 1, axis=ax)
            diag += br + bl
        new = (num - (h * h) * b) / diag
        m = color_mask(p.shape, color)
        p[m] = new[m]
    return p


# ----------------------------------------------------------------------------
# Grid transfer
# ----------------------------------------------------------------------------
def restrict(r):
    dim = r.ndim
    if dim == 2:
        ny, nx = r.shape
        return r.reshape(ny // 2, 2, nx // 2, 2).mean(axis=(1, 3))
    nz, ny, nx = r.shape
    return r.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def _prolong_axis(e, ax):
    """Cell-centred linear interpolation along one axis (length doubles)."""
    n = e.shape[ax]
    left = np.roll(e, 1, axis=ax)
    right = np.roll(e, -1, axis=ax)
    even = 0.75 * e + 0.25 * left       # fine cell 2I sits toward I-1
    odd = 0.75 * e + 0.25 * right       # fine cell 2I+1 sits toward I+1
    shape = list(e.shape)
    shape[ax] = 2 * n
    out = np.empty(shape, dtype=e.dtype)
    sl_e = [slice(None)] * e.ndim
    sl_o = [slice(None)] * e.ndim
    sl_e[ax] = slice(0, None, 2)
    sl_o[ax] = slice(1, None, 2)
    out[tuple(sl_e)] = even
    out[tuple(sl_o)] = odd
    return out


def prolong(e):
    out = e
    for ax in range(e.ndim):
        out = _prolong_axis(out, ax)
    return out


def coarsen_beta(beta):
    """Coarse face coefficient = mean of the fine faces covering the coarse face."""
    dim = beta[0].ndim
    out = []
    for d in range(dim):
        ax = dim - 1 - d
        sl = [slice(None)] * dim
        sl[ax] = slice(0, None, 2)       # fine faces on coarse face planes
        f = beta[d][tuple(sl)]
        # average over the other axes in pairs
        for a in range(dim):
            if a == ax:
                continue
            n = f.shape[a]
            shp = list(f.shape)
            shp[a:a + 1] = [n // 2, 2]
            f = f.reshape(shp).mean(axis=a + 1)
        out.append(f)
    return out


# ----------------------------------------------------------------------------
# Exact solves
# ----------------------------------------------------------------------------
def dense_matrix(beta, h):
    shape = beta[0].shape
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = apply_A(e.reshape(shape), beta, h).ravel()
    return A


def bordered_solve(A, b):
    """Solve A x = b, sum(x) = 0 through [[A, 1], [1^T, 0]]."""
    N = A.shape[0]
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = A
    M[:N, N] = 1.0
    M[N, :N] = 1.0
    rhs_ = np.zeros(N + 1)
    rhs_[:N] = b
    return np.linalg.solve(M, rhs_)[:N]


def direct_solve(b, beta, h):
    A = dense_matrix(beta, h)
    return bordered_solve(A, b.ravel()).reshape(b.shape)


def fft_solve(b, beta_const, h):
    """Constant-coefficient periodic solve by diagonalisation (zero-mean)."""
    shape = b.shape
    lam = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = np.arange(n)
        s = np.sin(np.pi * k / n) ** 2
        sh = [1] * len(shape)
        sh[ax] = n
        lam = lam + s.reshape(sh)
    lam = -(4.0 * beta_const / (h * h)) * lam
    bh = np.fft.fftn(b)
    ph = np.zeros_like(bh)
    nz = lam != 0.0
    ph[nz] = bh[nz] / lam[nz]
    return np.real(np.fft.ifftn(ph))


# ----------------------------------------------------------------------------
# Multigrid
# ----------------------------------------------------------------------------
def face_beta_f32(rho):
    """Float32 face coefficients formed in float32 from the float32 densities."""
    r = np.asarray(rho, dtype=np.float64).astype(np.float32)
    dim = r.ndim
    return [np.float32(2.0) / (r + np.roll(r, 1, axis=dim - 1 - d)) for d in range(dim)]


class Hierarchy:
    def __init__(self, beta, h, n_coarsest=4, dtype=np.float64, rho=None):
        self.levels = []
        b = [np.asarray(x, dtype=np.float64) for x in beta]
        hl = h
        while True:
            if not self.levels and rho is not None and dtype == np.float32:
                self.levels.append((face_beta_f32(rho), hl))
            else:
                self.levels.append(([x.astype(dtype) for x in b], hl))
            if min(b[0].shape) <= n_coarsest:
                break
            b = coarsen_beta(b)
            hl = 2.0 * hl
        # the coarsest level keeps float64 coefficients for its exact solve
        bc, hc = [np.asarray(x, dtype=np.float64) for x in b], hl
        self.coarse_A = dense_matrix(bc, hc)
        self.dtype = dtype


def vcycle(hier, level, p, b, nu1=2, nu2=2):
    beta, h = hier.levels[level]
    if level == len(hier.levels) - 1:
        x = bordered_solve(hier.coarse_A, np.asarray(b, dtype=np.float64).ravel())
        return x.reshape(b.shape).astype(p.dtype)
    for _ in range(nu1):
        rbgs_sweep(p, b, beta, h)
    r = b - apply_A(p, beta, h)
    bc = restrict(r)
    ec = vcycle(hier, level + 1, np.zeros_like(bc), bc, nu1, nu2)
    p += prolong(ec)
    for _ in range(nu2):
        rbgs_sweep(p, b, beta, h)
    return p


def rel_residual(p, b, beta, h):
    r = b - apply_A(p, beta, h)
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b * b)))


def mg_solve(b, beta, h, p0=None, rtol=1e-10, max_cycles=100, nu1=2, nu2=2, n_coarsest=4,
             fixed_cycles=None):
    """FP64 V-cycles; returns (p, cycles, residual history)."""
    hier = Hierarchy(beta, h, n_coarsest)
    p = np.zeros_like(b) if p0 is None else np.array(p0, dtype=np.float64)
    hist = [rel_residual(p, b, beta, h)]
    cycles = 0
    while (fixed_cycles is None and hist[-1] > rtol and cycles < max_cycles) or \
          (fixed_cycles is not None and cycles < fixed_cycles):
        p = vcycle(hier, 0, p, b, nu1, nu2)
        p -= p.mean()
        cycles += 1
        hist.append(rel_residual(p, b, beta, h))
    return p, cycles, hist


def mg_solve_mixed(b, beta, h, p0=None, rtol=1e-10, max_cycles=100, nu1=2, nu2=2,
                   n_coarsest=4, fixed_cycles=None, rho=None):
    """Float32 V-cycle inside float64 defect correction (rho: the finest
    level's cell densities, from which its float32 coefficients are formed)."""
    hier = Hierarchy(beta, h, n_coarsest, dtype=np.float32, rho=rho)
    p = np.zeros_like(b) if p0 is None else np.array(p0, dtype=np.float64)
    hist = [rel_residual(p, b, beta, h)]
    cycles = 0
    while (fixed_cycles is None and hist[-1] > rtol and cycles < max_cycles) or \
          (fixed_cycles is not None and cycles < fixed_cycles):
        r = b - apply_A(p, beta, h)
        r32 = r.astype(np.float32)
        e = vcycle(hier, 0, np.zeros_like(r32), r32, nu1, nu2)
        p = p + e.astype(np.float64)
        p -= p.mean()
        cycles += 1
        hist.append(rel_residual(p, b, beta, h))
    return p, cycles, hist


# ----------------------------------------------------------------------------
# Flexible conjugate gradients preconditioned by multigrid
# ----------------------------------------------------------------------------
def fcg(apply, precond, b, x0=None, rtol=1e-10, max_iter=100, fixed_iters=None):
    """Flexible CG for an SPD (or, as here, positive semidefinite with b in
    its range) operator. Returns (x, iterations, history of ||r|| / ||b||),
    r updated recursively:

        r = b - A x, z = M(r), d = z, rz = (r, z)
        repeat: q = A d, alpha = rz / (d, q), x += alpha d, r -= alpha q,
                z = M(r), beta = (r_new - r_old, z) / rz = -alpha (q, z) / rz,
                rz = (r, z), d = z + beta d
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn]
    it = 0

    def done():
        if fixed_iters is not None:
            return it >= fixed_iters
        return hist[-1] <= rtol or it >= max_iter

    if done():
        return x, it, hist
    z = precond(r)
    d = z.copy()
    rz = np.vdot(r, z)
    while True:
        q = apply(d)
        alpha = rz / np.vdot(d, q)
        x += alpha * d
        r -= alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bn)
        if fixed_iters is None and hist[-1] <= rtol:
            # the stop is decided on the true residual; when it has not
            # reached rtol it replaces the recursive one and CG goes on
            r_true = b - apply(x)
            hist[-1] = np.linalg.norm(r_true) / bn
            if hist[-1] > rtol:
                r = r_true
        if done():
            break
        z = precond(r)
        beta = -alpha * np.vdot(q, z) / rz
        rz = np.vdot(r, z)
        d = z + beta * d
    return x, it, hist


def mg_pcg(b, beta, h, p0=None, rtol=1e-10, max_iter=100, nu1=2, nu2=2, n_coarsest=4,
           fixed_iters=None, mixed=False, rho=None):
    """FCG with one V(nu1, nu2) cycle from zero as preconditioner (float32
    V-cycle on fl32(r) when mixed, its finest coefficients from rho when
    given); mean of p removed at the end."""
    hier = Hierarchy(beta, h, n_coarsest, dtype=np.float32 if mixed else np.float64, rho=rho)

    def precond(r):
        if mixed:
            r32 = r.astype(np.float32)
            return vcycle(hier, 0, np.zeros_like(r32), r32, nu1, nu2).astype(np.float64)
        return vcycle(hier, 0, np.zeros_like(r), r, nu1, nu2)

    p, it, hist = fcg(lambda v: apply_A(v, beta, h), precond, b, p0, rtol, max_iter, fixed_iters)
    p -= p.mean()
    return p, it, hist

