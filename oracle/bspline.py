"""Least-squares B-spline relocation of 2D markers and curvature (oracle).

Section 4 of the paper, followed step by step in plain scalar Python floats
(IEEE binary64; only + - * / and sqrt are used, each written out in a fixed
order so that an independent C++ implementation can reproduce the result bit
for bit):

1. advance: X* = X + dt U (forward Euler; the paper does not name the marker
   integrator);
2. parameters: chord-length distance travelled along the closed polyline
   from the first marker (the first marker is arbitrary);
3. knots: an arithmetic progression of spacing close to 1.5 grid cells; the
   curve is closed, so the span count is g = max(7, round(L / 1.5h)) and the
   spacing L / g (an exact 1.5h spacing cannot close the curve);
4. basis: the Cox-de Boor recursion (eq bspline; B_{i,0} = 1 on its own knot
   interval and 0 elsewhere), degree 3 ("order 3 ... continuity of
   curvature"), periodic;
5. coefficients: least squares for x(t) and y(t) separately (eq bspline_ls)
   through the normal equations, solved by a dense Cholesky factorisation;
   a non-positive pivot (Schoenberg-Whitney violated) is an error;
6. redistribution: markers at constant arc spacing along the fitted curve
   (8-point Gauss-Legendre arc length per span, then 6 Newton steps per
   marker), starting at the arc position of the first old marker;
7. curvature: eq ten_f with the tangents (eq b_tan) taken half-way between
   neighbouring markers: kappa_k = |T_{k+1/2} - T_{k-1/2}| / ds, positive
   when the curve turns counter-clockwise. Surface-tension density
   fs_k = sigma kappa_k, arc element ds_k = ds, unit inward normal = left
   perpendicular of the tangent at the marker.
"""
import math

# 8-point Gauss-Legendre rule on [-1, 1] (Abramowitz & Stegun, Table 25.4)
GL_X = (-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
        0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363)
GL_W = (0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
        0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763)

NEWTON_STEPS = 6


class BSplineError(RuntimeError):
    pass


def cox_de_boor(u):
    """Nonzero cubic and quadratic basis values on a span with local knots
    kappa_j = j (j = -3..4) at local parameter u.

    Returns (B3, B2): B3[r] = B_{s-3+r,3}(u), r = 0..3; B2[r] = B_{s-2+r,2}(u),
    r = 0..2, from the recursion
      B_{i,d} = (u - k_i)/(k_{i+d} - k_i) B_{i,d-1}
              + (k_{i+d+1} - u)/(k_{i+d+1} - k_{i+1}) B_{i+1,d-1}.
    """
    # B[d] maps basis index offset i (relative to the span, -d..0) to value
    B = {0: {0: 1.0}}
    for d in (1, 2, 3):
        cur = {}
        prev = B[d - 1]
        for i in range(-d, 1):
            lo = prev.get(i, 0.0)
            hi = prev.get(i + 1, 0.0)
            a = (u - float(i)) / (float(i + d) - float(i))
            b = (float(i + d + 1) - u) / (float(i + d + 1) - float(i + 1))
            cur[i] = a * lo + b * hi
        B[d] = cur
    return [B[3][i] for i in (-3, -2, -1, 0)], [B[2][i] for i in (-2, -1, 0)]


def _span_of(v, g):
    s = int(math.floor(v))
    if s > g - 1:
        s = g - 1
    if s < 0:
        s = 0
    return s


class ClosedCubic:
    def __init__(self, cx, cy):
        self.cx, self.cy = cx, cy
        self.g = len(cx)

    def point(self, s, u):
        B3, _ = cox_de_boor(u)
        x = 0.0
        y = 0.0
        for r in range(4):
            i = (s - 3 + r) % self.g
            x = x + self.cx[i] * B3[r]
            y = y + self.cy[i] * B3[r]
        return x, y

    def deriv(self, s, u):
        """dC/du on span s: sum_i c_i (3/(k_{i+3}-k_i) B_{i,2} - 3/(k_{i+4}-k_{i+1}) B_{i+1,2})."""
        _, B2 = cox_de_boor(u)
        q = {-2: B2[0], -1: B2[1], 0: B2[2]}
        dx = 0.0
        dy = 0.0
        for r in range(4):
            i = r - 3  # offset relative to the span
            db = (3.0 / 3.0) * q.get(i, 0.0) - (3.0 / 3.0) * q.get(i + 1, 0.0)
            ci = (s - 3 + r) % self.g
            dx = dx + self.cx[ci] * db
            dy = dy + self.cy[ci] * db
        return dx, dy

    def speed(self, s, u):
        dx, dy = self.deriv(s, u)
        return math.sqrt(dx * dx + dy * dy)

    def arc(self, s, u):
        """Arc length from the start of span s to local parameter u (8-point GL)."""
        half = 0.5 * u
        acc = 0.0
        for q in range(8):
            acc = acc + GL_W[q] * self.speed(s, half * (1.0 + GL_X[q]))
        return half * acc


def fit(X, h):
    """Least-squares closed cubic through markers X (list of (x, y)),
    parametrised by chord length from the first marker, on g = max(7,
    round(L / 1.5h)) uniform spans of L / g."""
    N = len(X)
    t = [0.0] * (N + 1)
    for k in range(N):
        x0, y0 = X[k]
        x1, y1 = X[(k + 1) % N]
        dx = x1 - x0
        dy = y1 - y0
        t[k + 1] = t[k] + math.sqrt(dx * dx + dy * dy)
    L = t[N]
    g = int(math.floor(L / (1.5 * h) + 0.5))
    if g < 7:
        g = 7
    tau = L / g
    return lsq_closed_cubic(X, [t[k] / tau for k in range(N)], g), tau


def lsq_closed_cubic(X, v, g):
    """eq bspline_ls: the closed cubic on g unit spans minimising
    sum_k |C(v_k) - X_k|^2 for the parameters v (in span units), through the
    normal equations (B^T B) c = B^T X and a Cholesky factorisation."""
    N = len(X)
    M = [[0.0] * g for _ in range(g)]
    bx = [0.0] * g
    by = [0.0] * g
    for k in range(N):
        s = _span_of(v[k], g)
        u = v[k] - float(s)
        B3, _ = cox_de_boor(u)
        idx = [(s - 3 + r) % g for r in range(4)]
        xk, yk = X[k]
        for a in range(4):
            ia = idx[a]
            bx[ia] = bx[ia] + B3[a] * xk
            by[ia] = by[ia] + B3[a] * yk
            for b in range(4):
                ib = idx[b]
                M[ia][ib] = M[ia][ib] + B3[a] * B3[b]
    # dense Cholesky M = L L^T, row by row
    Lm = [[0.0] * g for _ in range(g)]
    for i in range(g):
        for j in range(i + 1):
            s_ = M[i][j]
            for k in range(j):
                s_ = s_ - Lm[i][k] * Lm[j][k]
            if i == j:
                if not s_ > 0.0:
                    raise BSplineError("least-squares matrix not positive definite")
                Lm[i][i] = math.sqrt(s_)
            else:
                Lm[i][j] = s_ / Lm[j][j]

    def solve(rhs):
        z = [0.0] * g
        for i in range(g):
            s_ = rhs[i]
            for k in range(i):
                s_ = s_ - Lm[i][k] * z[k]
            z[i] = s_ / Lm[i][i]
        c = [0.0] * g
        for i in range(g - 1, -1, -1):
            s_ = z[i]
            for k in range(i + 1, g):
                s_ = s_ - Lm[k][i] * c[k]
            c[i] = s_ / Lm[i][i]
        return c

    return ClosedCubic(solve(bx), solve(by))


def _locate(curve, S, ell, sigma, s_start):
    """Span and local parameter of arc position sigma (6 Newton steps)."""
    g = curve.g
    s = s_start
    while s < g - 1 and S[s + 1] <= sigma:
        s = s + 1
    target = sigma - S[s]
    u = target / ell[s]
    for _ in range(NEWTON_STEPS):
        u = u - (curve.arc(s, u) - target) / curve.speed(s, u)
    return s, u


def relocate(X, U, dt, h, sigma):
    """Advance, refit and redistribute; returns (X_new, fs, ds, nrm) as lists."""
    N = len(X)
    Xs = [(X[k][0] + dt * U[k][0], X[k][1] + dt * U[k][1]) for k in range(N)]
    curve, _ = fit(Xs, h)
    g = curve.g
    ell = [curve.arc(s, 1.0) for s in range(g)]
    S = [0.0] * (g + 1)
    for s in range(g):
        S[s + 1] = S[s] + ell[s]
    Lc = S[g]
    ds = Lc / N
    Xn, nrm = [], []
    s = 0
    for k in range(N):
        s, u = _locate(curve, S, ell, float(k) * ds, s)
        Xn.append(curve.point(s, u))
        dx, dy = curve.deriv(s, u)
        sp = math.sqrt(dx * dx + dy * dy)
        nrm.append((-dy / sp, dx / sp))
    T = []
    s = 0
    for k in range(N):
        s, u = _locate(curve, S, ell, (float(k) + 0.5) * ds, s)
        dx, dy = curve.deriv(s, u)
        sp = math.sqrt(dx * dx + dy * dy)
        T.append((dx / sp, dy / sp))
    fs = []
    for k in range(N):
        tm = T[(k - 1) % N]
        tp = T[k]
        ddx = tp[0] - tm[0]
        ddy = tp[1] - tm[1]
        kap = math.sqrt(ddx * ddx + ddy * ddy) / ds
        if tm[0] * tp[1] - tm[1] * tp[0] < 0.0:
            kap = -kap
        fs.append(sigma * kap)
    return Xn, fs, [ds] * N, nrm
