"""The paper's per-mode geometric multigrid (Sec. 3) -- oracle side (test
infrastructure only).

Correction-scheme V-cycle (Sec. 3, error equation L E = -D):
  pre-smooth nu_pre times, restrict the residual f - L u, recurse with a zero
  initial correction, prolong and add, post-smooth nu_post times; the
  coarsest level is solved by red-black point SOR (Sec. 3.3).

Smoother (Sec. 3.2, Algorithm 1, parallel ordering of Sec. 5.2): one
smoothing step = a radial-line phase then a polar-line phase.  A phase relaxes
the lines of one zebra colour (0-based even line index first), each by n_sor
SOR passes in even-odd point order (0-based even points first), then the
lines of the other colour.  The line right-hand side (source minus the fixed
couplings to neighbouring lines) does not change while a line is relaxed, so
every pass is a point update with the line's omega (Appendix A, WKB).

Transfers (Sec. 3.1): restriction and prolongation are bilinear in (r^2,
theta) (spherical) or (R, z) (cylindrical).  Prolongation uses the printed
opposite-corner area weights.  For restriction the printed weight S_ij
multiplies the fine point it is measured from; the default here reads it as
the opposite-corner (bilinear) weight like the prolongation, the literal
reading is available with ``restriction="literal"``.  Coarse ghosts in the
prolongation follow the homogeneous boundary condition of the error as the
coarse operator states it ((-1)^m mirror at poles, kappa_c at Dirichlet
edges, below).

Coarsening: factor two in both directions while both sides are even, the
smaller coarse side stays >= 2, the coarse inner radial ghost face stays at
r > 0 and the level has more than 128 cells (the paper does not fix the
coarsest size; a level that small is solved to convergence); the coarse
operator is rediscretised on the coarse faces.  The
paper leaves the coarse boundary closure open; here the error vanishes on
every level at the point where the problem grid puts it (the finest ghost
centre), not at the coarse ghost centre: a coarse Dirichlet ghost is
kappa_c times the adjacent coarse cell, with kappa_c from linear
interpolation through that point (coarse_dirichlet_kappa).  Only the
convergence rate depends on this (the finest operator is unchanged); it
takes m = 0 of the log-radial 128x64 sphere from 20 to 12 V-cycles.

Stopping rule (reading of the 1e-8 tolerance, Sec. 6 and Appendix B): mode m
is converged when ||D^m||_V <= tol * max(||D^m_0||_V, 1e-6 max_m' ||D^m'_0||_V)
where D_0 is the defect of the zero guess with the solve's boundary data and
||.||_V the volume-weighted RMS (Eq. L2_norm).
"""
import numpy as np

from .geometry import SPH, Axis1D, radial_face
from .omega import omega_1d, omega_2d
from .operator import PlaneOperator, main_edges

FLOOR = 1e-6
# by default a level of at most this many cells is the coarsest (it is
# solved to convergence; coarser levels would only add smoothing latency);
# the depth is a parameter of the hierarchy (the paper leaves it open)
MAX_COARSEST = 128


def level_sizes(spec, max_coarsest=MAX_COARSEST):
    """Level shapes: halve until a level has at most max_coarsest cells
    (after at least one halving), both sides stay even, the smaller coarse
    side stays >= 2 and the coarse inner ghost face stays at r > 0."""
    sizes = [(spec.n_a, spec.n_b)]
    s = 1
    while True:
        na, nb = sizes[-1]
        if na * nb <= max_coarsest and len(sizes) > 1:
            break
        if na % 2 or nb % 2 or min(na, nb) // 2 < 2:
            break
        if radial_face(spec, -2 * s) <= 0.0:     # coarse inner ghost face
            break
        sizes.append((na // 2, nb // 2))
        s *= 2
    return sizes


def coarse_dirichlet_kappa(fine0: Axis1D, coarse: Axis1D):
    """(kappa_lo, kappa_hi) of a coarse level's Dirichlet edges along one
    axis: the coarse ghost value g = kappa * (first coarse cell) that makes
    the straight line through the coarse ghost and first cell centres vanish
    at the finest level's ghost centre."""
    xg, x0, x1 = fine0.cent[0], coarse.cent[0], coarse.cent[1]
    k_lo = -(xg - x0) / (x1 - xg)
    n0, nc = fine0.n, coarse.n
    xg, xn1, xn = fine0.cent[n0 + 1], coarse.cent[nc + 1], coarse.cent[nc]
    k_hi = -(xn1 - xg) / (xg - xn)
    return k_lo, k_hi


class MGLevel:
    def __init__(self, spec, level):
        s = 2 ** level
        self.spec = spec
        self.stride = s
        A = Axis1D(spec, "a", 1, spec.n_a // s, s)
        B = Axis1D(spec, "b", 1, spec.n_b // s, s)
        self.A, self.B = A, B
        dk = {}
        if level > 0:
            dk["a_lo"], dk["a_hi"] = coarse_dirichlet_kappa(Axis1D(spec, "a", 1, spec.n_a, 1), A)
            dk["b_lo"], dk["b_hi"] = coarse_dirichlet_kappa(Axis1D(spec, "b", 1, spec.n_b, 1), B)
        self.op = PlaneOperator(spec, A, B, main_edges(spec), dk)
        self.n_a, self.n_b = A.n, B.n
        self.ua, self.da, self.ub, self.db = self.op.coupling_arrays()
        self.R = self.op.R
        self.vol = self.op.vol
        self._cache = {}

    def diag(self, m):
        key = ("d", m)
        if key not in self._cache:
            self._cache[key] = self.op.diag(m)
        return self._cache[key]

    def omega_lines(self, m):
        """(omega of every radial line j, omega of every polar line i)."""
        key = ("w", m)
        if key not in self._cache:
            c = self.diag(m)
            wr = np.array([omega_1d(self.A.cent, self.da, self.ua, c[:, j]) for j in range(self.n_b)])
            wb = np.array([omega_1d(self.B.cent, self.R[i] * self.db, self.R[i] * self.ub, c[i, :])
                           for i in range(self.n_a)])
            self._cache[key] = (wr, wb)
        return self._cache[key]

    def omega_coarse(self, m):
        key = ("w2", m)
        if key not in self._cache:
            Rb = self.R[:, None]
            self._cache[key] = omega_2d(self.A.cent, self.B.cent, self.ua, self.da,
                                        Rb * self.ub[None, :], Rb * self.db[None, :], self.diag(m))
        return self._cache[key]

    def apply(self, u, m):
        return self.op.apply(u, m)

    # -- one colour class of point updates -----------------------------------
    def _update(self, U, f, m, i0, j0, w):
        """SOR update of interior points with i % 2 == i0, j % 2 == j0 (0-based)
        in the padded array U (n_a+2, n_b+2); w broadcastable to that subset."""
        na, nb = self.n_a, self.n_b
        ii = slice(1 + i0, na + 1, 2)
        jj = slice(1 + j0, nb + 1, 2)
        nbsum = (self.ua[i0::2, None] * U[2 + i0:na + 2:2, jj]
                 + self.da[i0::2, None] * U[i0:na:2, jj]
                 + self.R[i0::2, None] * (self.ub[None, j0::2] * U[ii, 2 + j0:nb + 2:2]
                                          + self.db[None, j0::2] * U[ii, j0:nb:2]))
        c = self.diag(m)[i0::2, j0::2]
        tmp = (f[i0::2, j0::2] - nbsum) / c
        U[ii, jj] = (1.0 - w) * U[ii, jj] + w * tmp

    def smooth_exact(self, u, f, m):
        """One alternating step with exact line relaxation (the tridiagonal
        solve the paper names as the ideal, Sec. 3.2): zebra radial lines,
        then zebra polar lines, each line solved by the Thomas algorithm."""
        c = self.diag(m)
        U = np.zeros((self.n_a + 2, self.n_b + 2), dtype=np.complex128)
        U[1:-1, 1:-1] = u
        R = self.R
        for lc in (0, 1):                       # radial lines j
            js = np.arange(lc, self.n_b, 2)
            rhs = f[:, js] - R[:, None] * (self.ub[None, js] * U[1:-1, js + 2] + self.db[None, js] * U[1:-1, js])
            U[1:-1, js + 1] = thomas(self.da[:, None] * np.ones((1, len(js))), c[:, js],
                                     self.ua[:, None] * np.ones((1, len(js))), rhs)
        for lc in (0, 1):                       # polar lines i
            is_ = np.arange(lc, self.n_a, 2)
            rhs = f[is_, :] - (self.ua[is_, None] * U[is_ + 2, 1:-1] + self.da[is_, None] * U[is_, 1:-1])
            lo = (R[is_, None] * self.db[None, :]).T
            up = (R[is_, None] * self.ub[None, :]).T
            U[is_ + 1, 1:-1] = thomas(lo, c[is_, :].T, up, rhs.T).T
        u[...] = U[1:-1, 1:-1]

    def smooth(self, u, f, m, n_sor):
        """One alternating step: radial lines, then polar lines."""
        wr, wb = self.omega_lines(m)
        U = np.zeros((self.n_a + 2, self.n_b + 2), dtype=np.complex128)
        U[1:-1, 1:-1] = u
        for lc in (0, 1):                       # radial lines j, zebra colour lc
            w = wr[lc::2][None, :]
            for _ in range(n_sor):
                for pc in (0, 1):               # even-odd points i along the line
                    self._update(U, f, m, pc, lc, w)
        for lc in (0, 1):                       # polar lines i, zebra colour lc
            w = wb[lc::2][:, None]
            for _ in range(n_sor):
                for pc in (0, 1):
                    self._update(U, f, m, lc, pc, w)
        u[...] = U[1:-1, 1:-1]

    def coarse_solve(self, f, m, rtol=1e-10, max_sweeps=20000):
        """Red-black point SOR from a zero start until the residual 2-norm
        drops by rtol (or max_sweeps)."""
        w = self.omega_coarse(m)
        U = np.zeros((self.n_a + 2, self.n_b + 2), dtype=np.complex128)
        r0 = np.linalg.norm(f)
        sweeps = 0
        if r0 == 0.0:
            return U[1:-1, 1:-1].copy(), 0
        while sweeps < max_sweeps:
            for colour in (0, 1):               # red: (i + j) even
                for i0 in (0, 1):
                    j0 = (colour + i0) % 2
                    self._update(U, f, m, i0, j0, w)
            sweeps += 1
            if np.linalg.norm(f - self.apply(U[1:-1, 1:-1], m)) <= rtol * r0:
                break
        return U[1:-1, 1:-1].copy(), sweeps


def thomas(lower, diag, upper, rhs):
    """Solve tridiagonal systems along axis 0 (columns are independent
    systems): lower[k] x[k-1] + diag[k] x[k] + upper[k] x[k+1] = rhs[k]."""
    n = diag.shape[0]
    cp = np.zeros(diag.shape)
    dp = np.zeros(rhs.shape, dtype=np.result_type(rhs, np.float64))
    cp[0] = upper[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for k in range(1, n):
        den = diag[k] - lower[k] * cp[k - 1]
        cp[k] = upper[k] / den
        dp[k] = (rhs[k] - lower[k] * dp[k - 1]) / den
    x = np.zeros_like(dp)
    x[-1] = dp[-1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def _transfer_coord(geometry, which, x):
    """Coordinate in which transfers are bilinear: r^2 (spherical radius),
    theta, R or z."""
    if which == "a" and geometry == SPH:
        return x * x
    return x


def restriction_weights_1d(fine: Axis1D, coarse: Axis1D, geometry, which, literal=False):
    """(n_c, 2) weights of the two fine children of each coarse cell."""
    xf = _transfer_coord(geometry, which, fine.cent)
    xc = _transfer_coord(geometry, which, coarse.cent)
    n_c = coarse.n
    lo = xf[1:2 * n_c:2]          # children 2I-1 (1-based)
    hi = xf[2:2 * n_c + 1:2]      # children 2I
    X = xc[1:n_c + 1]
    w_lo = np.abs(hi - X) / np.abs(hi - lo)
    w_hi = np.abs(X - lo) / np.abs(hi - lo)
    if literal:
        w_lo, w_hi = w_hi, w_lo
    return np.stack([w_lo, w_hi], axis=1)


def prolongation_matrix_1d(fine: Axis1D, coarse: Axis1D, geometry, which, k_lo, k_hi):
    """(n_f, n_c) matrix of the 1D bilinear factor with coarse ghosts folded
    as ghost = kappa * adjacent coarse cell."""
    xf = _transfer_coord(geometry, which, fine.cent)
    xc = _transfer_coord(geometry, which, coarse.cent)
    n_f, n_c = fine.n, coarse.n
    P = np.zeros((n_f, n_c))
    for k in range(1, n_f + 1):
        I = (k + 1) // 2                       # coarse parent, 1-based
        if k % 2:                              # inner child: between I-1 and I
            c0, c1 = I - 1, I
        else:                                  # outer child: between I and I+1
            c0, c1 = I, I + 1
        x0, x1, x = xc[c0], xc[c1], xf[k]
        w0 = abs(x1 - x) / abs(x1 - x0)
        w1 = abs(x - x0) / abs(x1 - x0)
        for c, w in ((c0, w0), (c1, w1)):
            if c == 0:
                P[k - 1, 0] += k_lo * w
            elif c == n_c + 1:
                P[k - 1, n_c - 1] += k_hi * w
            else:
                P[k - 1, c - 1] += w
    return P


class Hierarchy:
    """The multigrid hierarchy of the problem grid and its V-cycle."""

    def __init__(self, spec, nu_pre=2, nu_post=2, n_sor=2, restriction="bilinear", line_solver="sor",
                 max_coarsest=MAX_COARSEST):
        self.spec = spec
        self.nu_pre, self.nu_post, self.n_sor = nu_pre, nu_post, n_sor
        self.line_solver = line_solver
        self.sizes = level_sizes(spec, max_coarsest)
        self.levels = [MGLevel(spec, l) for l in range(len(self.sizes))]
        lit = restriction == "literal"
        self.rw = []
        for l in range(len(self.levels) - 1):
            f, c = self.levels[l], self.levels[l + 1]
            self.rw.append((restriction_weights_1d(f.A, c.A, spec.geometry, "a", lit),
                            restriction_weights_1d(f.B, c.B, spec.geometry, "b", lit)))
        self._pcache = {}

    def restrict(self, l, r):
        wa, wb = self.rw[l]
        t = wa[:, 0, None] * r[0::2, :] + wa[:, 1, None] * r[1::2, :]
        return wb[None, :, 0] * t[:, 0::2] + wb[None, :, 1] * t[:, 1::2]

    def prolong(self, l, e, m):
        """Prolongation from level l+1 to level l."""
        key = (l, m % 2)
        if key not in self._pcache:
            f, c = self.levels[l], self.levels[l + 1]
            k = c.op.kappa
            Pa = prolongation_matrix_1d(f.A, c.A, self.spec.geometry, "a", k("a_lo", m), k("a_hi", m))
            Pb = prolongation_matrix_1d(f.B, c.B, self.spec.geometry, "b", k("b_lo", m), k("b_hi", m))
            self._pcache[key] = (Pa, Pb)
        Pa, Pb = self._pcache[key]
        return Pa @ e @ Pb.T

    def _smooth(self, lev, u, f, m):
        if self.line_solver == "exact":
            lev.smooth_exact(u, f, m)
        else:
            lev.smooth(u, f, m, self.n_sor)

    def vcycle(self, u, f, m, l=0):
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            u[...], _ = lev.coarse_solve(f, m)
            return
        for _ in range(self.nu_pre):
            self._smooth(lev, u, f, m)
        r = f - lev.apply(u, m)
        fc = self.restrict(l, r)
        ec = np.zeros_like(fc)
        self.vcycle(ec, fc, m, l + 1)
        u += self.prolong(l, ec, m)
        for _ in range(self.nu_post):
            self._smooth(lev, u, f, m)

    def defect_norm(self, u, f, m):
        lev = self.levels[0]
        return float(lev.op.norm_v(f - lev.apply(u, m)))

    def solve(self, f_modes, tol, u0=None, max_cycles=100, modes=None):
        """Solve every mode to the stopping rule; returns (u, cycles, final
        relative defects).  ``modes`` gives the azimuthal index of each plane
        (default 0..M-1)."""
        M = f_modes.shape[0]
        modes = list(range(M)) if modes is None else list(modes)
        u = np.zeros_like(f_modes, dtype=np.complex128) if u0 is None else np.array(u0, dtype=np.complex128)
        lev = self.levels[0]
        d0 = np.array([float(lev.op.norm_v(f_modes[m])) for m in range(M)])
        floor = FLOOR * d0.max() if M else 0.0
        thresh = tol * np.maximum(d0, floor)
        cycles = np.zeros(M, dtype=int)
        res = np.zeros(M)
        for p in range(M):
            m = modes[p]
            d = self.defect_norm(u[p], f_modes[p], m)
            while d > thresh[p] and cycles[p] < max_cycles:
                self.vcycle(u[p], f_modes[p], m)
                cycles[p] += 1
                d = self.defect_norm(u[p], f_modes[p], m)
            res[p] = d / max(d0[p], floor) if max(d0[p], floor) > 0 else 0.0
        return u, cycles, res
