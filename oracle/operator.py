"""Per-mode 2D Helmholtz operator L_m of Eqs. helmholz_sph / helmholz_cyl --
oracle side (test infrastructure only).

For spherical grids (Eq. discrete_poisson_sph with Eq. eigenv_sph)

  (L_m u)_ij = up_a[i] u_{i+1,j} + dn_a[i] u_{i-1,j}
             + R_i (up_b[j] u_{i,j+1} + dn_b[j] u_{i,j-1})
             + c_ij u_ij,
  c_ij = -(up_a + dn_a)[i] - R_i (up_b + dn_b)[j] - s_m^2 R_i T_j,

and for cylindrical grids (Eq. discrete_poisson_cyl with Eq. eigenv_cyl) the
same with R_i = 1 and the azimuthal term -s_m^2 W_i.

Boundary conditions act through one ghost cell per edge:
* Dirichlet: the ghost holds a given value (zero for the homogeneous
  problems of Sec. 4 step 1 and the multigrid error equation);
* pole: the ghost is (-1)^m times the adjacent cell (parity relation at the
  end of Sec. 4.2);
* Neumann: the flux through the edge face is prescribed (inner radial edge of
  the extended DGF domain, Sec. 4.2).
A ghost that is a fixed multiple kappa of the adjacent cell (pole: (-1)^m;
Neumann, homogeneous part: +1) is eliminated into the diagonal, so the
operator acts on interior values only; prescribed data moves to the
right-hand side (``dirichlet_rhs`` / ``neumann_rhs``).
"""
import numpy as np
import scipy.sparse as sp

from .geometry import SPH, Axis1D, mode_s2

DIRICHLET = "dirichlet"
POLE = "pole"
NEUMANN = "neumann"
EDGES = ("a_lo", "a_hi", "b_lo", "b_hi")


def kappa(kind, m):
    """Ghost = kappa * adjacent interior value for the homogeneous BC."""
    if kind == DIRICHLET:
        return 0.0
    if kind == POLE:
        return -1.0 if (m % 2) else 1.0
    if kind == NEUMANN:
        return 1.0
    raise ValueError(kind)


class PlaneOperator:
    """L_m on a rectangle of cells described by two Axis1D objects."""

    def __init__(self, spec, A: Axis1D, B: Axis1D, edges, dirichlet_kappa=None):
        self.spec, self.A, self.B = spec, A, B
        self.edges = dict(edges)
        # ghost factor of Dirichlet edges (0 unless a coarse multigrid level
        # moves its homogeneous condition off the ghost centre)
        self.dk = dict(dirichlet_kappa or {})
        self.n_a, self.n_b = A.n, B.n
        self.up_a, self.dn_a = A.interior_couplings()
        self.up_b, self.dn_b = B.interior_couplings()
        self.R = A.metric_R() if spec.geometry == SPH else np.ones(A.n)
        self.Pa = A.lambda_factor()
        self.Pb = B.lambda_factor()
        self.vol = np.outer(A.vol[1:-1], B.vol[1:-1])   # 2D volume weight

    # -- coefficients -------------------------------------------------------
    def coupling_arrays(self):
        """Off-diagonal coefficient arrays with the ghost couplings removed
        (ghost terms live in the diagonal or on the right-hand side)."""
        ua, da = self.up_a.copy(), self.dn_a.copy()
        ub, db = self.up_b.copy(), self.dn_b.copy()
        ua[-1] = 0.0
        da[0] = 0.0
        ub[-1] = 0.0
        db[0] = 0.0
        return ua, da, ub, db

    def kappa(self, edge, m):
        """Ghost = kappa * adjacent interior value on `edge` for mode m."""
        if self.edges[edge] == DIRICHLET:
            return self.dk.get(edge, 0.0)
        return kappa(self.edges[edge], m)

    def diag(self, m):
        """Diagonal c_ij of L_m with the kappa-ghosts folded in."""
        s2 = float(mode_s2(self.spec.n_phi, m))
        R = self.R[:, None]
        dn_a = self.dn_a.copy()
        if self.edges["a_lo"] == NEUMANN:
            # ghost = first cell (+ data): the inner coupling cancels exactly,
            # so the ghost centroid (possibly at r <= 0) is never used.
            dn_a[0] = 0.0
        else:
            dn_a[0] = self.dn_a[0] * (1.0 - self.kappa("a_lo", m))
        ca = -(self.up_a + dn_a)
        ca[-1] += self.kappa("a_hi", m) * self.up_a[-1]
        cb = -(self.up_b + self.dn_b)
        cb[0] += self.kappa("b_lo", m) * self.dn_b[0]
        cb[-1] += self.kappa("b_hi", m) * self.up_b[-1]
        c = ca[:, None] + R * cb[None, :] - s2 * self.Pa[:, None] * self.Pb[None, :]
        return c

    # -- application ----------------------------------------------------------
    def apply(self, u, m):
        """(L_m u) for interior values u of shape (n_a, n_b)."""
        ua, da, ub, db = self.coupling_arrays()
        out = self.diag(m) * u
        out[:-1, :] += ua[:-1, None] * u[1:, :]
        out[1:, :] += da[1:, None] * u[:-1, :]
        Rb = self.R[:, None]
        out[:, :-1] += Rb * ub[None, :-1] * u[:, 1:]
        out[:, 1:] += Rb * db[None, 1:] * u[:, :-1]
        return out

    def matrix(self, m):
        """Sparse matrix of L_m, row-major (a slow, b fast) unknown order."""
        na, nb = self.n_a, self.n_b
        idx = np.arange(na * nb).reshape(na, nb)
        ua, da, ub, db = self.coupling_arrays()
        rows = [idx.ravel()]
        cols = [idx.ravel()]
        vals = [self.diag(m).ravel()]
        Rb = np.repeat(self.R[:, None], nb, axis=1)
        rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel())
        vals.append(np.repeat(ua[:-1, None], nb, axis=1).ravel())
        rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel())
        vals.append(np.repeat(da[1:, None], nb, axis=1).ravel())
        rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel())
        vals.append((Rb[:, :-1] * ub[None, :-1]).ravel())
        rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel())
        vals.append((Rb[:, 1:] * db[None, 1:]).ravel())
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(na * nb, na * nb))

    # -- boundary data -------------------------------------------------------
    def dirichlet_rhs(self, ghosts):
        """Right-hand-side change -(coupling to ghost) * ghost value for the
        Dirichlet edges.  ``ghosts`` maps edge name -> array of ghost values
        along that edge (length n_b for a_lo/a_hi, n_a for b_lo/b_hi)."""
        out = np.zeros((self.n_a, self.n_b), dtype=np.result_type(*[np.asarray(v) for v in ghosts.values()], np.float64))
        if "a_lo" in ghosts:
            out[0, :] -= self.dn_a[0] * ghosts["a_lo"]
        if "a_hi" in ghosts:
            out[-1, :] -= self.up_a[-1] * ghosts["a_hi"]
        if "b_lo" in ghosts:
            out[:, 0] -= self.R * self.dn_b[0] * ghosts["b_lo"]
        if "b_hi" in ghosts:
            out[:, -1] -= self.R * self.up_b[-1] * ghosts["b_hi"]
        return out

    def neumann_face_factor(self):
        """Face area over cell volume of the inner radial face of the first
        cell: the flux A * dG/dr through it divided by Delta V."""
        lo, hi = self.A.faces[1], self.A.faces[2]
        if self.spec.geometry == SPH:
            return 3.0 * lo**2 / (hi**3 - lo**3)
        return 2.0 * lo / (hi**2 - lo**2)

    def neumann_rhs(self, dgdr):
        """Right-hand-side change for a prescribed inner radial derivative
        dgdr (length n_b): the ghost equals first - h * dgdr, whose known part
        moves to the right-hand side as + (A/dV) * dgdr."""
        out = np.zeros((self.n_a, self.n_b), dtype=np.asarray(dgdr).dtype)
        out[0, :] += self.neumann_face_factor() * dgdr
        return out

    def norm_v(self, u):
        """Volume-weighted RMS (Eq. L2_norm) of a plane (or stack of planes
        along the first axis)."""
        w = self.vol / self.vol.sum()
        return np.sqrt(np.sum(np.abs(u) ** 2 * w, axis=(-2, -1)))


def main_edges(spec):
    """Edge conditions of the problem grid: Dirichlet (ghost potential)
    everywhere except at poles."""
    return {
        "a_lo": DIRICHLET,
        "a_hi": DIRICHLET,
        "b_lo": POLE if spec.pole_lo() else DIRICHLET,
        "b_hi": POLE if spec.pole_hi() else DIRICHLET,
    }


def main_operator(spec, level=0):
    """L_m on multigrid level `level` (0 = finest) of the problem grid."""
    s = 2 ** level
    A = Axis1D(spec, "a", 1, spec.n_a // s, s)
    B = Axis1D(spec, "b", 1, spec.n_b // s, s)
    return PlaneOperator(spec, A, B, main_edges(spec))
