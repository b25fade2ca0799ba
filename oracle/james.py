"""James (1977) vacuum boundary: screening masses, discrete Green's functions
and the boundary convolution (Sec. 4) -- oracle side (test infrastructure
only).

Ghost cells.  The Dirichlet ghost cells of the problem grid (pole edges have
none) are enumerated in the fixed order: inner radial (i=0, j=1..n_b), outer
radial (i=n_a+1, j=1..n_b), lower theta/z (i=1..n_a, j=0), upper theta/z
(i=1..n_a, j=n_b+1).  Indices are global fine-grid indices; interior cells
are 1..n.

Screening mass (Eqs. charge_sph, charge_cyl): sigma at a ghost cell is
(1/4piG) times the ghost cell's own coupling toward its interior neighbour
times Psi there (Psi vanishes on and outside the boundary).  The 1/(4 pi G)
is applied in both geometries.

Discrete Green's function (Sec. 4.2).  Gt^m(t <- s) = G^m * Delta V_s with
Delta V_s the full 3D volume (including Delta phi) of the source ghost cell s;
it solves L_m Gt = 4 pi G e_s on a box of cells around the source, with
* Dirichlet ring values Delta V_s * Gc^m, where Gc^m is the unnormalised
  m-th Fourier coefficient of -G/|x - x'| (Eqs. DGF_bc_sph / DGF_bc_cyl,
  k = 0..N_phi-1);
* on the inner radial edge of a clipped or extended box, the radial
  derivative of Gc^m as a Neumann condition (the derivative equations of
  Sec. 4.2, k = 0..N_phi-1), evaluated on the edge face;
* pole parity where the box reaches a pole.
Boxes: uniform radial grids use the auxiliary grid of (2 n_pad + 1)^2 cells
centred on the source (outer ring = Dirichlet data, (2 n_pad - 1)^2 cells
solved); when its inner ghost cell would reach r <= 0 the box is clipped at
the innermost positive face with the Neumann condition there, and at a pole
with parity.  Logarithmic radial grids use the extended domain: n_a - n_pad
cells added inside, n_pad outside, and n_b/2 above and below unless the edge
is a pole.  Field ghosts inside the box take the solved value, all others
Delta V_s * Gc^m.

Parity status: the DGF tables are *parity unpinned* beyond the physics checks
(analytic potentials, consistency of the auxiliary and extended definitions,
agreement with Gc far from the source); there is no closed form.
"""
import math

import numpy as np
import scipy.sparse.linalg as spla

from .geometry import SPH, LOG, Axis1D, radial_face
from .operator import DIRICHLET, NEUMANN, POLE, PlaneOperator, main_edges

FOUR_PI = 4.0 * math.pi


# -- ghost cells of the problem grid -------------------------------------------
class GhostSet:
    """The Dirichlet ghost cells of the problem grid with their geometry."""

    def __init__(self, spec):
        self.spec = spec
        A = Axis1D(spec, "a", 1, spec.n_a, 1)
        B = Axis1D(spec, "b", 1, spec.n_b, 1)
        self.A, self.B = A, B
        edges = main_edges(spec)
        R = A.metric_R() if spec.geometry == SPH else np.ones(spec.n_a)
        gi, gj, coup, edge = [], [], [], []
        up0, _ = A.couplings(0)
        _, dnN = A.couplings(spec.n_a + 1)
        for j in range(1, spec.n_b + 1):
            gi.append(0); gj.append(j); coup.append(up0); edge.append("a_lo")
        for j in range(1, spec.n_b + 1):
            gi.append(spec.n_a + 1); gj.append(j); coup.append(dnN); edge.append("a_hi")
        if edges["b_lo"] == DIRICHLET:
            upb0, _ = B.couplings(0)
            for i in range(1, spec.n_a + 1):
                gi.append(i); gj.append(0); coup.append(R[i - 1] * upb0); edge.append("b_lo")
        if edges["b_hi"] == DIRICHLET:
            _, dnbN = B.couplings(spec.n_b + 1)
            for i in range(1, spec.n_a + 1):
                gi.append(i); gj.append(spec.n_b + 1); coup.append(R[i - 1] * dnbN); edge.append("b_hi")
        self.i = np.array(gi)
        self.j = np.array(gj)
        self.coupling = np.array(coup, dtype=np.float64)   # ghost -> interior
        self.edge = np.array(edge)
        self.a = A.cent[self.i]
        self.b = B.cent[self.j]
        self.dv3 = A.vol[self.i] * B.vol[self.j] * spec.dphi
        self.n = len(self.i)

    def adjacent(self):
        """Interior (0-based) cell adjacent to every ghost."""
        ia = np.clip(self.i, 1, self.spec.n_a) - 1
        jb = np.clip(self.j, 1, self.spec.n_b) - 1
        return ia, jb


def screening_mass(spec, ghosts, psi_modes):
    """sigma^m at every ghost cell, shape (n_modes, n_ghost)."""
    ia, jb = ghosts.adjacent()
    return ghosts.coupling[None, :] * psi_modes[:, ia, jb] / (FOUR_PI * spec.G)


def boundary_ghost_values(spec, ghosts, values):
    """Map per-ghost values (n_ghost,) to the per-edge dict used by
    PlaneOperator.dirichlet_rhs."""
    out = {}
    for e in ("a_lo", "a_hi", "b_lo", "b_hi"):
        sel = ghosts.edge == e
        if np.any(sel):
            out[e] = values[sel]
    return out


# -- continuous-kernel Fourier coefficients ------------------------------------
def _angles(n_phi, m):
    k = np.arange(n_phi)
    return np.cos(2.0 * math.pi * k / n_phi), np.cos(2.0 * math.pi * m * k / n_phi)


def kernel_mode(spec, m, a, b, a_s, b_s):
    """Gc^m(x, x_s) = -G sum_k cos(2 pi m k/N) / |x - x_s(phi_k)| for field
    points (a, b) (arrays) and one source (a_s, b_s) (Eq. DGF_bc_sph /
    DGF_bc_cyl)."""
    ck, cmk = _angles(spec.n_phi, m)
    a = np.asarray(a, dtype=np.float64)[..., None]
    b = np.asarray(b, dtype=np.float64)[..., None]
    if spec.geometry == SPH:
        A = a * a + a_s * a_s - 2.0 * a * a_s * np.cos(b) * math.cos(b_s)
        B = 2.0 * a * a_s * np.sin(b) * math.sin(b_s)
        d2 = A - B * ck
    else:
        d2 = a * a + a_s * a_s - 2.0 * a * a_s * ck + (b - b_s) ** 2
    return -spec.G * np.sum(cmk / np.sqrt(d2), axis=-1)


def kernel_mode_dr(spec, m, a, b, a_s, b_s):
    """Radial derivative of Gc^m at field points (a, b) (the derivative
    equations of Sec. 4.2)."""
    ck, cmk = _angles(spec.n_phi, m)
    a = np.asarray(a, dtype=np.float64)[..., None]
    b = np.asarray(b, dtype=np.float64)[..., None]
    if spec.geometry == SPH:
        A = a * a + a_s * a_s - 2.0 * a * a_s * np.cos(b) * math.cos(b_s)
        B = 2.0 * a * a_s * np.sin(b) * math.sin(b_s)
        C = a - a_s * np.cos(b) * math.cos(b_s)
        D = a_s * np.sin(b) * math.sin(b_s)
        num = C - D * ck
        den = (A - B * ck) ** 1.5
    else:
        num = a - a_s * ck
        den = (a * a + a_s * a_s - 2.0 * a * a_s * ck + (b - b_s) ** 2) ** 1.5
    return spec.G * np.sum(num * cmk / den, axis=-1)


# -- boxes ----------------------------------------------------------------------
def _first_positive_cell(spec):
    """Smallest global radial cell index whose inner face is > 0."""
    i = 1
    while radial_face(spec, i - 2) > 0.0:
        i -= 1
        if i < -100000:
            raise ValueError("radial law never reaches zero")
    return i


def _b_range(spec, lo_want, hi_want):
    """Clip a theta/z index range at poles; returns (lo, hi, edge_lo, edge_hi)."""
    lo, hi = lo_want, hi_want
    e_lo = e_hi = DIRICHLET
    if spec.pole_lo() and lo <= 1:
        lo, e_lo = 1, POLE
    if spec.pole_hi() and hi >= spec.n_b:
        hi, e_hi = spec.n_b, POLE
    if spec.geometry == SPH:
        from .geometry import b_face
        if e_lo == DIRICHLET and b_face(spec, lo - 2) < 0.0:
            raise ValueError("DGF box crosses theta = 0 away from a pole")
        if e_hi == DIRICHLET and b_face(spec, hi + 1) > math.pi:
            raise ValueError("DGF box crosses theta = pi away from a pole")
    return lo, hi, e_lo, e_hi


def aux_box(spec, i_s, j_s, n_pad):
    """Index box (interior cells) and edge kinds of the auxiliary grid of a
    source at global (i_s, j_s)."""
    h = n_pad - 1
    i_lo, i_hi = i_s - h, i_s + h
    e_alo = DIRICHLET
    if radial_face(spec, i_lo - 2) <= 0.0:
        i_lo = _first_positive_cell(spec)
        e_alo = NEUMANN
    j_lo, j_hi, e_blo, e_bhi = _b_range(spec, j_s - h, j_s + h)
    return (i_lo, i_hi, j_lo, j_hi), {"a_lo": e_alo, "a_hi": DIRICHLET, "b_lo": e_blo, "b_hi": e_bhi}


def extended_box(spec, n_pad):
    """Index box and edge kinds of the extended domain (log radial grids)."""
    i_lo, i_hi = 1 - (spec.n_a - n_pad), spec.n_a + n_pad
    if spec.pole_lo() and spec.pole_hi():
        j_lo, j_hi, e_blo, e_bhi = 1, spec.n_b, POLE, POLE
    else:
        ext = spec.n_b // 2
        j_lo, j_hi, e_blo, e_bhi = _b_range(spec, 1 - ext, spec.n_b + ext)
    return (i_lo, i_hi, j_lo, j_hi), {"a_lo": NEUMANN, "a_hi": DIRICHLET, "b_lo": e_blo, "b_hi": e_bhi}


def dgf_method(spec):
    return "extended" if spec.radial == LOG else "aux"


def _box_rhs(spec, op, m, a_s, b_s, dv_s, src_local, homogeneous=False):
    """Right-hand side of L_m Gt = 4 pi G e_s with the box boundary data
    (none when ``homogeneous``: zero ghosts and zero inner flux)."""
    A, B = op.A, op.B
    rhs = np.zeros((op.n_a, op.n_b))
    rhs[src_local] += FOUR_PI * spec.G
    if homogeneous:
        return rhs
    ghosts = {}
    if op.edges["a_lo"] == DIRICHLET:
        ghosts["a_lo"] = dv_s * kernel_mode(spec, m, np.full(op.n_b, A.cent[0]), B.cent[1:-1], a_s, b_s)
    if op.edges["a_hi"] == DIRICHLET:
        ghosts["a_hi"] = dv_s * kernel_mode(spec, m, np.full(op.n_b, A.cent[-1]), B.cent[1:-1], a_s, b_s)
    if op.edges["b_lo"] == DIRICHLET:
        ghosts["b_lo"] = dv_s * kernel_mode(spec, m, A.cent[1:-1], np.full(op.n_a, B.cent[0]), a_s, b_s)
    if op.edges["b_hi"] == DIRICHLET:
        ghosts["b_hi"] = dv_s * kernel_mode(spec, m, A.cent[1:-1], np.full(op.n_a, B.cent[-1]), a_s, b_s)
    if ghosts:
        rhs += op.dirichlet_rhs(ghosts)
    if op.edges["a_lo"] == NEUMANN:
        face = A.faces[1]
        rhs += op.neumann_rhs(dv_s * kernel_mode_dr(spec, m, np.full(op.n_b, face), B.cent[1:-1], a_s, b_s))
    return rhs


def _box_operator(spec, box, edges):
    i_lo, i_hi, j_lo, j_hi = box
    A = Axis1D(spec, "a", i_lo, i_hi, 1)
    B = Axis1D(spec, "b", j_lo, j_hi, 1)
    return PlaneOperator(spec, A, B, edges)


def dgf_tables(spec, n_pad=16, method=None, modes=None, homogeneous=False):
    """Gt^m(t <- s) for all ghost pairs, shape (n_modes, n_ghost, n_ghost)
    (row = field ghost t, column = source ghost s).  ``homogeneous`` drops
    the box boundary data (used only to pin the source normalisation: the
    remaining part is exactly reciprocal, Gt(t <- s) / dV_s = Gt(s <- t) /
    dV_t, because the finite-volume operator is symmetric in the
    volume-weighted inner product).  The full tables are only approximately
    reciprocal (the boundary data of one source seen from another is not
    symmetric); see the module docstring for what pins them."""
    method = method or dgf_method(spec)
    gh = GhostSet(spec)
    modes = range(spec.n_modes) if modes is None else modes
    modes = list(modes)
    out = np.zeros((len(modes), gh.n, gh.n))
    if method == "extended":
        box, edges = extended_box(spec, n_pad)
        i_lo, i_hi, j_lo, j_hi = box
        if not (np.all((gh.i >= i_lo) & (gh.i <= i_hi)) and np.all((gh.j >= j_lo) & (gh.j <= j_hi))):
            raise ValueError(f"extended DGF box {box} does not contain every ghost cell (n_pad {n_pad} >= n_a?)")
        op = _box_operator(spec, box, edges)
        for mi, m in enumerate(modes):
            lu = spla.splu(op.matrix(m).tocsc())
            rhs = np.zeros((op.n_a * op.n_b, gh.n))
            for s in range(gh.n):
                src = (gh.i[s] - i_lo, gh.j[s] - j_lo)
                rhs[:, s] = _box_rhs(spec, op, m, gh.a[s], gh.b[s], gh.dv3[s], src, homogeneous).ravel()
            sol = lu.solve(rhs).reshape(op.n_a, op.n_b, gh.n)
            out[mi] = sol[gh.i - i_lo, gh.j - j_lo, :]
        return out
    for mi, m in enumerate(modes):
        for s in range(gh.n):
            box, edges = aux_box(spec, gh.i[s], gh.j[s], n_pad)
            i_lo, i_hi, j_lo, j_hi = box
            op = _box_operator(spec, box, edges)
            src = (gh.i[s] - i_lo, gh.j[s] - j_lo)
            rhs = _box_rhs(spec, op, m, gh.a[s], gh.b[s], gh.dv3[s], src, homogeneous)
            sol = spla.spsolve(op.matrix(m).tocsc(), rhs.ravel()).reshape(op.n_a, op.n_b)
            inside = (gh.i >= i_lo) & (gh.i <= i_hi) & (gh.j >= j_lo) & (gh.j <= j_hi)
            col = np.empty(gh.n)
            far = ~inside
            col[far] = gh.dv3[s] * kernel_mode(spec, m, gh.a[far], gh.b[far], gh.a[s], gh.b[s])
            col[inside] = sol[gh.i[inside] - i_lo, gh.j[inside] - j_lo]
            out[mi, :, s] = col
    return out


def boundary_potential(dgf, sigma):
    """Theta^m at every ghost = sum_s Gt^m(t <- s) sigma^m_s (Eqs. theta_left
    ... theta_top)."""
    return np.einsum("mts,ms->mt", dgf, sigma)
