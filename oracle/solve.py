"""The seven-step workflow of Sec. 5.1 -- oracle side (test infrastructure
only).

  1. DGF tables (precomputed once per grid, Sec. 4.2)
  2. forward azimuthal DFT of rho (Sec. 2.2)
  3. L_m Psi^m = 4 pi G rho^m with Psi = 0 on the boundary (Sec. 4 step 1)
  4. screening masses sigma^m (Eqs. charge_sph / charge_cyl)
  5. Theta^m = sum Gt^m sigma^m (Eqs. theta_left .. theta_top)
  6. L_m Phi^m = 4 pi G rho^m with Phi = -Theta^m on the boundary
  7. inverse DFT.

Steps 3 and 6 are linear systems whose exact solution is what the multigrid
of Sec. 3 converges to; the oracle solves them directly (sparse LU, the plain
definition).  ``oracle.multigrid`` holds the paper's iteration itself.
"""
import math

import numpy as np
import scipy.sparse.linalg as spla

from . import fourier
from .geometry import GridSpec
from .james import GhostSet, boundary_ghost_values, boundary_potential, dgf_tables, screening_mass
from .operator import main_operator

FOUR_PI = 4.0 * math.pi


class OraclePlan:
    """Precomputed per-grid data (operator, ghost set, DGF tables)."""

    def __init__(self, spec: GridSpec, n_pad=16, dgf_method=None, dgf=None):
        self.spec = spec
        self.op = main_operator(spec, 0)
        self.ghosts = GhostSet(spec)
        self.dgf = dgf if dgf is not None else dgf_tables(spec, n_pad=n_pad, method=dgf_method)
        self._lu = {}

    def lu(self, m):
        if m not in self._lu:
            self._lu[m] = spla.splu(self.op.matrix(m).tocsc())
        return self._lu[m]

    def solve_modes(self, rhs_modes):
        """Exact solution of L_m u^m = rhs^m for every mode (sparse LU of the
        real operator applied to real and imaginary parts)."""
        na, nb = self.spec.n_a, self.spec.n_b
        out = np.empty(rhs_modes.shape, dtype=np.complex128)
        for m in range(rhs_modes.shape[0]):
            lu = self.lu(m)
            r = np.asarray(rhs_modes[m], dtype=np.complex128).reshape(-1)
            out[m] = (lu.solve(r.real.copy()) + 1j * lu.solve(r.imag.copy())).reshape(na, nb)
        return out

    def source_modes(self, rho):
        """f^m = 4 pi G rho^m (steps 2)."""
        return FOUR_PI * self.spec.G * fourier.forward(rho)

    def boundary_rhs(self, theta_modes):
        """Right-hand-side change of step 6 (ghost potential -Theta^m)."""
        out = np.zeros((theta_modes.shape[0], self.spec.n_a, self.spec.n_b), dtype=np.complex128)
        for m in range(theta_modes.shape[0]):
            out[m] = self.op.dirichlet_rhs(boundary_ghost_values(self.spec, self.ghosts, -theta_modes[m]))
        return out

    def solve(self, rho, return_parts=False):
        """Phi (n_a, n_b, n_phi) for a real density rho of the same shape."""
        f = self.source_modes(rho)
        psi = self.solve_modes(f)
        sigma = screening_mass(self.spec, self.ghosts, psi)
        theta = boundary_potential(self.dgf, sigma)
        f2 = f + self.boundary_rhs(theta)
        phi_m = self.solve_modes(f2)
        phi = fourier.inverse(phi_m, self.spec.n_phi)
        if return_parts:
            return phi, dict(f=f, psi=psi, sigma=sigma, theta=theta, f2=f2, phi_modes=phi_m)
        return phi


def solve(spec, rho, **kw):
    return OraclePlan(spec, **kw).solve(rho)
