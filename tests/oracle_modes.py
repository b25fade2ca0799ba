"""The oracle's potential for sampled azimuthal modes only.

After the forward FFT every mode is an independent 2D problem (Sec. 2.2), so
Phi^m of a few modes follows from the seven steps run on those modes alone:
exact solve with zero ghosts, screening masses (Eqs. charge_sph/cyl), the
boundary convolution with the DGF table of that mode (Sec. 4.2), and the
exact solve with the ghosts at -Theta.  This keeps the oracle affordable on
grids whose full DGF tables would take long to build."""
import numpy as np

from oracle.james import boundary_ghost_values, dgf_tables, screening_mass
from oracle.solve import OraclePlan


def oracle_modes(spec, rho, modes, n_pad=16):
    """{m: Phi^m (n_a, n_b) complex} for the modes `modes` of density rho."""
    op = OraclePlan(spec, n_pad=n_pad, dgf=np.zeros((spec.n_modes, 1, 1)))
    f = op.source_modes(rho)
    gh = op.ghosts
    out = {}
    for m in modes:
        print(f"[oracle] mode {m}", flush=True)
        psi = op.lu(m).solve(f[m].real.ravel().copy()) + 1j * op.lu(m).solve(f[m].imag.ravel().copy())
        psi = psi.reshape(spec.n_a, spec.n_b)
        sigma = screening_mass(spec, gh, psi[None])[0]
        theta = dgf_tables(spec, n_pad=n_pad, modes=[m])[0] @ sigma
        f2 = f[m] + op.op.dirichlet_rhs(boundary_ghost_values(spec, gh, -theta))
        phi = op.lu(m).solve(f2.real.ravel().copy()) + 1j * op.lu(m).solve(f2.imag.ravel().copy())
        out[m] = phi.reshape(spec.n_a, spec.n_b)
    return out
