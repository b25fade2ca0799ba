"""WKB estimate of the optimal SOR parameter (Appendix A) -- oracle side
(test infrastructure only).

For a tridiagonal line system lower_j u_{j-1} + diag_j u_j + upper_j u_{j+1}
with points x_1..x_N and Dirichlet positions x_0, x_{N+1}:

  rho_J ~ | sum_j (lower_j + upper_j) cos(pi delta_j / L) w_j / sum_j diag_j w_j |,
  w_j = sin^2(pi (x_j - x_0) / L),  delta_j = x_j - x_{j-1},  L = x_{N+1} - x_0,
  omega = 2 / (1 + sqrt(1 - rho_J^2))            (Eq. omega_opt_mu).

The two-dimensional estimate used by the coarsest-grid red-black SOR is the
p = q = 1 term of the 2D formula of Appendix A (the printed max over p, q is
garbled; the lowest mode is the one the 1D analysis keeps).
"""
import numpy as np


def jacobi_radius_1d(x, lower, upper, diag):
    """x: positions including the two end (ghost) positions, length N+2."""
    x = np.asarray(x, dtype=np.float64)
    L = x[-1] - x[0]
    xi = x[1:-1]
    delta = x[1:-1] - x[:-2]
    w = np.sin(np.pi * (xi - x[0]) / L) ** 2
    num = np.sum((np.asarray(lower) + np.asarray(upper)) * np.cos(np.pi * delta / L) * w)
    den = np.sum(np.asarray(diag) * w)
    return abs(num / den)


def omega_from_radius(rho):
    rho = min(rho, 1.0)
    return 2.0 / (1.0 + np.sqrt(max(0.0, 1.0 - rho * rho)))


def omega_1d(x, lower, upper, diag):
    return omega_from_radius(jacobi_radius_1d(x, lower, upper, diag))


def omega_2d(xa, xb, ua, da, ub, db, diag):
    """2D estimate: xa, xb include ghost positions; ua/da are (n_a,) radial
    couplings, ub/db are (n_a, n_b) polar couplings (already times R_i),
    diag is (n_a, n_b)."""
    La = xa[-1] - xa[0]
    Lb = xb[-1] - xb[0]
    da_ = xa[1:-1] - xa[:-2]
    db_ = xb[1:-1] - xb[:-2]
    wa = np.sin(np.pi * (xa[1:-1] - xa[0]) / La) ** 2
    wb = np.sin(np.pi * (xb[1:-1] - xb[0]) / Lb) ** 2
    w = wa[:, None] * wb[None, :]
    num = np.sum(((ua + da)[:, None] * np.cos(np.pi * da_ / La)[:, None]
                  + (ub + db) * np.cos(np.pi * db_ / Lb)[None, :]) * w)
    den = np.sum(diag * w)
    return omega_from_radius(abs(num / den))
