"""Pins of the CPU oracle against what the paper and the mathematics fix
(closed forms, an independent general finite-volume assembly, brute force on
tiny inputs, invariants).  No GPU."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.sparse.linalg as spla

from oracle import fourier
from oracle.geometry import (Axis1D, GridSpec, cell_centres, cell_volumes_3d,
                             centroid_a, centroid_b, mode_s2)
from oracle.james import GhostSet, dgf_tables, kernel_mode
from oracle.multigrid import Hierarchy
from oracle.omega import omega_1d
from oracle.operator import main_operator
from oracle.solve import OraclePlan
from tests import analytic, fv3d
from workloads.densities import smooth_sphere, uniform_sphere

SPH, CYL = "spherical", "cylindrical"


def _spec(geom, rad, n_a, n_b, n_phi):
    if geom == SPH:
        lims = (0.1, 1.0, 0.0, math.pi) if rad == "uniform" else (0.05, 5.0, 0.0, math.pi)
    else:
        lims = (0.2, 2.0, -0.5, 0.5) if rad == "uniform" else (0.05, 5.0, -2.5, 2.5)
    return GridSpec(geom, rad, n_a, n_b, n_phi, *lims)


# -- geometry (Sec. 2.1) --------------------------------------------------------
@pytest.mark.parametrize("geom,rad", [(SPH, "uniform"), (SPH, "log"), (CYL, "uniform"), (CYL, "log")])
def test_volumes_sum_to_domain_volume(geom, rad):
    spec = _spec(geom, rad, 24, 12, 8)
    total = cell_volumes_3d(spec).sum() * spec.n_phi
    if geom == SPH:
        exact = 4.0 / 3.0 * math.pi * (spec.a_max**3 - spec.a_min**3)
    else:
        exact = math.pi * (spec.a_max**2 - spec.a_min**2) * (spec.b_max - spec.b_min)
    assert abs(total - exact) <= 1e-12 * exact


def test_partial_theta_volume():
    spec = GridSpec(SPH, "uniform", 16, 16, 8, 1.9, 3.5, 0.34 * math.pi, 0.66 * math.pi)
    total = cell_volumes_3d(spec).sum() * spec.n_phi
    exact = 2 * math.pi / 3 * (3.5**3 - 1.9**3) * (math.cos(0.34 * math.pi) - math.cos(0.66 * math.pi))
    assert abs(total - exact) <= 1e-12 * exact


def test_centroids_match_quadrature():
    for lo, hi in [(0.1, 0.13), (1.0, 1.5), (0.05, 0.0517)]:
        num = si.quad(lambda r: r**3, lo, hi)[0]
        den = si.quad(lambda r: r**2, lo, hi)[0]
        assert abs(centroid_a(SPH, lo, hi) - num / den) < 1e-12 * hi
        num = si.quad(lambda r: r**2, lo, hi)[0]
        den = si.quad(lambda r: r, lo, hi)[0]
        assert abs(centroid_a(CYL, lo, hi) - num / den) < 1e-12 * hi
    for lo, hi in [(0.0, 0.1), (1.2, 1.3), (math.pi - 0.2, math.pi)]:
        num = si.quad(lambda t: t * math.sin(t), lo, hi)[0]
        den = si.quad(lambda t: math.sin(t), lo, hi)[0]
        assert abs(centroid_b(SPH, lo, hi) - num / den) < 1e-11


def test_pole_ghost_is_mirror():
    spec = _spec(SPH, "uniform", 8, 8, 8)
    B = Axis1D(spec, "b", 1, 8, 1)
    assert B.cent[0] == -B.cent[1]
    assert abs(B.cent[-1] - (2 * math.pi - B.cent[-2])) < 1e-15
    assert B.sin_faces[1] == 0.0 and B.sin_faces[-2] == 0.0


def test_azimuthal_eigenvalue_closed_form():
    # the 3-point phi stencil on P^m_k = exp(2 pi i m k / N) gives -s_m^2 / dphi^2 * dphi^2 ...
    n = 24
    dphi = 2 * math.pi / n
    k = np.arange(n)
    for m in range(n // 2 + 1):
        p = np.exp(2j * math.pi * m * k / n)
        lap = (np.roll(p, -1) - 2 * p + np.roll(p, 1)) / dphi**2
        assert np.allclose(lap, -mode_s2(n, m) * p, atol=1e-10 * max(1.0, mode_s2(n, m)))


# -- per-mode operator vs the general 3D FV form (Sec. 2.1, Sec. 2.2) -------------
@pytest.mark.parametrize("geom,rad", [(SPH, "uniform"), (SPH, "log"), (CYL, "uniform"), (CYL, "log")])
def test_mode_operator_matches_general_fv_form(geom, rad):
    spec = _spec(geom, rad, 6, 4, 8)
    A3, _, _ = fv3d.assemble(spec)
    op = main_operator(spec)
    rng = np.random.default_rng(0)
    k = np.arange(spec.n_phi)
    for m in range(spec.n_modes):
        u2 = rng.standard_normal((spec.n_a, spec.n_b)) + 1j * rng.standard_normal((spec.n_a, spec.n_b))
        u3 = u2[:, :, None] * np.exp(2j * math.pi * m * k / spec.n_phi)[None, None, :]
        lhs = (A3 @ u3.ravel()).reshape(u3.shape)
        rhs = op.apply(u2, m)[:, :, None] * np.exp(2j * math.pi * m * k / spec.n_phi)[None, None, :]
        assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(lhs).max()


@pytest.mark.parametrize("geom,rad", [(SPH, "uniform"), (CYL, "log")])
def test_spectral_split_matches_3d_direct_solve(geom, rad):
    """FFT + per-mode solves + inverse FFT == one 3D sparse solve of the full
    FV system with the same Dirichlet ghost data."""
    spec = _spec(geom, rad, 8, 4, 8)
    A3, rhs_g, _ = fv3d.assemble(spec)
    rng = np.random.default_rng(1)
    rho = rng.standard_normal((spec.n_a, spec.n_b, spec.n_phi))
    gpos = fv3d.ghost_positions(spec)
    phi_k = (np.arange(spec.n_phi) + 0.5) * spec.dphi
    ghosts = {e: np.cos(2 * phi_k)[None, :] * (1 + a)[:, None] + np.sin(3 * phi_k)[None, :] * b[:, None]
              for e, (a, b) in gpos.items()}
    f3 = 4 * math.pi * spec.G * rho.ravel() + rhs_g(ghosts)
    phi3 = spla.spsolve(A3.tocsc(), f3).reshape(rho.shape)
    plan = OraclePlan(spec, dgf=np.zeros((spec.n_modes, 1, 1)))
    f = plan.source_modes(rho)
    gm = {e: fourier.forward(g[:, None, :])[:, :, 0] for e, g in ghosts.items()}
    for m in range(spec.n_modes):
        f[m] += plan.op.dirichlet_rhs({e: gm[e][m] for e in gm})
    phi_s = fourier.inverse(plan.solve_modes(f), spec.n_phi)
    assert np.abs(phi_s - phi3).max() <= 1e-11 * np.abs(phi3).max()


# -- Fourier transform (Sec. 2.2) ------------------------------------------------------
@pytest.mark.parametrize("n", [8, 12, 24, 96])
def test_dft_matches_plain_sums(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    X = fourier.forward(x[None, None, :])[:, 0, 0]
    assert np.allclose(X, fourier.forward_plain(x), atol=1e-13)
    assert np.allclose(fourier.inverse(X[:, None, None], n)[0, 0], x, atol=1e-12)
    assert np.allclose(fourier.inverse_plain(X, n), x, atol=1e-12)
    # a shift by k0 cells multiplies mode m by exp(-2 pi i m k0 / n)
    k0 = 3
    Xs = fourier.forward(np.roll(x, k0)[None, None, :])[:, 0, 0]
    m = np.arange(n // 2 + 1)
    assert np.allclose(Xs, X * np.exp(-2j * math.pi * m * k0 / n), atol=1e-13)


# -- 1D model problems of Appendix A.6 ---------------------------------------------
def _radial_1d(spec):
    A = Axis1D(spec, "a", 1, spec.n_a, 1)
    up, dn = A.interior_couplings()
    return A, up, dn


@pytest.mark.parametrize("rad", ["uniform", "log"])
def test_radial_shell_second_order(rad):
    """Appendix A.6 radial problem with a grid-aligned shell (faces 3N/4 and
    7N/8): clean second order in the volume-weighted L2 error."""
    errs = []
    for n in (64, 128, 256):
        spec = GridSpec(SPH, rad, n, 2, 4, 1e-3, 1.0, 0.0, math.pi)
        A, up, dn = _radial_1d(spec)
        R1, R2 = A.faces[1 + 3 * n // 4], A.faces[1 + 7 * n // 8]
        r = A.cent[1:-1]
        lo, hi = A.faces[1:n + 1], A.faces[2:n + 2]
        rho = ((lo >= R1 - 1e-15) & (hi <= R2 + 1e-15)).astype(float)
        diag = -(up + dn)
        T = np.diag(diag) + np.diag(up[:-1], 1) + np.diag(dn[1:], -1)
        b = 4 * math.pi * rho
        b[0] -= dn[0] * analytic.shell_potential(A.cent[0], R1, R2)
        b[-1] -= up[-1] * analytic.shell_potential(A.cent[-1], R1, R2)
        u = np.linalg.solve(T, b)
        ex = analytic.shell_potential(r, R1, R2)
        w = A.vol[1:-1]
        errs.append(math.sqrt(np.sum(((u - ex) / ex) ** 2 * w) / w.sum()))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert errs[-1] < 5e-4


def test_polar_problem_second_order():
    errs = []
    for n in (32, 64, 128):
        spec = GridSpec(SPH, "uniform", 2, n, 4, 1.0, 2.0, math.pi / 6, 5 * math.pi / 6)
        B = Axis1D(spec, "b", 1, n, 1)
        up, dn = B.interior_couplings()
        t = B.cent[1:-1]
        T = np.diag(-(up + dn)) + np.diag(up[:-1], 1) + np.diag(dn[1:], -1)
        b = analytic.polar_source(t)
        b[0] -= dn[0] * math.sin(2 * B.cent[0])
        b[-1] -= up[-1] * math.sin(2 * B.cent[-1])
        u = np.linalg.solve(T, b)
        errs.append(np.abs(u - np.sin(2 * t)).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def _sor_iterations(lower, diag, upper, b, omega, tol=1e-8, cap=20000):
    """Red-black SOR (a consistent ordering, so Young's theory and the optimal
    omega are those of lexicographic SOR) from zero to a relative residual tol."""
    n = len(diag)
    u = np.zeros(n)
    r0 = np.linalg.norm(b)
    for it in range(1, cap + 1):
        for p in (0, 1):
            s = slice(p, n, 2)
            nb = np.zeros(n)
            nb[1:] += lower[1:] * u[:-1]
            nb[:-1] += upper[:-1] * u[1:]
            u[s] = (1 - omega) * u[s] + omega * (b[s] - nb[s]) / diag[s]
        res = b - (diag * u + np.concatenate([[0], lower[1:] * u[:-1]]) + np.concatenate([upper[:-1] * u[1:], [0]]))
        if np.linalg.norm(res) <= tol * r0:
            return it
    return cap


@pytest.mark.parametrize("case", ["radial_log", "radial_uniform", "polar"])
def test_wkb_omega_near_empirical_optimum(case):
    """Appendix A.6: sweep omega over [1.6, 2.0] in 70 steps; the WKB value
    sits within a few sweep steps of the empirical optimum, and within 0.02 of
    Young's optimum computed from the exact Jacobi spectral radius."""
    n = 128
    if case == "polar":
        spec = GridSpec(SPH, "uniform", 2, n, 4, 1.0, 2.0, math.pi / 6, 5 * math.pi / 6)
        ax = Axis1D(spec, "b", 1, n, 1)
        b = analytic.polar_source(ax.cent[1:-1])
    else:
        spec = GridSpec(SPH, case.split("_")[1], n, 2, 4, 1e-3, 1.0, 0.0, math.pi)
        ax = Axis1D(spec, "a", 1, n, 1)
        b = 4 * math.pi * ((ax.cent[1:-1] > 0.3) & (ax.cent[1:-1] < 0.6))
    up, dn = ax.interior_couplings()
    diag = -(up + dn)
    lower = dn.copy(); lower[0] = 0.0
    upper = up.copy(); upper[-1] = 0.0
    w_pred = omega_1d(ax.cent, lower, upper, diag)
    grid = np.linspace(1.6, 2.0, 70, endpoint=False)
    counts = np.array([_sor_iterations(lower, diag, upper, b, w) for w in grid])
    assert abs(w_pred - grid[counts.argmin()]) < 4 * (grid[1] - grid[0])
    mj = -(np.diag(lower[1:], -1) + np.diag(upper[:-1], 1)) / diag[:, None]
    rho = np.max(np.abs(np.linalg.eigvals(mj)))
    w_young = 2.0 / (1.0 + math.sqrt(1.0 - rho * rho))
    assert abs(w_pred - w_young) < 0.02


# -- multigrid (Sec. 3) -------------------------------------------------------------
@pytest.mark.parametrize("geom,rad,n", [(SPH, "uniform", 32), (SPH, "log", 64), (CYL, "uniform", 32), (CYL, "log", 64)])
def test_multigrid_converges_to_direct_solution(geom, rad, n):
    spec = _spec(geom, rad, n, n // 2, 16)
    a, b, p = cell_centres(spec)
    cen = (0.5, 1.3, 0.4) if geom == SPH else (1.0, 0.05, 0.4)
    rho = smooth_sphere(geom, a, b, p, cen, 0.3)
    plan = OraclePlan(spec, dgf=np.zeros((spec.n_modes, 1, 1)))
    f = plan.source_modes(rho)
    exact = plan.solve_modes(f)
    u, cycles, res = Hierarchy(spec).solve(f, 1e-12)
    assert np.abs(u - exact).max() <= 1e-9 * np.abs(exact).max()
    assert np.all(res <= 1e-12 + 1e-18)
    assert cycles[0] == cycles.max()            # m = 0 is the slowest mode


def test_multigrid_mode_dependence_and_rate():
    """Appendix B: low m slowest, high m in one or two V-cycles; the m = 0
    contraction per cycle is well below one (the paper needs ~16 cycles for
    1e-8, i.e. ~0.32 per cycle)."""
    spec = _spec(SPH, "log", 128, 64, 128)
    a, b, p = cell_centres(spec)
    rho = uniform_sphere(SPH, a, b, p, (0.8, 1.4, 0.3), 0.4) + uniform_sphere(SPH, a, b, p, (1.2, 1.7, 3.0), 0.5)
    plan = OraclePlan(spec, dgf=np.zeros((spec.n_modes, 1, 1)))
    f = plan.source_modes(rho)
    h = Hierarchy(spec)
    sel = [0, 4, 16, 32, 64]
    u, cycles, _ = h.solve(f[sel], 1e-8, modes=sel)
    assert np.all(np.diff(cycles) <= 0)          # higher m never needs more cycles
    assert cycles[-1] <= 2
    assert 10 <= cycles[0] <= 25


def test_literal_restriction_reading_converges_slowly_on_log_grid():
    """The literal reading of the restriction weights (S_ij multiplying the
    fine point it is measured from) gives a much slower V-cycle on a
    logarithmic grid than the opposite-corner (bilinear) reading: over three
    times the per-cycle defect reduction factor on 128x64 (with a hierarchy
    that coarsens further, to 4x2, it diverges).  Pins the reading
    documented in the multigrid module."""
    spec = _spec(SPH, "log", 128, 64, 8)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((spec.n_a, spec.n_b)) + 0j
    ratios = {}
    for mode in ("bilinear", "literal"):
        h = Hierarchy(spec, restriction=mode)
        u = np.zeros_like(f)
        h.vcycle(u, f, 0)
        d1 = h.defect_norm(u, f, 0)
        for _ in range(4):
            h.vcycle(u, f, 0)
        ratios[mode] = (h.defect_norm(u, f, 0) / d1) ** 0.25
    assert ratios["bilinear"] < 0.25
    assert ratios["literal"] > 3.0 * ratios["bilinear"]


# -- James boundary and the full pipeline (Secs. 4, 5.1) -------------------------------
def _error(spec, phi, ex):
    w = cell_volumes_3d(spec)[:, :, None] * np.ones(spec.n_phi)
    return math.sqrt(np.sum(((phi - ex) / ex) ** 2 * w) / np.sum(w)), np.abs((phi - ex) / ex).max()


@pytest.mark.parametrize("geom,rad,cen,radius", [
    (SPH, "uniform", (0.5, 1.3, 0.4), 0.3),
    (SPH, "log", (1.0, 1.3, 0.4), 0.8),
    (CYL, "uniform", (1.0, 0.05, 0.4), 0.4),
    (CYL, "log", (1.0, 0.5, 0.3), 0.8),
])
def test_smooth_sphere_second_order(geom, rad, cen, radius):
    """Closed-form potential of a compact smooth sphere: error falls ~4x per
    doubling (Sec. 6.1.3) and is small at N = 64."""
    errs = []
    for n in (32, 64):
        spec = _spec(geom, rad, n, n // 2, n)
        a, b, p = cell_centres(spec)
        rho = smooth_sphere(geom, a, b, p, cen, radius)
        phi = OraclePlan(spec, n_pad=16).solve(rho)
        d = analytic.distance(geom, a, b, p, cen)
        errs.append(_error(spec, phi, analytic.smooth_sphere_potential(d, radius)))
    assert errs[0][0] / errs[1][0] > 3.0
    assert errs[1][0] < 2e-3 and errs[1][1] < 1.5e-2


def test_uniform_sphere_potential_small_grid():
    """Sec. 6.1.1 closed form on the 32x16x32 spherical grid (r in [0.1, 1],
    full theta) with a sphere of radius 0.3 at (0.5, pi/2, 0)."""
    spec = GridSpec(SPH, "uniform", 32, 16, 32, 0.1, 1.0, 0.0, math.pi)
    a, b, p = cell_centres(spec)
    cen = (0.5, math.pi / 2, 0.0)
    rho = uniform_sphere(SPH, a, b, p, cen, 0.3)
    phi = OraclePlan(spec).solve(rho)
    d = analytic.distance(SPH, a, b, p, cen)
    l2, mx = _error(spec, phi, analytic.uniform_sphere_potential(d, 0.3, 4.0 / 3.0 * math.pi * 0.3**3))
    assert l2 < 3e-2 and mx < 8e-2


def test_pipeline_satisfies_3d_fv_equations():
    """The returned Phi with ghost values -Theta (transformed back to real
    space) solves the 3D FV system of the general form to rounding."""
    spec = _spec(SPH, "log", 16, 8, 8)
    a, b, p = cell_centres(spec)
    rng = np.random.default_rng(5)
    rho = smooth_sphere(SPH, a, b, p, (1.0, 1.3, 0.4), 0.8) + 0.1 * rng.random((16, 8, 8))
    plan = OraclePlan(spec, n_pad=8)
    phi, parts = plan.solve(rho, return_parts=True)
    gh = plan.ghosts
    ghost_modes = -parts["theta"]                  # (M, n_ghost)
    real = fourier.inverse(ghost_modes.T[:, None, :].transpose(2, 0, 1), spec.n_phi)[:, 0, :]
    ghosts = {}
    for e in ("a_lo", "a_hi", "b_lo", "b_hi"):
        sel = gh.edge == e
        if np.any(sel):
            ghosts[e] = real[sel]
    A3, rhs_g, _ = fv3d.assemble(spec)
    res = A3 @ phi.ravel() - (4 * math.pi * rho.ravel() + rhs_g(ghosts))
    assert np.abs(res).max() <= 1e-10 * np.abs(4 * math.pi * rho).max()


def test_boundary_independence():
    """Vacuum boundaries: enlarging the domain around the same density must
    not change the potential beyond the DGF truncation error."""
    small = GridSpec(CYL, "uniform", 16, 16, 16, 0.5, 1.3, -0.4, 0.4)
    big = GridSpec(CYL, "uniform", 32, 32, 16, 0.1, 1.7, -0.8, 0.8)
    out = []
    for spec in (small, big):
        a, b, p = cell_centres(spec)
        rho = smooth_sphere(CYL, a, b, p, (0.9, 0.0, 1.0), 0.3)
        out.append((a, b, OraclePlan(spec).solve(rho)))
    (a0, b0, phi0), (a1, b1, phi1) = out
    i0 = np.searchsorted(np.round(a1, 12), np.round(a0, 12))
    j0 = np.searchsorted(np.round(b1, 12), np.round(b0, 12))
    assert np.allclose(a1[i0], a0) and np.allclose(b1[j0], b0)
    sub = phi1[np.ix_(i0, j0, np.arange(16))]
    assert np.abs(sub - phi0).max() <= 2e-3 * np.abs(phi0).max()


def test_invariants_shift_linearity_symmetry():
    spec = _spec(SPH, "uniform", 16, 8, 16)
    a, b, p = cell_centres(spec)
    plan = OraclePlan(spec, n_pad=8)
    rng = np.random.default_rng(7)
    r1 = smooth_sphere(SPH, a, b, p, (0.5, 1.2, 0.5), 0.3)
    r2 = rng.random(r1.shape)
    p1, p2 = plan.solve(r1), plan.solve(r2)
    assert np.abs(plan.solve(2.0 * r1 - 3.0 * r2) - (2.0 * p1 - 3.0 * p2)).max() <= 1e-12 * np.abs(p2).max() * 5
    assert np.abs(plan.solve(np.roll(r1, 5, axis=2)) - np.roll(p1, 5, axis=2)).max() <= 1e-13 * np.abs(p1).max()
    mirror = plan.solve(r1[:, ::-1, :])            # theta -> pi - theta
    assert np.abs(mirror - p1[:, ::-1, :]).max() <= 1e-12 * np.abs(p1).max()
    axi = plan.solve(np.repeat(r1[:, :, :1], spec.n_phi, axis=2))
    assert np.abs(axi - axi[:, :, :1]).max() <= 1e-13 * np.abs(axi).max()


def test_dgf_aux_and_extended_agree():
    """Two of the paper's DGF constructions on one grid (auxiliary grid and
    extended domain) agree to the truncation accuracy, and both approach the
    continuous kernel away from the source."""
    spec = GridSpec(CYL, "uniform", 16, 8, 16, 0.5, 2.0, -0.5, 0.5)
    aux = dgf_tables(spec, n_pad=8, method="aux", modes=[0, 3])
    ext = dgf_tables(spec, n_pad=12, method="extended", modes=[0, 3])
    assert np.abs(aux - ext).max() <= 6e-3 * np.abs(ext).max(), "aux and extended DGF disagree"
    gh = GhostSet(spec)
    s = 0
    far = np.abs(gh.a - gh.a[s]) + np.abs(gh.b - gh.b[s]) > 0.8
    # m = 0: the discrete and continuous kernels agree away from the source
    # (for m comparable to N_phi they differ by the discrete eigenvalue).
    k = gh.dv3[s] * kernel_mode(spec, 0, gh.a[far], gh.b[far], gh.a[s], gh.b[s])
    assert np.abs(ext[0, far, s] - k).max() <= 2e-2 * np.abs(k).max(), "far-field DGF"


def test_thomas_matches_dense_solve():
    from oracle.multigrid import thomas
    rng = np.random.default_rng(11)
    n, k = 17, 5
    lo, up = rng.random((n, k)), rng.random((n, k))
    dg = -(lo + up) - 0.1 - rng.random((n, k))
    rhs = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    x = thomas(lo, dg, up, rhs)
    for c in range(k):
        A = np.diag(dg[:, c]) + np.diag(lo[1:, c], -1) + np.diag(up[:-1, c], 1)
        assert np.allclose(A @ x[:, c], rhs[:, c], atol=1e-13)


def test_exact_line_relaxation_handles_strong_anisotropy():
    """Cylindrical log grid reaching R = 3e-3 (cell aspect ratio ~1e3): the
    two-pass SOR line smoother stalls, exact line relaxation (the ideal of
    Sec. 3.2) keeps the V-cycle contracting."""
    spec = GridSpec(CYL, "log", 80, 24, 12, 0.00315, 31.5, -5.0, 5.0)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((spec.n_a, spec.n_b)) + 0j
    rates = {}
    for ls in ("sor", "exact"):
        h = Hierarchy(spec, line_solver=ls)
        u = np.zeros_like(f)
        for _ in range(4):
            h.vcycle(u, f, 0)
        d1 = h.defect_norm(u, f, 0)
        for _ in range(4):
            h.vcycle(u, f, 0)
        rates[ls] = (h.defect_norm(u, f, 0) / d1) ** 0.25
    assert rates["sor"] > 0.8
    assert rates["exact"] < 0.25


# -- pins of the gravitational constant, the DGF, the ghost potential, the
#    transfers and the 2D omega --------------------------------------------------
def _ghost_xyz(geom, a, b, phi):
    A, B, P = np.asarray(a)[:, None], np.asarray(b)[:, None], np.asarray(phi)[None, :]
    if geom == SPH:
        return A * np.sin(B) * np.cos(P), A * np.sin(B) * np.sin(P), A * np.cos(B) * np.ones_like(P)
    return A * np.cos(P) * np.ones_like(B), A * np.sin(P) * np.ones_like(B), B * np.ones_like(P)


@pytest.mark.parametrize("geom,rad,cen,radius", [
    (SPH, "log", (1.0, 1.3, 0.4), 0.8),
    (CYL, "uniform", (1.0, 0.05, 0.4), 0.4),
])
def test_gravitational_constant_enters_every_step(geom, rad, cen, radius):
    """G = 0.5 against the closed form with G explicit (Sec. 6.1.1 form of the
    smooth sphere, Gauss's law).  G enters the source (4 pi G rho, Eq.
    poisson_discrete), the screening mass (1/(4 pi G), Eqs. charge_sph/cyl)
    and the DGF (4 pi G delta and the -G kernel of Eqs. DGF_bc_sph/cyl): a
    factor dropped or doubled in any one of them breaks Phi(G) = G Phi(1)
    (the boundary term then scales with another power of G) and moves the
    result off the closed form by far more than the truncation error."""
    errs = []
    for n in (16, 32):
        spec1 = _spec(geom, rad, n, n // 2, n)
        spec = GridSpec(*[getattr(spec1, k) for k in ("geometry", "radial", "n_a", "n_b", "n_phi",
                                                       "a_min", "a_max", "b_min", "b_max")], G=0.5)
        a, b, p = cell_centres(spec)
        rho = smooth_sphere(geom, a, b, p, cen, radius)
        npad = 8 if n == 16 else 16
        phi_half = OraclePlan(spec, n_pad=npad).solve(rho)
        phi_one = OraclePlan(spec1, n_pad=npad).solve(rho)
        assert np.abs(phi_half - 0.5 * phi_one).max() <= 1e-12 * np.abs(phi_one).max()
        d = analytic.distance(geom, a, b, p, cen)
        errs.append(_error(spec, phi_half, analytic.smooth_sphere_potential(d, radius, G=0.5)))
    assert errs[0][0] / errs[1][0] > 3.0, errs
    assert errs[1][0] < 1e-2, errs


@pytest.mark.parametrize("geom,rad", [(SPH, "log"), (CYL, "log"), (CYL, "uniform")])
def test_dgf_source_part_exactly_reciprocal(geom, rad):
    """Without the box boundary data the extended-domain table is the
    volume-weighted inverse of the symmetric finite-volume operator times
    4 pi G, so Gt(t <- s) / dV_s = Gt(s <- t) / dV_t to rounding (Sec. 4.2,
    with Gt = G^m dV_s of Eq. Theta_fft).  A wrong source normalisation (2D
    instead of 3D volume, the field cell's volume instead of the source's)
    or an unsymmetric coupling breaks it."""
    spec = _spec(geom, rad, 16, 8, 8)
    gh = GhostSet(spec)
    T = dgf_tables(spec, n_pad=8, method="extended", modes=[0, 1, 4], homogeneous=True)
    S = T / gh.dv3[None, None, :]
    assert np.abs(S - S.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(S).max()
    # and the inverse itself: applying the box operator to a column gives
    # 4 pi G at the source (checked through the ghost rows: positive-definite
    # sign of the self term of an attractive potential)
    assert np.all(np.diagonal(T, axis1=1, axis2=2) < 0.0)


def test_dgf_reciprocity_improves_under_refinement():
    """The full tables carry boundary data from the continuous kernel, which
    is reciprocal itself, so the discrete reciprocity defect falls as the
    grid is refined (log sphere: about 8x per doubling; log cylinder:
    about 2x)."""
    defects = {SPH: [], CYL: []}
    for n in (16, 32):
        for geom in (SPH, CYL):
            spec = _spec(geom, "log", n, n // 2, 8)
            gh = GhostSet(spec)
            T = dgf_tables(spec, n_pad=n // 2, method="extended", modes=[0, 2])
            S = T / gh.dv3[None, None, :]
            defects[geom].append(np.abs(S - S.transpose(0, 2, 1)).max() / np.abs(S).max())
    assert defects[SPH][1] < defects[SPH][0] / 4 and defects[SPH][1] < 1e-5, defects
    assert defects[CYL][1] < defects[CYL][0] / 1.5 and defects[CYL][1] < 1e-2, defects


@pytest.mark.parametrize("geom,rad,cen,radius", [
    (SPH, "uniform", (0.5, 1.3, 0.4), 0.3),
    (SPH, "log", (1.0, 1.3, 0.4), 0.8),
    (CYL, "log", (1.0, 0.5, 0.3), 0.8),
])
def test_ghost_potential_second_order(geom, rad, cen, radius):
    """The James boundary potential: -Theta at the ghost-cell centres (back in
    real space) is the potential of the isolated density there (Sec. 4, step
    3 sets the second solve's boundary to it), so it converges to the closed
    form at second order (error / 4 per doubling, Sec. 6.1.3)."""
    errs = []
    for n in (32, 64):
        spec = _spec(geom, rad, n, n // 2, n)
        a, b, p = cell_centres(spec)
        rho = smooth_sphere(geom, a, b, p, cen, radius)
        plan = OraclePlan(spec, n_pad=16)
        _, parts = plan.solve(rho, return_parts=True)
        gh = plan.ghosts
        theta = fourier.inverse(parts["theta"][:, :, None], spec.n_phi)[:, 0, :]   # (n_ghost, n_phi)
        x, y, z = _ghost_xyz(geom, gh.a, gh.b, p)
        from workloads.densities import point_cartesian
        cx, cy, cz = point_cartesian(geom, *cen)
        d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
        ex = analytic.smooth_sphere_potential(d, radius)
        errs.append(np.abs(-theta - ex).max() / np.abs(ex).max())
    assert errs[0] / errs[1] > 3.5, errs
    assert errs[1] < 5e-3, errs


def _transfer_x(geom, which, x):
    return x * x if (which == "a" and geom == SPH) else x


@pytest.mark.parametrize("geom,rad", [(SPH, "uniform"), (SPH, "log"), (CYL, "uniform"), (CYL, "log")])
def test_transfers_reproduce_linear_fields(geom, rad):
    """Sec. 3.1: restriction and prolongation are bilinear in (r^2, theta)
    (spherical) or (R, z) (cylindrical).  Restricting a field linear in
    those coordinates gives its values at the coarse centroids exactly;
    prolonging one gives its values at the fine centroids exactly.  Where the
    stencil touches a coarse ghost: at a pole for fields even (m even) or odd
    (m odd) across it; at a Dirichlet edge for fields that vanish at the
    finest ghost centre (where the error's boundary condition sits on every
    level), on the axes whose transfer coordinate is the coordinate itself
    (theta, R, z).  The coarse ghost factor is set by a straight line in r
    and the spherical radial transfer is linear in r^2, so on that axis the
    coarse ghost is checked to lie on the line in r that vanishes at the
    finest ghost centre."""
    from oracle.multigrid import prolongation_matrix_1d, restriction_weights_1d
    if geom == SPH:
        spec = GridSpec(SPH, rad, 32, 16, 8, *((0.1, 1.0) if rad == "uniform" else (0.05, 5.0)), 0.0, math.pi)
    else:
        spec = _spec(geom, rad, 32, 16, 8)
    h = Hierarchy(spec)
    fine, coarse = h.levels[0], h.levels[1]
    rng = np.random.default_rng(4)
    for which, F, C in (("a", fine.A, coarse.A), ("b", fine.B, coarse.B)):
        xf = _transfer_x(geom, which, F.cent)
        xc = _transfer_x(geom, which, C.cent)
        c0, c1 = rng.standard_normal(2)
        w = restriction_weights_1d(F, C, geom, which)
        restricted = w[:, 0] * (c0 + c1 * xf[1:-1:2]) + w[:, 1] * (c0 + c1 * xf[2::2])
        assert np.abs(restricted - (c0 + c1 * xc[1:-1])).max() <= 1e-13 * (abs(c0) + abs(c1) * np.abs(xc).max())
        for m in (0, 1):
            k = coarse.op.kappa
            e_lo, e_hi = (("a_lo", "a_hi") if which == "a" else ("b_lo", "b_hi"))
            P = prolongation_matrix_1d(F, C, geom, which, k(e_lo, m), k(e_hi, m))
            n_f = F.n
            inner = np.arange(2, n_f - 2)
            g = c0 + c1 * xc[1:-1]
            assert np.abs((P @ g)[inner] - (c0 + c1 * xf[1:-1][inner])).max() <= 1e-12 * np.abs(g).max()
            for edge, rows, x_ghost in ((e_lo, [0, 1], F.cent[0]), (e_hi, [n_f - 2, n_f - 1], F.cent[n_f + 1])):
                kind = coarse.op.edges[edge]
                if kind == "pole":
                    if m % 2:                      # odd across the pole: c1 * theta (or pi - theta)
                        xp = 0.0 if edge.endswith("lo") else math.pi
                        g = c1 * (xc[1:-1] - xp)
                        ex = c1 * (xf[1:-1] - xp)
                    else:                          # even: constant
                        g = np.full(C.n, c0)
                        ex = np.full(n_f, c0)
                elif which == "a" and geom == SPH:
                    g = c1 * (C.cent[1:-1] - x_ghost)      # straight line in r through the finest ghost
                    lo = edge.endswith("lo")
                    ghost_val = k(edge, m) * (g[0] if lo else g[-1])
                    cg = C.cent[0] if lo else C.cent[-1]
                    assert abs(ghost_val - c1 * (cg - x_ghost)) <= 1e-12 * abs(c1) * abs(cg), edge
                    continue
                else:                              # Dirichlet: vanishes at the finest ghost centre
                    xg = _transfer_x(geom, which, np.array([x_ghost]))[0]
                    g = c1 * (xc[1:-1] - xg)
                    ex = c1 * (xf[1:-1] - xg)
                assert np.abs((P @ g)[rows] - ex[rows]).max() <= 1e-12 * np.abs(ex).max(), (edge, m)


@pytest.mark.parametrize("shift", [0.0, 37.0])
def test_omega_2d_exact_for_constant_coefficients(shift):
    """Appendix A's 2D estimate: for the constant-coefficient 5-point operator
    (optionally with a constant Helmholtz shift, as the mode term adds) the
    weighted Rayleigh quotient with the lowest sine mode is the exact Jacobi
    spectral radius, so omega_2d equals Young's optimum 2 / (1 + sqrt(1 -
    rho^2)) computed from the eigenvalues of the Jacobi matrix."""
    from oracle.omega import omega_2d
    na, nb, hx, hy = 12, 7, 0.3, 0.11
    xa, xb = hx * np.arange(na + 2), hy * np.arange(nb + 2)
    ua = np.full(na, 1 / hx**2)
    ub = np.full((na, nb), 1 / hy**2)
    diag = np.full((na, nb), -2 / hx**2 - 2 / hy**2 - shift)
    w = omega_2d(xa, xb, ua, ua.copy(), ub, ub.copy(), diag)
    n = na * nb
    J = np.zeros((n, n))
    idx = np.arange(n).reshape(na, nb)
    for i in range(na):
        for j in range(nb):
            for ii, jj, c in ((i + 1, j, ua[0]), (i - 1, j, ua[0]), (i, j + 1, ub[0, 0]), (i, j - 1, ub[0, 0])):
                if 0 <= ii < na and 0 <= jj < nb:
                    J[idx[i, j], idx[ii, jj]] = -c / diag[i, j]
    rho = np.abs(np.linalg.eigvals(J)).max()
    assert abs(w - 2.0 / (1.0 + math.sqrt(1.0 - rho * rho))) < 1e-12
