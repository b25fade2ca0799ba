"""Pins of the face acceleration oracle (oracle/acceleration.py) against
what the paper and the mathematics fix:

* closed forms of the two-point difference quotient for potentials whose
  discrete gradient is known exactly (linear fields, the field of a point
  mass, a uniform field in spherical and cylindrical coordinates), on
  interior and boundary faces;
* the finite-volume identity of Eq. poisson_finite_vol: the divergence of
  the face field, built from the face areas and cell volumes of Eqs.
  surface_sph / vol_sph (surface_cyl / vol_cyl), is minus the discrete
  Laplacian that the (separately pinned) per-mode operator applies, ghost
  couplings included -- a wrong distance, sign or index in any direction
  breaks it;
* zero on faces lying on a pole.
"""
import math

import numpy as np
import pytest

from oracle import acceleration as acc
from oracle import fourier
from oracle.geometry import Axis1D, GridSpec, cell_centres
from oracle.james import GhostSet, boundary_ghost_values
from oracle.operator import main_operator

CYL = GridSpec("cylindrical", "uniform", 10, 8, 12, 0.2, 2.0, -0.5, 0.5)
CYL_LOG = GridSpec("cylindrical", "log", 12, 6, 8, 0.05, 5.0, -2.5, 2.5)
SPH = GridSpec("spherical", "log", 12, 10, 8, 0.05, 5.0, 0.0, math.pi)
SPH_PART = GridSpec("spherical", "uniform", 8, 12, 6, 1.9, 3.5, 0.34 * math.pi, 0.66 * math.pi)


def _centroids(spec):
    A = Axis1D(spec, "a", 1, spec.n_a, 1)
    B = Axis1D(spec, "b", 1, spec.n_b, 1)
    return A.cent, B.cent


def _field(spec, fn):
    """fn(a, b, phi) at cell centroids and at the ghost centroids."""
    a, b, p = cell_centres(spec)
    gh = GhostSet(spec)
    A, B = np.meshgrid(a, b, indexing="ij")
    phi = fn(A[:, :, None], B[:, :, None], p[None, None, :])
    pg = fn(gh.a[:, None], gh.b[:, None], p[None, :])
    return phi, gh, pg


@pytest.mark.parametrize("spec", [CYL, CYL_LOG], ids=["cyl-uni", "cyl-log"])
def test_linear_field_cylindrical(spec):
    phi, gh, pg = _field(spec, lambda R, z, p: 0.7 * R - 1.3 * z + 0.0 * p)
    g_a, g_b, g_phi = acc.face_acceleration(spec, phi, gh, pg)
    assert np.allclose(g_a, -0.7, rtol=0, atol=1e-12)
    assert np.allclose(g_b, 1.3, rtol=0, atol=1e-12)
    assert np.allclose(g_phi, 0.0, atol=1e-12)


def test_uniform_x_field_cylindrical():
    spec = CYL
    phi, gh, pg = _field(spec, lambda R, z, p: R * np.cos(p) + 0.0 * z)
    g_a, g_b, g_phi = acc.face_acceleration(spec, phi, gh, pg)
    _, _, p = cell_centres(spec)
    dphi = spec.dphi
    assert np.allclose(g_a, -np.cos(p)[None, None, :], atol=1e-12)
    assert np.allclose(g_b, 0.0, atol=1e-12)
    # -(cos(p + dphi) - cos p) / dphi = sin(p + dphi/2) sin(dphi/2) / (dphi/2)
    exact = np.sin(p + 0.5 * dphi) * np.sin(0.5 * dphi) / (0.5 * dphi)
    assert np.allclose(g_phi, exact[None, None, :], atol=1e-12)


def test_point_mass_spherical():
    spec = SPH
    phi, gh, pg = _field(spec, lambda r, t, p: -1.0 / r + 0.0 * t + 0.0 * p)
    g_a, g_b, g_phi = acc.face_acceleration(spec, phi, gh, pg)
    a_c, _ = _centroids(spec)
    exact = -1.0 / (a_c[:-1] * a_c[1:])        # -(1/r_i - 1/r_{i+1}) / (r_{i+1} - r_i)
    assert np.allclose(g_a, exact[:, None, None], rtol=1e-12, atol=0)
    assert np.allclose(g_b, 0.0, atol=1e-12) and np.allclose(g_phi, 0.0, atol=1e-12)


@pytest.mark.parametrize("spec", [SPH, SPH_PART], ids=["sph-poles", "sph-part"])
def test_uniform_z_field_spherical(spec):
    phi, gh, pg = _field(spec, lambda r, t, p: r * np.cos(t) + 0.0 * p)
    g_a, g_b, g_phi = acc.face_acceleration(spec, phi, gh, pg)
    a_c, b_c = _centroids(spec)
    assert np.allclose(g_a, -np.cos(b_c[1:-1])[None, :, None], atol=1e-12)
    # -(r_i cos t_{j+1} - r_i cos t_j) / (r_i (t_{j+1} - t_j))
    exact = (np.cos(b_c[:-1]) - np.cos(b_c[1:])) / (b_c[1:] - b_c[:-1])
    if spec.pole_lo():
        exact[0] = 0.0
    if spec.pole_hi():
        exact[-1] = 0.0
    assert np.allclose(g_b, exact[None, :, None], atol=1e-12)
    assert np.allclose(g_phi, 0.0, atol=1e-12)


def _areas(spec):
    """Face areas (Eqs. surface_sph / surface_cyl) of one phi cell and the
    cell volumes (Eqs. vol_sph / vol_cyl)."""
    na, nb = spec.n_a, spec.n_b
    A = Axis1D(spec, "a", 1, na, 1)
    B = Axis1D(spec, "b", 1, nb, 1)
    ra, tb = A.faces[1:na + 2], B.faces[1:nb + 2]
    rlo, rhi, blo, bhi = ra[:-1], ra[1:], tb[:-1], tb[1:]
    dphi = spec.dphi
    if spec.geometry == "spherical":
        sinf = np.where((tb == 0.0) | (tb == math.pi), 0.0, np.sin(tb))
        A_a = ra[:, None] ** 2 * (np.cos(blo) - np.cos(bhi))[None, :] * dphi
        A_b = 0.5 * (rhi**2 - rlo**2)[:, None] * sinf[None, :] * dphi
        A_p = 0.5 * (rhi**2 - rlo**2)[:, None] * (bhi - blo)[None, :]
        dV = (rhi**3 - rlo**3)[:, None] / 3.0 * (np.cos(blo) - np.cos(bhi))[None, :] * dphi
    else:
        # cells indexed (R, phi, z) in the paper: phi faces Delta R Delta z,
        # z faces (R+^2 - R-^2) Delta phi / 2
        A_a = ra[:, None] * dphi * (bhi - blo)[None, :]
        A_b = np.broadcast_to(0.5 * (rhi**2 - rlo**2)[:, None] * dphi, (na, nb + 1))
        A_p = (rhi - rlo)[:, None] * (bhi - blo)[None, :]
        dV = 0.5 * (rhi**2 - rlo**2)[:, None] * dphi * (bhi - blo)[None, :]
    return A_a, A_b, A_p, dV


@pytest.mark.parametrize("spec", [CYL, CYL_LOG, SPH, SPH_PART], ids=["cyl-uni", "cyl-log", "sph-log", "sph-part"])
def test_divergence_is_minus_operator(spec):
    rng = np.random.default_rng(11)
    gh = GhostSet(spec)
    phi = rng.standard_normal((spec.n_a, spec.n_b, spec.n_phi))
    pg = rng.standard_normal((gh.n, spec.n_phi))
    g_a, g_b, g_p = acc.face_acceleration(spec, phi, gh, pg)
    A_a, A_b, A_p, dV = _areas(spec)
    div = (A_a[1:, :, None] * g_a[1:] - A_a[:-1, :, None] * g_a[:-1]
           + A_b[:, 1:, None] * g_b[:, 1:] - A_b[:, :-1, None] * g_b[:, :-1]
           + A_p[:, :, None] * (g_p - np.roll(g_p, 1, axis=2))) / dV[:, :, None]
    op = main_operator(spec, 0)
    modes = fourier.forward(phi)
    gmodes = np.moveaxis(np.fft.rfft(pg, axis=-1) / spec.n_phi, -1, 0)   # (n_modes, n_ghost)
    lap = np.empty_like(modes)
    for m in range(spec.n_modes):
        lap[m] = op.apply(modes[m], m) - op.dirichlet_rhs(boundary_ghost_values(spec, gh, gmodes[m]))
    ref = fourier.inverse(lap, spec.n_phi)
    assert np.abs(-div - ref).max() < 1e-10 * np.abs(ref).max()


def test_ghost_potential_is_inverse_transform_of_minus_theta():
    spec = SPH
    rng = np.random.default_rng(3)
    n_g = 20
    th = rng.standard_normal((spec.n_modes, n_g)) + 1j * rng.standard_normal((spec.n_modes, n_g))
    th[0].imag = 0.0
    th[-1].imag = 0.0
    out = acc.ghost_potential(spec, th)
    for g in range(n_g):
        assert np.allclose(out[g], -fourier.inverse_plain(th[:, g], spec.n_phi), atol=1e-12)
