"""Pins of the mesh-segment reference potential (oracle/segment.py) against
closed forms and additivity, and of the segment densities against the
exact segment volume on the aligned grids of the mesh-segment test.  No
GPU."""
import math

import numpy as np
import pytest

from oracle.geometry import GridSpec, cell_volumes_3d, radial_face, b_face
from oracle.segment import segment_density, segment_potential
from tests import analytic
from workloads import segment as W

PTS = np.array([[0.1, 0.2, 0.3], [0.5, -0.2, 0.1], [1.5, 0.3, -0.4], [0.0, 0.0, 2.0], [-0.3, 0.95, 0.2]])


def test_uniform_sphere_and_shell_closed_forms():
    """Full-range segments: a ball of radius 0.7 (Sec. 6.1.1 closed form) and
    a shell 0.4 <= r <= 0.9 (the Appendix A radial problem's closed form)."""
    d = np.linalg.norm(PTS, axis=1)
    phi = segment_potential("spherical", (0.0, 0.7, 0.0, math.pi, 0.0, 2 * math.pi), PTS)
    ex = analytic.uniform_sphere_potential(d, 0.7, 4.0 / 3.0 * math.pi * 0.7**3)
    assert np.abs(phi - ex).max() <= 1e-12 * np.abs(ex).max()
    phi = segment_potential("spherical", (0.4, 0.9, 0.0, math.pi, 0.0, 2 * math.pi), PTS)
    ex = analytic.shell_potential(d, 0.4, 0.9)
    assert np.abs(phi - ex).max() <= 1e-12 * np.abs(ex).max()


def test_solid_cylinder_on_axis_closed_form():
    """Full-range cylindrical segment 0 <= R <= a, z1 <= z <= z2: on the axis
    Phi(z) = -2 pi G rho int_{z1}^{z2} (sqrt((z'-z)^2 + a^2) - |z'-z|) dz'."""
    a, z1, z2 = 0.8, -0.5, 0.7
    zs = np.array([-1.2, -0.3, 0.1, 0.69, 2.0])
    pts = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], axis=1)
    phi = segment_potential("cylindrical", (0.0, a, z1, z2, 0.0, 2 * math.pi), pts)
    F = lambda t: 0.5 * (t * np.sqrt(t * t + a * a) + a * a * np.arcsinh(t / a)) - 0.5 * t * np.abs(t)
    ex = -2.0 * math.pi * (F(z2 - zs) - F(z1 - zs))
    assert np.abs(phi - ex).max() <= 1e-12 * np.abs(ex).max()


@pytest.mark.parametrize("geom", ["spherical", "cylindrical"])
def test_additivity_over_adjacent_segments(geom):
    """The potential of a segment is the sum over any split of it along r/R,
    theta/z or phi (pins every kind of face and its normal's sign)."""
    if geom == "spherical":
        whole = (0.4, 1.1, 0.3, 2.2, 0.2, 4.0)
        parts = [(0.4, 0.7, 0.3, 2.2, 0.2, 4.0), (0.7, 1.1, 0.3, 1.1, 0.2, 4.0), (0.7, 1.1, 1.1, 2.2, 0.2, 1.9),
                 (0.7, 1.1, 1.1, 2.2, 1.9, 4.0)]
    else:
        whole = (0.4, 1.1, -0.6, 0.5, 0.2, 4.0)
        parts = [(0.4, 0.7, -0.6, 0.5, 0.2, 4.0), (0.7, 1.1, -0.6, 0.1, 0.2, 4.0), (0.7, 1.1, 0.1, 0.5, 0.2, 1.9),
                 (0.7, 1.1, 0.1, 0.5, 1.9, 4.0)]
    pts = np.array([[0.9, 0.1, 0.2], [0.2, 0.5, -0.1], [-1.0, 0.4, 0.6], [0.3, -0.7, 0.05]])
    w = segment_potential(geom, whole, pts)
    s = sum(segment_potential(geom, q, pts) for q in parts)
    assert np.abs(w - s).max() <= 1e-11 * np.abs(w).max()


@pytest.mark.parametrize("name", list(W.CONFIGS))
def test_segment_density_is_grid_aligned(name):
    """On the mesh-segment grids the segment's boundary lies on cell faces at
    every N of the convergence study: the cells it covers hold exactly its
    volume."""
    geom, _, seg, _ = W.CONFIGS[name]
    a1, a2, b1, b2, p1, p2 = seg
    for N in (16, 32, 64):
        spec = GridSpec(**W.grid(name, N))
        fa = radial_face(spec, np.arange(N + 1))
        fb = b_face(spec, np.arange(N + 1))
        rho = segment_density(geom, seg, fa, fb, spec.n_phi)
        mass = float(np.sum(rho * cell_volumes_3d(spec)[:, :, None]))
        if geom == "spherical":
            vol = (a2**3 - a1**3) / 3.0 * (math.cos(b1) - math.cos(b2)) * (p2 - p1)
        else:
            vol = 0.5 * (a2**2 - a1**2) * (b2 - b1) * (p2 - p1)
        assert abs(mass - vol) <= 1e-12 * vol, (name, N)
