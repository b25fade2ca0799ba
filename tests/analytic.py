"""Closed-form potentials and 1D model problems used to pin the oracle.

Sources: the uniform-sphere potential of the double-sphere test (Sec. 6.1.1),
the radial shell and polar problems of Appendix A.6, and the potential of the
compact smooth sphere rho0 (1 - d^2/a^2)^3 (derived here from Gauss's law:
Phi(d) = -G M(<d)/d - 4 pi G int_d^a rho(s) s ds).
"""
import math

import numpy as np

from workloads.densities import point_cartesian, to_cartesian


def distance(geometry, a, b, phi, centre):
    x, y, z = to_cartesian(geometry, a, b, phi)
    cx, cy, cz = point_cartesian(geometry, *centre)
    return np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)


def uniform_sphere_potential(d, radius, mass, G=1.0):
    """Sec. 6.1.1: -G M (3a^2 - d^2)/(2 a^3) inside, -G M / d outside."""
    return np.where(d < radius, -G * mass * (3 * radius**2 - d**2) / (2 * radius**3), -G * mass / np.maximum(d, 1e-300))


def smooth_sphere_potential(d, radius, rho0=1.0, G=1.0):
    a = radius
    M = 4 * math.pi * rho0 * a**3 * 16.0 / 315.0
    m_in = 4 * math.pi * rho0 * (d**3 / 3 - 3 * d**5 / (5 * a**2) + 3 * d**7 / (7 * a**4) - d**9 / (9 * a**6))
    outer = rho0 * (a**2 / 8 - d**2 / 2 + 3 * d**4 / (4 * a**2) - d**6 / (2 * a**4) + d**8 / (8 * a**6))
    inner = -G * m_in / np.maximum(d, 1e-300) - 4 * math.pi * G * outer
    return np.where(d < a, inner, -G * M / np.maximum(d, 1e-300))


def shell_potential(r, R1, R2):
    """Appendix A.6 radial problem: (1/r^2)(r^2 u')' = 4 pi rho, rho = 1 on
    [R1, R2]."""
    r = np.asarray(r, dtype=np.float64)
    inside = -2 * math.pi * (R2**2 - R1**2) * np.ones_like(r)
    mid = -(2 * math.pi / (3 * r)) * (3 * R2**2 * r - 2 * R1**3 - r**3)
    out = -(4 * math.pi / (3 * r)) * (R2**3 - R1**3)
    return np.where(r < R1, inside, np.where(r <= R2, mid, out))


def polar_source(theta):
    """Appendix A.6 polar problem: f with solution u = sin 2 theta."""
    return (2 * np.cos(theta) * np.cos(2 * theta) - 4 * np.sin(theta) * np.sin(2 * theta)) / np.sin(theta)
