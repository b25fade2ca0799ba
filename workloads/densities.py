"""Seeded synthetic densities (no solver arithmetic; see package docstring).

Coordinates: spherical (r, theta, phi) or cylindrical (R, phi, z).  Every
sampler takes the 1D coordinate arrays of the cell centres (a, b, phi) -- a =
r or R, b = theta or z -- and returns an (n_a, n_b, n_phi) float64 array with
phi fastest.
"""
import math

import numpy as np

SPH = "spherical"
CYL = "cylindrical"


def to_cartesian(geometry, a, b, phi):
    """Broadcast (a, b, phi) cell-centre arrays to Cartesian x, y, z of shape
    (n_a, n_b, n_phi)."""
    A = np.asarray(a, dtype=np.float64)[:, None, None]
    B = np.asarray(b, dtype=np.float64)[None, :, None]
    P = np.asarray(phi, dtype=np.float64)[None, None, :]
    if geometry == SPH:
        x = A * np.sin(B) * np.cos(P)
        y = A * np.sin(B) * np.sin(P)
        z = A * np.cos(B) * np.ones_like(P)
    else:
        x = A * np.cos(P) * np.ones_like(B)
        y = A * np.sin(P) * np.ones_like(B)
        z = B * np.ones_like(A) * np.ones_like(P)
    return x, y, z


def point_cartesian(geometry, a, b, phi):
    """Cartesian position of one point given in the grid's coordinates."""
    if geometry == SPH:
        return (a * math.sin(b) * math.cos(phi), a * math.sin(b) * math.sin(phi), a * math.cos(b))
    return (a * math.cos(phi), a * math.sin(phi), b)


def uniform_sphere(geometry, a, b, phi, centre, radius, rho0=1.0):
    """rho0 where the cell centre lies inside the sphere, else 0.  centre is
    given in the grid's own coordinates (a, b, phi)."""
    x, y, z = to_cartesian(geometry, a, b, phi)
    cx, cy, cz = point_cartesian(geometry, *centre)
    d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
    return np.where(d2 < radius * radius, rho0, 0.0)


def plummer(geometry, a, b, phi, centre, scale, mass=1.0):
    """Plummer sphere rho = 3 M / (4 pi s^3) (1 + d^2/s^2)^(-5/2): smooth,
    with the closed-form potential -G M / sqrt(d^2 + s^2)."""
    x, y, z = to_cartesian(geometry, a, b, phi)
    cx, cy, cz = point_cartesian(geometry, *centre)
    d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
    return 3.0 * mass / (4.0 * math.pi * scale**3) * (1.0 + d2 / scale**2) ** (-2.5)


def gaussian_blobs(geometry, a, b, phi, centres, widths, amps):
    """sum_b A_b exp(-|x - c_b|^2 / (2 w_b^2)) with centres in the grid's
    coordinates."""
    x, y, z = to_cartesian(geometry, a, b, phi)
    out = np.zeros(x.shape)
    for c, w, amp in zip(centres, widths, amps):
        cx, cy, cz = point_cartesian(geometry, *c)
        d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
        out += amp * np.exp(-d2 / (2.0 * w * w))
    return out


def draw_blobs(rng, geometry, radial, a_min, a_max, b_min, b_max, n_blobs):
    """Blob parameters drawn in the order centres (u1, u2, u3 per blob),
    widths U[0.05, 0.3], amplitudes lognormal(0, 1).  Centres are uniform in
    (ln a or a, b, phi) over the domain (log or uniform radial law)."""
    u = rng.random((n_blobs, 3))
    if radial == "log":
        ac = np.exp(math.log(a_min) + u[:, 0] * (math.log(a_max) - math.log(a_min)))
    else:
        ac = a_min + u[:, 0] * (a_max - a_min)
    bc = b_min + u[:, 1] * (b_max - b_min)
    pc = u[:, 2] * 2.0 * math.pi
    widths = rng.uniform(0.05, 0.3, n_blobs)
    amps = rng.lognormal(0.0, 1.0, n_blobs)
    return [tuple(c) for c in zip(ac, bc, pc)], widths, amps


def spiral_disk(a, b, phi, scale_r=0.5, scale_h=0.05, amp=0.1, pitch=0.2):
    """Cylindrical exponential disk with a two-armed logarithmic spiral:
    exp(-R/scale_r) * N(z; 0, scale_h) * (1 + amp cos(2 phi - ln R / pitch))."""
    R = np.asarray(a, dtype=np.float64)[:, None, None]
    z = np.asarray(b, dtype=np.float64)[None, :, None]
    P = np.asarray(phi, dtype=np.float64)[None, None, :]
    vert = np.exp(-z * z / (2.0 * scale_h**2)) / (math.sqrt(2.0 * math.pi) * scale_h)
    return np.exp(-R / scale_r) * vert * (1.0 + amp * np.cos(2.0 * P - np.log(R) / pitch))


def keplerian_blobs(rng, n_blobs, a_min, a_max):
    """Initial blob set of the orbiting-snapshot workload: radii log-uniform
    in [0.2, 2] (clipped to the domain), theta = pi/2 + N(0, 0.15), phi
    uniform, widths U[0.05, 0.3], amplitudes lognormal(0, 1)."""
    lo, hi = max(0.2, a_min), min(2.0, a_max)
    r = np.exp(rng.uniform(math.log(lo), math.log(hi), n_blobs))
    th = math.pi / 2 + rng.normal(0.0, 0.15, n_blobs)
    ph0 = rng.uniform(0.0, 2.0 * math.pi, n_blobs)
    widths = rng.uniform(0.05, 0.3, n_blobs)
    amps = rng.lognormal(0.0, 1.0, n_blobs)
    return r, th, ph0, widths, amps


def keplerian_snapshot(a, b, phi, blobs, t):
    """Spherical density of the blob set at time t: blob phase advances at
    the Keplerian rate r^(-3/2) (G M_c = 1)."""
    r, th, ph0, widths, amps = blobs
    centres = [(r[i], th[i], ph0[i] + r[i] ** -1.5 * t) for i in range(len(r))]
    return gaussian_blobs(SPH, a, b, phi, centres, widths, amps)


def smooth_sphere(geometry, a, b, phi, centre, radius, rho0=1.0):
    """Compact, smooth sphere rho0 (1 - d^2/radius^2)^3 for d < radius, else
    0 (twice continuously differentiable; closed-form potential)."""
    x, y, z = to_cartesian(geometry, a, b, phi)
    cx, cy, cz = point_cartesian(geometry, *centre)
    q = ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (radius * radius)
    return np.where(q < 1.0, rho0 * (1.0 - q) ** 3, 0.0)


def keplerian_snapshot_device(a, b, phi, blobs, t, device="cuda"):
    """keplerian_snapshot evaluated with torch on `device` (same formula, for
    generating long trajectories of large grids quickly); returns a float64
    tensor of shape (n_a, n_b, n_phi)."""
    import torch
    r, th, ph0, widths, amps = blobs
    A = torch.as_tensor(np.asarray(a), dtype=torch.float64, device=device)[:, None, None]
    B = torch.as_tensor(np.asarray(b), dtype=torch.float64, device=device)[None, :, None]
    P = torch.as_tensor(np.asarray(phi), dtype=torch.float64, device=device)[None, None, :]
    x = A * torch.sin(B) * torch.cos(P)
    y = A * torch.sin(B) * torch.sin(P)
    z = (A * torch.cos(B)).expand(-1, -1, P.shape[2])
    out = torch.zeros(x.shape, dtype=torch.float64, device=device)
    for i in range(len(r)):
        cx, cy, cz = point_cartesian(SPH, r[i], th[i], ph0[i] + r[i] ** -1.5 * t)
        d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
        out += amps[i] * torch.exp(-d2 / (2.0 * widths[i] * widths[i]))
    return out
