"""The mesh-segment test configurations (Sec. 6.1.2, Table of source and
domain parameters): a uniform-density segment of a spherical or cylindrical
grid, aligned with the grid's faces, on N x N x 2N (spherical r, theta,
phi) or N x 2N x N (cylindrical R, phi, z) cells.  Grid and source
parameters only; no solver arithmetic."""
import math

PI = math.pi
S2 = math.sqrt(2.0)

# name: (geometry, radial, source (a1, a2, b1, b2, phi1, phi2), domain (a_min, a_max, b_min, b_max))
CONFIGS = {
    "sph-log": ("spherical", "log", (S2, 2 * S2, 0.38 * PI, 0.54 * PI, 0.0, 0.25 * PI), (1.0, 4.0, 0.34 * PI, 0.66 * PI)),
    "cyl-log": ("cylindrical", "log", (S2, 2 * S2, -0.9375, 0.9375, 0.0, 0.25 * PI), (1.0, 4.0, -1.5, 1.5)),
    "sph-uni": ("spherical", "uniform", (2.1, 3.2, 0.38 * PI, 0.54 * PI, 0.0, 0.25 * PI), (1.9, 3.5, 0.34 * PI, 0.66 * PI)),
    "cyl-uni": ("cylindrical", "uniform", (2.1, 3.2, -0.6, 0.6, 0.0, 0.25 * PI), (1.9, 3.5, -1.2, 1.2)),
}


def grid(name, N):
    """GridSpec keyword arguments of configuration `name` at resolution N
    (n_a = N radial cells, n_b = N polar or vertical cells, n_phi = 2N)."""
    geometry, radial, _, (a0, a1, b0, b1) = CONFIGS[name]
    return dict(geometry=geometry, radial=radial, n_a=N, n_b=N, n_phi=2 * N, a_min=a0, a_max=a1, b_min=b0, b_max=b1)


def source(name):
    return CONFIGS[name][2]
