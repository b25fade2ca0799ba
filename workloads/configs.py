"""The benchmark workloads: grids and seeded synthetic densities shaped like
the paper's test problems (no solver arithmetic here).

c1  spherical uniform 32x16x32, r in [0.1, 1], full theta: uniform sphere of
    radius 0.3 at (r, theta, phi) = (0.5, pi/2, 0); rel. residual 1e-10.
c2  spherical log 128x64x128, r in [0.05, 5], full theta: 8 Gaussian blobs
    (seed 2; centres uniform in (ln r, theta, phi), widths U[0.05, 0.3],
    amplitudes lognormal(0, 1)); all 65 modes batched.
c3  cylindrical uniform N_R x N_phi x N_z = 256x256x128, R in [0.2, 2],
    z in [-0.5, 0.5]: exponential disk (scale 0.5) with Gaussian vertical
    profile (scale height 0.05) and a two-armed spiral.
c4  16 independent problems solved as one batch (seed 4): 4 each of
    {spherical, cylindrical} x {uniform, log radial}, N drawn from
    {64, 96, 128, 192}; spherical (N_r, N_theta, N_phi) = (N, N/2, N),
    cylindrical (N_R, N_z, N_phi) = (N, N/2, N); domains as c1 (spherical
    uniform), c2 (spherical log), c3 (cylindrical uniform) and R in
    [0.05, 5], z in [-2.5, 2.5] (cylindrical log); 8 Gaussian blobs each as
    c2 with per-problem seed 4000 + p.
c5  spherical log 256x128x256, r in [0.05, 5]: 12 blobs on Keplerian
    orbits; snapshot t of the sequence (seed 5).
"""
import math

import numpy as np

from . import densities as D

PI = math.pi

GRIDS = {
    "c1": dict(geometry="spherical", radial="uniform", n_a=32, n_b=16, n_phi=32, a_min=0.1, a_max=1.0,
               b_min=0.0, b_max=PI),
    "c2": dict(geometry="spherical", radial="log", n_a=128, n_b=64, n_phi=128, a_min=0.05, a_max=5.0,
               b_min=0.0, b_max=PI),
    "c3": dict(geometry="cylindrical", radial="uniform", n_a=256, n_b=128, n_phi=256, a_min=0.2, a_max=2.0,
               b_min=-0.5, b_max=0.5),
    "c5": dict(geometry="spherical", radial="log", n_a=256, n_b=128, n_phi=256, a_min=0.05, a_max=5.0,
               b_min=0.0, b_max=PI),
}

DESCRIPTION = {
    "c1": "spherical uniform 32x16x32, r in [0.1,1], uniform sphere R=0.3 at (0.5, pi/2, 0)",
    "c2": "spherical log-r 128x64x128, r in [0.05,5], 8 Gaussian blobs (seed 2), all 65 modes batched",
    "c3": "cylindrical uniform 256x256x128 (R,phi,z), R in [0.2,2], z in [-0.5,0.5], spiral exponential disk",
    "c4": "16-problem batch (seed 4): sph/cyl x uniform/log, N in {64,96,128,192}, 8 Gaussian blobs each",
    "c5": "spherical log-r 256x128x256, r in [0.05,5], 12 Keplerian Gaussian blobs (seed 5)",
}

C4_DOMAINS = {
    ("spherical", "uniform"): (0.1, 1.0, 0.0, PI),
    ("spherical", "log"): (0.05, 5.0, 0.0, PI),
    ("cylindrical", "uniform"): (0.2, 2.0, -0.5, 0.5),
    ("cylindrical", "log"): (0.05, 5.0, -2.5, 2.5),
}


def c4_grids(seed=4):
    """Grids of the 16-problem batch, in problem order."""
    rng = np.random.default_rng(seed)
    kinds = [(g, r) for g in ("spherical", "cylindrical") for r in ("uniform", "log") for _ in range(4)]
    sizes = rng.choice([64, 96, 128, 192], size=len(kinds))
    out = []
    for (geo, rad), n in zip(kinds, sizes):
        a0, a1, b0, b1 = C4_DOMAINS[(geo, rad)]
        out.append(dict(geometry=geo, radial=rad, n_a=int(n), n_b=int(n) // 2, n_phi=int(n), a_min=a0, a_max=a1,
                        b_min=b0, b_max=b1))
    return out


def c4_density(p, grid, a, b, phi):
    """Density of problem p of the batch: 8 blobs drawn as in c2 (seed 4000 + p)."""
    rng = np.random.default_rng(4000 + p)
    cen, w, amp = D.draw_blobs(rng, grid["geometry"], grid["radial"], grid["a_min"], grid["a_max"], grid["b_min"],
                               grid["b_max"], 8)
    return D.gaussian_blobs(grid["geometry"], a, b, phi, cen, w, amp)


def density(name, a, b, phi, t=0.0):
    """Density of workload `name` at cell centres (a, b, phi)."""
    g = GRIDS[name]
    if name == "c1":
        return D.uniform_sphere(g["geometry"], a, b, phi, (0.5, PI / 2, 0.0), 0.3)
    if name == "c2":
        rng = np.random.default_rng(2)
        cen, w, amp = D.draw_blobs(rng, g["geometry"], g["radial"], g["a_min"], g["a_max"], g["b_min"], g["b_max"], 8)
        return D.gaussian_blobs(g["geometry"], a, b, phi, cen, w, amp)
    if name == "c3":
        return D.spiral_disk(a, b, phi)
    if name == "c5":
        rng = np.random.default_rng(5)
        blobs = D.keplerian_blobs(rng, 12, g["a_min"], g["a_max"])
        return D.keplerian_snapshot(a, b, phi, blobs, t)
    raise KeyError(name)


def c5_blobs(seed=5, name="c5"):
    """Blob set of an orbiting trajectory (seed 5: the measured one; 50-57:
    the training trajectories of the learned guess)."""
    g = GRIDS[name]
    return D.keplerian_blobs(np.random.default_rng(seed), 12, g["a_min"], g["a_max"])


def keplerian_dt(name="c5"):
    """Snapshot cadence of the orbiting workload: the fastest blob moves half
    an azimuthal cell per step."""
    g = GRIDS[name]
    rng = np.random.default_rng(5)
    r = D.keplerian_blobs(rng, 12, g["a_min"], g["a_max"])[0]
    return 0.5 * (2 * PI / g["n_phi"]) / (r.min() ** -1.5)
