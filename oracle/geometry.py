"""Finite-volume geometry of spherical (r, theta, phi) and cylindrical
(R, phi, z) grids -- oracle side (test infrastructure only).

Follows Sec. 2.1.1 (Eqs. cell_centers_sph, vol_sph, surface_sph and the
discrete spherical Laplacian with its factors R_i, T_j) and Sec. 2.1.2 (the
cylindrical centroid, volume, areas and W_i).  The meridional plane of a mode
is indexed (a, b): a = r or R (radial), b = theta (spherical) or z
(cylindrical).

Readings where the paper is silent:
* Log radial faces are geometric, face(f) = a_min * (a_max/a_min)**(f/N).
* Ghost cells continue the face law of their level; a ghost across a pole is
  the mirror cell (Eq. geomtric), so its centroid is -theta_1 or
  2*pi - theta_N.
* A face lying on a pole has sin(theta) = 0 exactly (zero area).
* Level l of the multigrid hierarchy uses every 2**l-th fine face.
"""
import math
from dataclasses import dataclass

import numpy as np

SPH = "spherical"
CYL = "cylindrical"
UNIFORM = "uniform"
LOG = "log"


@dataclass(frozen=True)
class GridSpec:
    """Problem grid: n_a radial cells in [a_min, a_max], n_b polar (theta)
    or vertical (z) cells in [b_min, b_max], n_phi azimuthal cells over
    [0, 2 pi)."""
    geometry: str
    radial: str
    n_a: int
    n_b: int
    n_phi: int
    a_min: float
    a_max: float
    b_min: float
    b_max: float
    G: float = 1.0

    @property
    def n_modes(self):
        return self.n_phi // 2 + 1

    @property
    def dphi(self):
        return 2.0 * math.pi / self.n_phi

    def pole_lo(self):
        return self.geometry == SPH and self.b_min == 0.0

    def pole_hi(self):
        return self.geometry == SPH and abs(self.b_max - math.pi) < 1e-12


def radial_face(spec, f):
    """Radial face coordinate at integer fine face index f (face 0 = a_min,
    face n_a = a_max); any integer is allowed (ghost/extended cells)."""
    f = np.asarray(f, dtype=np.float64)
    if spec.radial == UNIFORM:
        return spec.a_min + f * ((spec.a_max - spec.a_min) / spec.n_a)
    return spec.a_min * np.power(spec.a_max / spec.a_min, f / spec.n_a)


def b_face(spec, f):
    """theta or z face coordinate at integer fine face index f (uniform).
    Faces that sit on a pole are returned as exactly 0 or pi."""
    f = np.asarray(f, dtype=np.float64)
    out = spec.b_min + f * ((spec.b_max - spec.b_min) / spec.n_b)
    if spec.pole_hi():
        out = np.where(f == spec.n_b, math.pi, out)
    if spec.pole_lo():
        out = np.where(f == 0, 0.0, out)
    return out


def _is_pole_face(spec, theta):
    return spec.geometry == SPH and (theta == 0.0 or theta == math.pi)


def _sin_face(spec, theta):
    s = np.sin(theta)
    if spec.geometry == SPH:
        s = np.where((theta == 0.0) | (theta == math.pi), 0.0, s)
    return s


def centroid_a(geometry, lo, hi):
    """Volume-weighted radial centroid of [lo, hi] (Eq. cell_centers_sph,
    cylindrical R_i of Sec. 2.1.2)."""
    if geometry == SPH:
        return 0.75 * (hi**4 - lo**4) / (hi**3 - lo**3)
    return (2.0 / 3.0) * (hi**3 - lo**3) / (hi**2 - lo**2)


def centroid_b(geometry, lo, hi):
    """theta centroid weighted by sin(theta) (Eq. cell_centers_sph) or the
    z midpoint."""
    if geometry == SPH:
        return (np.sin(hi) - np.sin(lo) + lo * np.cos(lo) - hi * np.cos(hi)) / (np.cos(lo) - np.cos(hi))
    return 0.5 * (lo + hi)


def volume_a(geometry, lo, hi):
    """Radial factor of the cell volume (Eq. vol_sph / vol_cyl)."""
    if geometry == SPH:
        return (hi**3 - lo**3) / 3.0
    return 0.5 * (hi**2 - lo**2)


def volume_b(geometry, lo, hi):
    """theta (cos lo - cos hi) or z (hi - lo) factor of the cell volume."""
    if geometry == SPH:
        return np.cos(lo) - np.cos(hi)
    return hi - lo


class Axis1D:
    """One coordinate axis of one level: interior cells with global coarse
    index I in [lo, hi] (stride s fine cells each) plus one ghost each side.

    Arrays use local index k = 0 (lower ghost), 1..n (interior), n+1 (upper
    ghost); faces[k] is the lower face of local cell k, faces[k+1] its upper
    face.
    """

    def __init__(self, spec, which, lo, hi, stride):
        self.spec = spec
        self.which = which            # "a" (radial) or "b" (theta / z)
        self.n = hi - lo + 1
        self.lo, self.hi, self.stride = lo, hi, stride
        fidx = (np.arange(lo - 2, hi + 2) * stride).astype(np.float64)
        if which == "a":
            faces = radial_face(spec, fidx)
        else:
            faces = b_face(spec, fidx)
        self.faces = faces
        g = spec.geometry
        flo, fhi = faces[:-1], faces[1:]
        if which == "a":
            cent = centroid_a(g, flo, fhi)
            vol = volume_a(g, flo, fhi)
        else:
            cent = centroid_b(g, flo, fhi)
            vol = volume_b(g, flo, fhi)
        # A ghost across a pole is the mirror image of the first cell.
        self.pole_lo = which == "b" and _is_pole_face(spec, faces[1])
        self.pole_hi = which == "b" and _is_pole_face(spec, faces[-2])
        if self.pole_lo:
            cent[0] = -cent[1]
        if self.pole_hi:
            cent[-1] = 2.0 * math.pi - cent[-2]
        self.cent = cent
        self.vol = vol                 # includes the two ghosts
        self.sin_faces = _sin_face(spec, faces) if (which == "b" and g == SPH) else None

    # coupling of local cell k (any k with both neighbours defined) to k+1, k-1
    def couplings(self, k):
        k = np.asarray(k)
        g = self.spec.geometry
        lo, hi = self.faces[k], self.faces[k + 1]
        x = self.cent[k]
        xp = self.cent[np.minimum(k + 1, self.n + 1)]
        xm = self.cent[np.maximum(k - 1, 0)]
        with np.errstate(divide="ignore", invalid="ignore"):
            if self.which == "a":
                if g == SPH:
                    den = hi**3 - lo**3
                    up = 3.0 * hi**2 / (den * (xp - x))
                    dn = 3.0 * lo**2 / (den * (x - xm))
                else:
                    den = hi**2 - lo**2
                    up = 2.0 * hi / (den * (xp - x))
                    dn = 2.0 * lo / (den * (x - xm))
            else:
                if g == SPH:
                    den = np.cos(lo) - np.cos(hi)
                    up = self.sin_faces[k + 1] / (den * (xp - x))
                    dn = self.sin_faces[k] / (den * (x - xm))
                else:
                    den = hi - lo
                    up = 1.0 / (den * (xp - x))
                    dn = 1.0 / (den * (x - xm))
        return up, dn

    def interior_couplings(self):
        k = np.arange(1, self.n + 1)
        return self.couplings(k)

    def metric_R(self):
        """R_i of Eq. discrete_poisson_sph (multiplies the theta operator);
        identically 1 for the cylindrical z operator."""
        k = np.arange(1, self.n + 1)
        if self.spec.geometry == SPH:
            lo, hi = self.faces[k], self.faces[k + 1]
            return 1.5 / self.cent[k] * (hi**2 - lo**2) / (hi**3 - lo**3)
        return np.ones(self.n)

    def ghost_R(self):
        """R_i evaluated at the two radial ghost cells (not used by the
        operator; kept for completeness of the ghost geometry)."""
        if self.spec.geometry != SPH:
            return np.ones(2)
        out = []
        for k in (0, self.n + 1):
            lo, hi = self.faces[k], self.faces[k + 1]
            out.append(1.5 / self.cent[k] * (hi**2 - lo**2) / (hi**3 - lo**3))
        return np.array(out)

    def lambda_factor(self):
        """Factor of -s_m^2 in the azimuthal eigenvalue that depends on this
        axis: spherical radial R_i, spherical theta T_j (Eq. eigenv_sph),
        cylindrical radial W_i (Eq. eigenv_cyl), cylindrical z 1."""
        k = np.arange(1, self.n + 1)
        lo, hi = self.faces[k], self.faces[k + 1]
        g = self.spec.geometry
        if self.which == "a":
            if g == SPH:
                return 1.5 / self.cent[k] * (hi**2 - lo**2) / (hi**3 - lo**3)
            return 2.0 / (self.cent[k] * (hi + lo))
        if g == SPH:
            return (hi - lo) / (np.sin(self.cent[k]) * (np.cos(lo) - np.cos(hi)))
        return np.ones(self.n)


def mode_s2(n_phi, m):
    """[sin(m pi / N_phi) / (pi / N_phi)]^2 of Eqs. eigenv_sph / eigenv_cyl."""
    m = np.asarray(m, dtype=np.float64)
    return (np.sin(m * math.pi / n_phi) / (math.pi / n_phi)) ** 2


def cell_volumes_3d(spec):
    """Delta V_{i,j,k} of every interior cell as an (n_a, n_b) array (the
    same for every azimuthal cell)."""
    A = Axis1D(spec, "a", 1, spec.n_a, 1)
    B = Axis1D(spec, "b", 1, spec.n_b, 1)
    return np.outer(A.vol[1:-1], B.vol[1:-1]) * spec.dphi


def cell_centres(spec):
    """Interior centroid coordinates (a_i, b_j, phi_k) as 1D arrays."""
    A = Axis1D(spec, "a", 1, spec.n_a, 1)
    B = Axis1D(spec, "b", 1, spec.n_b, 1)
    phi = (np.arange(spec.n_phi) + 0.5) * spec.dphi
    return A.cent[1:-1].copy(), B.cent[1:-1].copy(), phi
