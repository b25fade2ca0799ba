"""Gravitational acceleration g = -grad Phi on the cell faces -- oracle side
(test infrastructure only; nothing on the product path imports it).

The face-normal gradient is the two-point difference of Eq. gradient,
(Phi_N - Phi_i) / d_iN, with d_iN the distance between the two cell
centroids projected on the face normal.  Each directional term of the
discrete Laplacians of Sec. 2.1.1 / 2.1.2 is (A_f / Delta V) times that
quotient, which fixes the projected distances:

  spherical    r faces      r_{i+1} - r_i
               theta faces  r_i (theta_{j+1} - theta_j)
               phi faces    r_i sin(theta_j) (phi_{k+1} - phi_k)
  cylindrical  R faces      R_{i+1} - R_i
               z faces      z_{j+1} - z_j
               phi faces    R_i (phi_{k+1} - phi_k)

(cell centroids of Eqs. cell_centers_sph and the cylindrical centroids).
Readings where the paper is silent: a face on the domain boundary takes the
ghost cell's potential, which is the second solve's Dirichlet value, -Theta
(Sec. 4), transformed back to phi; a face lying on a pole has zero area and
carries g = 0.

Arrays (phi fastest, the meridional index order of the potential):
  g_a   (n_a + 1, n_b, n_phi)  face i - 1/2 at index i (radial)
  g_b   (n_a, n_b + 1, n_phi)  face j - 1/2 at index j (theta or z)
  g_phi (n_a, n_b, n_phi)      face k + 1/2 at index k (periodic)
each component along the increasing coordinate.
"""
import numpy as np

from . import fourier
from .geometry import SPH, Axis1D


def ghost_potential(spec, theta_modes):
    """Real ghost potential (n_ghost, n_phi) of the second solve: the
    inverse azimuthal transform of -Theta^m (theta_modes: (n_modes, n_ghost))."""
    x = -np.asarray(theta_modes, dtype=np.complex128)[:, :, None]
    return fourier.inverse(x, spec.n_phi)[:, 0, :]


def face_acceleration(spec, phi, ghosts, phi_ghost):
    """(g_a, g_b, g_phi) of the real potential phi (n_a, n_b, n_phi) with
    the ghost potential phi_ghost (n_ghost, n_phi) in the order of
    `ghosts` (a GhostSet)."""
    na, nb, nphi = spec.n_a, spec.n_b, spec.n_phi
    A = Axis1D(spec, "a", 1, na, 1)
    B = Axis1D(spec, "b", 1, nb, 1)
    a_c, b_c = A.cent, B.cent              # local 0..n+1, ghosts at both ends
    ext = np.zeros((na + 2, nb + 2, nphi))
    ext[1:-1, 1:-1] = phi
    ext[ghosts.i, ghosts.j] = phi_ghost
    sph = spec.geometry == SPH
    # radial faces: between local cells f and f+1, f = 0..na
    da = a_c[1:] - a_c[:-1]
    g_a = -(ext[1:, 1:-1] - ext[:-1, 1:-1]) / da[:, None, None]
    # theta / z faces: between local cells f and f+1, f = 0..nb
    db = b_c[1:] - b_c[:-1]
    dist_b = (a_c[1:-1][:, None] * db[None, :]) if sph else np.broadcast_to(db[None, :], (na, nb + 1))
    g_b = -(ext[1:-1, 1:] - ext[1:-1, :-1]) / dist_b[:, :, None]
    if B.pole_lo:
        g_b[:, 0] = 0.0
    if B.pole_hi:
        g_b[:, nb] = 0.0
    # azimuthal faces: between k and k+1 (periodic), uniform phi centroids
    metric = a_c[1:-1][:, None] * (np.sin(b_c[1:-1])[None, :] if sph else np.ones((1, nb)))
    g_phi = -(np.roll(phi, -1, axis=2) - phi) / (metric[:, :, None] * spec.dphi)
    return g_a, g_b, g_phi

