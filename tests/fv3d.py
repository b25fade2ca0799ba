"""Independent 3D assembly of the finite-volume Poisson operator from the
general face-flux form (Eq. poisson_discrete) with the face areas of Eqs.
surface_sph / surface_cyl, the volumes of Eqs. vol_sph / vol_cyl and the
normal distances between neighbouring centroids (radial: r_{i+1} - r_i;
polar: r_i (theta_{j+1} - theta_j); azimuthal: r_i sin(theta_j) dphi or
R_i dphi; vertical: z_{k+1} - z_k).  Poles have zero face area.  Used only
to pin the oracle's per-mode operator, spectral split and pipeline.

Unknown order: (i, j, k) row-major over (n_a, n_b, n_phi).  Dirichlet ghost
values are passed per edge as arrays over the edge's (other index, k).
"""
import math

import numpy as np
import scipy.sparse as sp


def _faces_and_centroids(spec):
    na, nb = spec.n_a, spec.n_b
    f = np.arange(-1, na + 2, dtype=np.float64)
    if spec.radial == "uniform":
        fa = spec.a_min + f * (spec.a_max - spec.a_min) / na
    else:
        fa = spec.a_min * (spec.a_max / spec.a_min) ** (f / na)
    g = np.arange(-1, nb + 2, dtype=np.float64)
    fb = spec.b_min + g * (spec.b_max - spec.b_min) / nb
    sph = spec.geometry == "spherical"
    pole_lo = sph and spec.b_min == 0.0
    pole_hi = sph and abs(spec.b_max - math.pi) < 1e-12
    if pole_lo:
        fb[1] = 0.0
    if pole_hi:
        fb[nb + 1] = math.pi
    lo, hi = fa[:-1], fa[1:]
    if sph:
        ca = 0.75 * (hi**4 - lo**4) / (hi**3 - lo**3)
        va = (hi**3 - lo**3) / 3.0
    else:
        ca = (2.0 / 3.0) * (hi**3 - lo**3) / (hi**2 - lo**2)
        va = 0.5 * (hi**2 - lo**2)
    lo, hi = fb[:-1], fb[1:]
    if sph:
        cb = (np.sin(hi) - np.sin(lo) + lo * np.cos(lo) - hi * np.cos(hi)) / (np.cos(lo) - np.cos(hi))
        if pole_lo:
            cb[0] = -cb[1]
        if pole_hi:
            cb[-1] = 2 * math.pi - cb[-2]
    else:
        cb = 0.5 * (lo + hi)
    return fa, fb, ca, cb, va, pole_lo, pole_hi


def assemble(spec):
    """Returns (A, rhs_from_ghosts, dv) where A is the sparse 3D operator
    (divided by volume), rhs_from_ghosts(ghosts) the right-hand-side change of
    Dirichlet ghost data and dv the (n_a, n_b) cell volumes (per phi cell)."""
    na, nb, nphi = spec.n_a, spec.n_b, spec.n_phi
    dphi = 2 * math.pi / nphi
    fa, fb, ca, cb, va, pole_lo, pole_hi = _faces_and_centroids(spec)
    sph = spec.geometry == "spherical"

    def sinf(t):
        return 0.0 if (sph and (t == 0.0 or t == math.pi)) else math.sin(t)

    N = na * nb * nphi
    idx = np.arange(N).reshape(na, nb, nphi)
    rows, cols, vals = [], [], []
    gcoef = {}          # (edge, i_or_j, ) -> coefficient of the ghost value
    dv = np.zeros((na, nb))
    for i in range(1, na + 1):
        rl, rh, r = fa[i], fa[i + 1], ca[i]
        for j in range(1, nb + 1):
            tl, th, t = fb[j], fb[j + 1], cb[j]
            if sph:
                V = (rh**3 - rl**3) / 3.0 * (math.cos(tl) - math.cos(th)) * dphi
                A_r = [rh**2 * (math.cos(tl) - math.cos(th)) * dphi, rl**2 * (math.cos(tl) - math.cos(th)) * dphi]
                A_b = [0.5 * (rh**2 - rl**2) * sinf(th) * dphi, 0.5 * (rh**2 - rl**2) * sinf(tl) * dphi]
                d_b = [r * (cb[j + 1] - t), r * (t - cb[j - 1])]
                A_p = 0.5 * (rh**2 - rl**2) * (th - tl)
                d_p = r * math.sin(t) * dphi
            else:
                V = 0.5 * (rh**2 - rl**2) * dphi * (th - tl)
                A_r = [rh * dphi * (th - tl), rl * dphi * (th - tl)]
                A_b = [0.5 * (rh**2 - rl**2) * dphi, 0.5 * (rh**2 - rl**2) * dphi]
                d_b = [cb[j + 1] - t, t - cb[j - 1]]
                A_p = (rh - rl) * (th - tl)
                d_p = r * dphi
            d_r = [ca[i + 1] - r, r - ca[i - 1]]
            dv[i - 1, j - 1] = V
            nbrs = [(+1, 0, A_r[0] / d_r[0]), (-1, 0, A_r[1] / d_r[1]),
                    (0, +1, A_b[0] / d_b[0]), (0, -1, A_b[1] / d_b[1])]
            for k in range(nphi):
                me = idx[i - 1, j - 1, k]
                diag = 0.0
                for di, dj, w in nbrs:
                    w = w / V
                    diag -= w
                    ii, jj = i + di, j + dj
                    if 1 <= ii <= na and 1 <= jj <= nb:
                        rows.append(me); cols.append(idx[ii - 1, jj - 1, k]); vals.append(w)
                    elif w != 0.0:
                        edge = "a_lo" if ii == 0 else "a_hi" if ii == na + 1 else "b_lo" if jj == 0 else "b_hi"
                        gcoef[(me, edge, (j if edge[0] == "a" else i) - 1, k)] = w
                wp = A_p / d_p / V
                for dk in (+1, -1):
                    rows.append(me); cols.append(idx[i - 1, j - 1, (k + dk) % nphi]); vals.append(wp)
                    diag -= wp
                rows.append(me); cols.append(me); vals.append(diag)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))

    def rhs_from_ghosts(ghosts):
        out = np.zeros(N, dtype=np.result_type(*[np.asarray(v) for v in ghosts.values()], np.float64))
        for (me, edge, p, k), w in gcoef.items():
            if edge in ghosts:
                out[me] -= w * ghosts[edge][p, k]
        return out

    return A, rhs_from_ghosts, dv


def ghost_positions(spec):
    """Centroid coordinates of the ghost cells of each Dirichlet edge:
    dict edge -> (a array, b array) along the edge."""
    fa, fb, ca, cb, va, pole_lo, pole_hi = _faces_and_centroids(spec)
    na, nb = spec.n_a, spec.n_b
    out = {"a_lo": (np.full(nb, ca[0]), cb[1:nb + 1]), "a_hi": (np.full(nb, ca[na + 1]), cb[1:nb + 1])}
    if not pole_lo:
        out["b_lo"] = (ca[1:na + 1], np.full(na, cb[0]))
    if not pole_hi:
        out["b_hi"] = (ca[1:na + 1], np.full(na, cb[nb + 1]))
    return out
