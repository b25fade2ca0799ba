"""Reference potential of a uniform-density mesh segment (Sec. 6.1.2, the
mesh-segment test and its Table of source and domain parameters) -- oracle
side (test infrastructure only).

A mesh segment is the region r1 <= r <= r2, th1 <= theta <= th2,
ph1 <= phi <= ph2 (spherical) or R1 <= R <= R2, z1 <= z <= z2,
ph1 <= phi <= ph2 (cylindrical) of uniform density rho0; with the grid's
faces on its boundary it is represented exactly by the cells.  The paper
takes its reference potential from published line-and-surface-integral
formulas; this oracle computes the same potential from its definition,
Phi(x) = -G rho0 int_V dV' / |x - x'|, turned into a surface integral by
the divergence theorem (div' of the unit vector (x' - x)/|x' - x| is
2 / |x' - x|, with no point source at x' = x):

    Phi(x) = -(G rho0 / 2) sum over the faces S of int_S (x' - x).n / |x' - x| dS'

with n the outward normal.  The integrand is bounded by 1 everywhere and
peaks (width: the distance from x to the face) where the face passes
closest to x, so each face is integrated by tensor Gauss-Legendre panels
graded geometrically toward that point.  Parity: pinned by closed forms
(uniform sphere and shell, on-axis potential of a solid cylinder) and by
additivity over adjacent segments; the published exact formulas
themselves are not reproduced ("parity unpinned" to them).
"""
import math

import numpy as np

SPH = "spherical"
CYL = "cylindrical"

_GL_X, _GL_W = np.polynomial.legendre.leggauss(10)


def _graded_rule(a, b, c, ratio=0.3, levels=20, pieces=16):
    """Nodes and weights on [a, b] graded toward c (clipped into [a, b]):
    split at c, then on each side panels whose widths shrink geometrically
    toward c (down to ratio^levels of the side), panels wider than
    (b - a) / pieces cut into equal parts, 10 Gauss-Legendre points each."""
    c = min(max(c, a), b)
    hmax = (b - a) / pieces
    xs, ws = [], []
    for lo, hi in ((c, b), (c, a)):          # from c outward on each side
        L = hi - lo
        if abs(L) <= 0.0:
            continue
        edges = [0.0] + [ratio ** k for k in range(levels, 0, -1)] + [1.0]
        for e0, e1 in zip(edges[:-1], edges[1:]):
            k = max(1, int(math.ceil(abs(L) * (e1 - e0) / hmax)))
            for q in range(k):
                p0 = lo + L * (e0 + (e1 - e0) * q / k)
                p1 = lo + L * (e0 + (e1 - e0) * (q + 1) / k)
                mid, half = 0.5 * (p0 + p1), 0.5 * (p1 - p0)
                xs.append(mid + half * _GL_X)
                ws.append(abs(half) * _GL_W)
    return np.concatenate(xs), np.concatenate(ws)


def _face_integral(x, pts, normals, dA):
    """sum over the face nodes of (x' - x).n / |x' - x| dA."""
    d = pts - x[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    num = np.sum(d * normals, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        val = np.where(r > 0.0, num / r, 0.0)
    return float(np.sum(val * dA))


def _sph_point(r, th, ph):
    return np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], axis=-1)


def _potential_sph(x, seg, G, rho0):
    r1, r2, t1, t2, p1, p2 = seg
    xr = math.sqrt(float(x @ x))
    xth = math.acos(max(-1.0, min(1.0, x[2] / xr))) if xr > 0 else 0.0
    xph = math.atan2(x[1], x[0]) % (2 * math.pi)
    s_x = math.hypot(x[0], x[1])
    total = 0.0
    # nearest azimuth of the segment's range to x (periodic)
    def near_phi():
        c = xph
        for k in (-1, 0, 1):
            cand = xph + 2 * math.pi * k
            if p1 <= cand <= p2:
                return cand
        return min((p1, p2), key=lambda v: min(abs(v - xph), 2 * math.pi - abs(v - xph)))
    # r faces: sphere of radius rf, normal +-r_hat, dS = rf^2 sin th dth dph
    for rf, sgn in ((r2, 1.0), (r1, -1.0)):
        if rf <= 0.0:
            continue
        th, wt = _graded_rule(t1, t2, xth)
        ph, wp = _graded_rule(p1, p2, near_phi())
        T, P = np.meshgrid(th, ph, indexing="ij")
        pts = _sph_point(rf, T, P).reshape(-1, 3)
        n = sgn * pts / rf
        dA = (rf * rf * np.sin(T) * np.outer(wt, wp)).ravel()
        total += _face_integral(x, pts, n, dA)
    # theta faces: cone th = tf, normal +-theta_hat, dS = r sin tf dr dph
    for tf, sgn in ((t2, 1.0), (t1, -1.0)):
        if math.sin(tf) <= 1e-15:
            continue
        r0 = max(0.0, s_x * math.sin(tf) + x[2] * math.cos(tf))
        rr, wr = _graded_rule(r1, r2, r0)
        ph, wp = _graded_rule(p1, p2, near_phi())
        Rm, P = np.meshgrid(rr, ph, indexing="ij")
        pts = _sph_point(Rm, np.full_like(Rm, tf), P).reshape(-1, 3)
        that = np.stack([np.cos(tf) * np.cos(P), np.cos(tf) * np.sin(P), -np.sin(tf) * np.ones_like(P)], axis=-1)
        n = sgn * that.reshape(-1, 3)
        dA = (Rm * math.sin(tf) * np.outer(wr, wp)).ravel()
        total += _face_integral(x, pts, n, dA)
    # phi faces: half-plane ph = pf, normal +-phi_hat, dS = r dr dth
    if (p2 - p1) < 2 * math.pi - 1e-12:
        for pf, sgn in ((p2, 1.0), (p1, -1.0)):
            e = np.array([math.cos(pf), math.sin(pf), 0.0])
            sp = max(0.0, float(x @ e))
            r0 = math.hypot(sp, x[2])
            th0 = math.atan2(sp, x[2])
            rr, wr = _graded_rule(r1, r2, r0)
            th, wt = _graded_rule(t1, t2, th0)
            Rm, T = np.meshgrid(rr, th, indexing="ij")
            pts = _sph_point(Rm, T, np.full_like(Rm, pf)).reshape(-1, 3)
            n = sgn * np.array([-math.sin(pf), math.cos(pf), 0.0])[None, :]
            dA = (Rm * np.outer(wr, wt)).ravel()
            total += _face_integral(x, pts, n, dA)
    return -0.5 * G * rho0 * total


def _potential_cyl(x, seg, G, rho0):
    R1, R2, z1, z2, p1, p2 = seg
    xph = math.atan2(x[1], x[0]) % (2 * math.pi)
    xR = math.hypot(x[0], x[1])

    def near_phi():
        for k in (-1, 0, 1):
            cand = xph + 2 * math.pi * k
            if p1 <= cand <= p2:
                return cand
        return min((p1, p2), key=lambda v: min(abs(v - xph), 2 * math.pi - abs(v - xph)))
    total = 0.0
    # R faces: cylinder R = Rf, normal +-R_hat, dS = Rf dph dz
    for Rf, sgn in ((R2, 1.0), (R1, -1.0)):
        if Rf <= 0.0:
            continue
        ph, wp = _graded_rule(p1, p2, near_phi())
        zz, wz = _graded_rule(z1, z2, x[2])
        P, Z = np.meshgrid(ph, zz, indexing="ij")
        pts = np.stack([Rf * np.cos(P), Rf * np.sin(P), Z], axis=-1).reshape(-1, 3)
        n = sgn * np.stack([np.cos(P), np.sin(P), np.zeros_like(P)], axis=-1).reshape(-1, 3)
        dA = (Rf * np.outer(wp, wz)).ravel()
        total += _face_integral(x, pts, n, dA)
    # z faces: plane z = zf, normal +-z_hat, dS = R dR dph
    for zf, sgn in ((z2, 1.0), (z1, -1.0)):
        rr, wr = _graded_rule(R1, R2, xR)
        ph, wp = _graded_rule(p1, p2, near_phi())
        Rm, P = np.meshgrid(rr, ph, indexing="ij")
        pts = np.stack([Rm * np.cos(P), Rm * np.sin(P), np.full_like(Rm, zf)], axis=-1).reshape(-1, 3)
        n = np.array([0.0, 0.0, sgn])[None, :]
        dA = (Rm * np.outer(wr, wp)).ravel()
        total += _face_integral(x, pts, n, dA)
    # phi faces: half-plane ph = pf, normal +-phi_hat, dS = dR dz
    if (p2 - p1) < 2 * math.pi - 1e-12:
        for pf, sgn in ((p2, 1.0), (p1, -1.0)):
            e = np.array([math.cos(pf), math.sin(pf), 0.0])
            sp = max(0.0, float(x @ e))
            rr, wr = _graded_rule(R1, R2, sp)
            zz, wz = _graded_rule(z1, z2, x[2])
            Rm, Z = np.meshgrid(rr, zz, indexing="ij")
            pts = np.stack([Rm * math.cos(pf), Rm * math.sin(pf), Z], axis=-1).reshape(-1, 3)
            n = sgn * np.array([-math.sin(pf), math.cos(pf), 0.0])[None, :]
            dA = np.outer(wr, wz).ravel()
            total += _face_integral(x, pts, n, dA)
    return -0.5 * G * rho0 * total


def segment_potential(geometry, seg, points, G=1.0, rho0=1.0):
    """Potential of the uniform segment `seg` = (a1, a2, b1, b2, phi1, phi2)
    (a = r or R, b = theta or z) at Cartesian points (n, 3)."""
    f = _potential_sph if geometry == SPH else _potential_cyl
    return np.array([f(np.asarray(x, dtype=np.float64), seg, G, rho0) for x in np.atleast_2d(points)])


def segment_density(geometry, seg, a_faces, b_faces, n_phi, rho0=1.0):
    """Cell densities (n_a, n_b, n_phi) of the segment on a grid whose faces
    are a_faces (n_a + 1), b_faces (n_b + 1) and n_phi equal azimuthal
    cells: rho0 in cells inside the segment (their faces lie on its
    boundary when the grid is aligned), 0 elsewhere; a cell counts as inside
    when its centre in face-index space is."""
    a1, a2, b1, b2, p1, p2 = seg
    am = 0.5 * (a_faces[:-1] + a_faces[1:])
    bm = 0.5 * (b_faces[:-1] + b_faces[1:])
    pm = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    ina = (am > a1) & (am < a2)
    inb = (bm > b1) & (bm < b2)
    inp = (pm > p1) & (pm < p2)
    return rho0 * (ina[:, None, None] & inb[None, :, None] & inp[None, None, :]).astype(np.float64)
