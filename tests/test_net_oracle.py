"""Pins of the learned-guess network's CPU oracle (oracle/net.py): the
BF16 rounding against torch's conversion, the 3x3 convolution against
scipy's correlation, the backward pass against central finite differences,
pooling / upsampling adjoints, and the zero-initialised output layer."""
import math

import numpy as np
import pytest
import scipy.signal

from oracle import net
from workloads.netinit import init_params, layer_shapes


def test_layer_order_matches_generator():
    assert [tuple(s) for s in net.layer_shapes()] == [tuple(s) for s in layer_shapes()]
    assert net.n_params() == init_params(0).size


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [1.0 + 2**-8, 1.0 + 3 * 2**-8, -(1.0 + 2**-8), 0.0, -0.0, 65504.0, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(x), ref)


def test_conv3_matches_scipy_correlation():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 7, 9, 3))
    W = rng.normal(size=(4, 9, 3))
    b = rng.normal(size=4)
    out = net.conv3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = np.full((7, 9), b[o])
            for c in range(3):
                k = W[o, :, c].reshape(3, 3)        # k[dy+1, dx+1]
                ref += scipy.signal.correlate2d(x[n, :, :, c], k, mode="same", boundary="fill")
            assert np.allclose(out[n, :, :, o], ref, atol=1e-12)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 8, 6, 3))
    y = rng.normal(size=(2, 4, 3, 3))
    assert math.isclose(np.sum(net.pool2(x) * y), np.sum(x * net.pool2_backward(y)), rel_tol=1e-12)
    assert math.isclose(np.sum(net.up2(y) * x), np.sum(y * net.up2_backward(x)), rel_tol=1e-12)


@pytest.mark.parametrize("levels,ch", [(2, 4), (3, 4)])
def test_backward_matches_finite_differences(levels, ch):
    rng = np.random.default_rng(4)
    P = net.n_params(levels, ch)
    params = rng.normal(0, 0.5, P)
    x = rng.normal(0, 1, (2, 8, 8, 8))
    t = rng.normal(0, 1, (2, 8, 8))

    def L(p):
        return net.loss(net.forward(p, x, rounding=False, levels=levels, ch=ch)[0], t)[0]

    out, cache = net.forward(params, x, rounding=False, levels=levels, ch=ch)
    grad = net.backward(params, cache, net.loss(out, t)[1], levels=levels, ch=ch)
    idx = rng.choice(P, 60, replace=False)
    h = 1e-6
    e = np.eye(1, P)
    fd = np.array([(L(params + h * np.roll(e[0], i)) - L(params - h * np.roll(e[0], i))) / (2 * h) for i in idx])
    assert np.max(np.abs(fd - grad[idx])) <= 1e-7 * np.max(np.abs(fd))


def test_zero_output_layer_gives_zero_change():
    x = np.random.default_rng(5).normal(size=(1, 16, 16, 8))
    out, _ = net.forward(init_params(7), x)
    assert np.all(out == 0.0)


def test_rounded_forward_is_close_to_exact():
    rng = np.random.default_rng(6)
    p = init_params(8, zero_output=False)
    x = rng.normal(size=(1, 16, 16, 8))
    a, _ = net.forward(p, x, rounding=True)
    b, _ = net.forward(p, x, rounding=False)
    assert np.linalg.norm(a - b) < 0.05 * np.linalg.norm(b)


# -- the learned guess's input assembly, candidate and judge --------------------
def _planes(rng, M, na, nb):
    return rng.standard_normal((M, na, nb)) + 1j * rng.standard_normal((M, na, nb))


def test_guess_images_layout_and_scaling():
    """Image k is the real (k odd, k = 0) or imaginary (k even > 0) part of
    mode (k + 1) // 2; channels 0-2 have unit RMS; the inputs do not change
    when f, f_prev and u_prev are scaled; the change channel is
    (f - f_prev) / RMS(f - f_prev)."""
    rng = np.random.default_rng(40)
    M, na, nb, m_max = 5, 12, 10, 3
    f, fp, up = _planes(rng, M, na, nb), _planes(rng, M, na, nb), _planes(rng, M, na, nb)
    x, sc = net.guess_images(f, fp, up, m_max)
    assert x.shape == (2 * m_max + 1, na, nb, 8) and sc.shape == (2 * m_max + 1, 4)
    for k in range(2 * m_max + 1):
        m = (k + 1) // 2
        part = (lambda z: z.imag) if (k > 0 and k % 2 == 0) else (lambda z: z.real)
        d = part(f[m]) - part(fp[m])
        assert np.allclose(x[k, :, :, 0] * sc[k, 0], part(f[m]), rtol=1e-14, atol=0)
        assert np.allclose(x[k, :, :, 1], d / math.sqrt(np.mean(d * d)), rtol=1e-13, atol=0)
        assert np.allclose(x[k, :, :, 2] * sc[k, 2], part(up[m]), rtol=1e-14, atol=0)
        assert np.allclose(np.sqrt(np.mean(x[k, :, :, :3] ** 2, axis=(0, 1))), 1.0, rtol=1e-13)
        assert np.all(x[k, :, :, 3] == m / 4.0)
        assert abs(sc[k, 3] - sc[k, 2] * sc[k, 1] / sc[k, 0]) <= 1e-15 * sc[k, 3]   # no u_{t-2}
    assert np.allclose(x[0, :, 0, 4], (np.arange(na) + 0.5) / na - 0.5)
    assert np.allclose(x[0, 0, :, 5], (np.arange(nb) + 0.5) / nb - 0.5)
    assert np.all(x[..., 6:] == 0.0)
    # channel 6: the previous change of the solution in units of the output scale
    u2 = _planes(rng, M, na, nb)
    x6, sc6 = net.guess_images(f, fp, up, m_max, uprev2=u2)
    assert np.array_equal(x6[..., :6], x[..., :6]) and np.all(x6[0, :, :, 7] == 0.0)
    assert np.array_equal(sc6[:, :3], sc[:, :3])
    for k in range(2 * m_max + 1):
        m = (k + 1) // 2
        part = (lambda z: z.imag) if (k > 0 and k % 2 == 0) else (lambda z: z.real)
        e = part(up[m]) - part(u2[m])
        assert abs(sc6[k, 3] - math.sqrt(np.mean(e * e))) <= 1e-14 * sc6[k, 3]
        assert np.allclose(x6[k, :, :, 6] * sc6[k, 3], e, rtol=1e-13, atol=0)
        assert abs(math.sqrt(np.mean(x6[k, :, :, 6] ** 2)) - 1.0) < 1e-13
        if m > 0:   # channel 7: the other part, as a rotation generator -i d: (Im d, -Re d)
            other = (up[m] - u2[m]).real if part(1j) != 0 else (up[m] - u2[m]).imag
            sign = -1.0 if part(1j) != 0 else 1.0
            assert np.allclose(x6[k, :, :, 7] * sc6[k, 3], sign * other, rtol=1e-13, atol=0)
    x2, _ = net.guess_images(3.5 * f, 3.5 * fp, -2.0 * up, m_max)
    assert np.allclose(x2[..., :2], x[..., :2], rtol=1e-13) and np.allclose(x2[..., 2], -x[..., 2], rtol=1e-13)
    # a zero plane keeps scale 1 (no division by zero)
    f0 = f.copy(); f0[1] = 0.0
    _, sc0 = net.guess_images(f0, f0, up, m_max)
    assert sc0[1, 0] == 1.0 and sc0[2, 1] == 1.0


def test_guess_candidate_inverts_the_target():
    """The training target is the correction the candidate needs, so the
    candidate built from a perfect prediction is u_t -- with the
    extrapolation from u_{t-2} and without it (the imaginary part of m = 0
    is only extrapolated); a zero prediction gives the extrapolation
    2 u_{t-1} - u_{t-2} itself."""
    rng = np.random.default_rng(41)
    M, na, nb, m_max = 6, 8, 6, 4
    f, fp, up, ut, u2 = (_planes(rng, M, na, nb) for _ in range(5))
    for prev2 in (None, u2):
        upk = up.copy()
        ext = upk if prev2 is None else 2 * upk - prev2
        upk[0] = upk[0].real + 1j * (ut[0].imag if prev2 is None else 0.5 * (ut[0].imag + prev2[0].imag))
        _, sc = net.guess_images(f, fp, upk, m_max, uprev2=prev2)
        y = net.guess_target(ut, upk, sc, m_max, uprev2=prev2)
        cand = net.guess_candidate(upk, y, sc, m_max, uprev2=prev2)
        assert np.allclose(cand, ut[:m_max + 1], rtol=0, atol=1e-13 * np.abs(ut).max())
    zero = net.guess_candidate(up, np.zeros((2 * m_max + 1, na, nb)), sc, m_max, uprev2=u2)
    assert np.allclose(zero, (2 * up - u2)[:m_max + 1], rtol=0, atol=1e-14 * np.abs(up).max())
    # the judge's baseline is that zero-correction candidate: the
    # extrapolation, or u_{t-1} before a second solution exists
    assert np.array_equal(net.guess_base(up, sc, m_max, uprev2=u2), zero)
    _, sc1 = net.guess_images(f, fp, up, m_max)
    assert np.array_equal(net.guess_base(up, sc1, m_max), up[:m_max + 1])


def test_guess_judge_prefers_the_better_start():
    """The judge picks the exact solution over a perturbed one in both
    directions, and keeps the previous solution on a tie."""
    from oracle.geometry import GridSpec
    from oracle.multigrid import MGLevel
    from oracle.solve import OraclePlan
    spec = GridSpec("spherical", "log", 16, 8, 8, 0.05, 5.0, 0.0, math.pi)
    rng = np.random.default_rng(42)
    f = _planes(rng, spec.n_modes, 16, 8)
    u = OraclePlan(spec, dgf=np.zeros((spec.n_modes, 1, 1))).solve_modes(f)
    lev = MGLevel(spec, 0)
    bad = u + 0.3 * np.abs(u).max() * np.cos(np.arange(8))[None, None, :]
    m_max = 2
    cand = np.stack([u[0], bad[1], u[2]])
    prev = np.stack([bad[0], u[1], u[2]])
    for ls in ("sor", "exact"):
        used, nc, nu = net.guess_judge(lev, f, cand, prev, m_max, line_solver=ls)
        assert list(used) == [1, 0, 0], (ls, nc, nu)
        assert nc[2] == nu[2]


def test_static_plane_is_left_alone():
    """A plane whose last change is below STATIC of its size (e.g. the
    axisymmetric mode of orbiting blobs) is
    static: s_o = 0, no change channel, no extrapolation, no correction and
    a zero training target."""
    rng = np.random.default_rng(43)
    M, na, nb, m_max = 3, 8, 6, 2
    f, fp, up, ut = (_planes(rng, M, na, nb) for _ in range(4))
    u2 = up + 1e-7 * _planes(rng, M, na, nb)               # a change far below 1e-4 of the plane
    x, sc = net.guess_images(f, fp, up, m_max, uprev2=u2)
    assert np.all(sc[:, 3] == 0.0) and np.all(x[..., 6:] == 0.0)
    y = rng.standard_normal((2 * m_max + 1, na, nb))
    assert np.array_equal(net.guess_candidate(up, y, sc, m_max, uprev2=u2), up[:m_max + 1])
    assert np.all(net.guess_target(ut, up, sc, m_max, uprev2=u2) == 0.0)
