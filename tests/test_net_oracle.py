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
