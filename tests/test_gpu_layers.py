"""Single layers of the learned-guess network on the GPU (smg_net_conv3,
smg_net_conv3_wgrad) against the oracle's 3x3 convolution and its weight
gradient, element by element.

Inputs and weights are BF16 values, so every product is exact in FP32 and
the only rounding on the GPU is the FP32 accumulation of K = 9 c_in terms
(then BF16 for activations).  For any summation order the FP32 sum lies
within delta = (K + 1) 2^-24 sum|terms| of the exact value, so each GPU
activation must lie within half a BF16 ulp plus delta of the oracle's exact
(FP64) pre-rounding value, and all but the rare values within delta of a
BF16 rounding midpoint must be bit-identical to the oracle's rounded
value.  Weight gradients (FP32, a sum over P pixels) must lie within
(P + 1) 2^-24 sum|terms| of the oracle's."""
import numpy as np
import pytest

from oracle import net as onet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0**-24


def _bits(v):
    """BF16 values (float64 array exactly representable) -> int16 bits."""
    return (np.asarray(v, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def _vals(bits):
    return (bits.astype(np.int16).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _ulp_bf16(v):
    """Spacing of BF16 values at |v| (2^(e - 7) for |v| in [2^e, 2^(e+1)))."""
    a = np.maximum(np.abs(v), 2.0**-126)
    return 2.0 ** (np.floor(np.log2(a)) - 7)


SHAPES = [(1, 8, 8, 8), (2, 32, 24, 32), (1, 33, 40, 64), (3, 16, 70, 8), (1, 5, 3, 32)]


@pytest.mark.parametrize("relu", [True, False])
@pytest.mark.parametrize("shape", SHAPES)
def test_conv3_layer_elementwise(shape, relu):
    from paper_2606_17636_amd import smg
    n, h, w, cin = shape
    rng = np.random.default_rng(hash((shape, relu)) % 2**31)
    x = onet.bf16(rng.normal(size=(n, h, w, cin)))
    W = onet.bf16(rng.normal(0.0, (2.0 / (9 * cin)) ** 0.5, size=(32, 9, cin)))
    b = rng.normal(0.0, 0.1, 32).astype(np.float32).astype(np.float64)
    print(f"[case] conv3 {shape} relu={relu}", flush=True)
    yb = smg.conv3_layer(torch.from_numpy(_bits(x)).cuda(), torch.from_numpy(_bits(W)).cuda(),
                         torch.from_numpy(b.astype(np.float32)).cuda(), relu=relu)
    y = _vals(yb.cpu().numpy())
    v = onet.conv3(x, W, b)
    mag = onet.conv3(np.abs(x), np.abs(W), np.abs(b))
    delta = (9 * cin + 1) * U * mag
    r = np.maximum(v, 0.0) if relu else v
    assert np.all(np.abs(y - r) <= 0.5 * _ulp_bf16(np.abs(r) + delta) + delta), np.abs(y - r).max()
    same = np.mean(y == onet.bf16(r))
    print("bit-identical fraction", same, flush=True)
    assert same >= 0.999


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3_wgrad_elementwise(shape):
    from paper_2606_17636_amd import smg
    n, h, w, cin = shape
    rng = np.random.default_rng(7 + hash(shape) % 2**31)
    x = onet.bf16(rng.normal(size=(n, h, w, cin)))
    g = onet.bf16(rng.normal(size=(n, h, w, 32)))
    print(f"[case] wgrad {shape}", flush=True)
    dW, db = smg.conv3_wgrad(torch.from_numpy(_bits(g)).cuda(), torch.from_numpy(_bits(x)).cuda())
    _, gW, gb = onet.conv3_backward(x, np.zeros((32, 9, cin)), g)
    _, mW, mb = onet.conv3_backward(np.abs(x), np.zeros((32, 9, cin)), np.abs(g))
    P = n * h * w
    eW = np.abs(dW.cpu().numpy().astype(np.float64) - gW)
    eb = np.abs(db.cpu().numpy().astype(np.float64) - gb)
    assert np.all(eW <= (P + 1) * U * mW + 1e-30), (eW / np.maximum(mW, 1e-30)).max()
    assert np.all(eb <= (P + 1) * U * mb + 1e-30), (eb / np.maximum(mb, 1e-30)).max()
    print("max error / sum|terms|", (eW / np.maximum(mW, 1e-30)).max(), flush=True)
