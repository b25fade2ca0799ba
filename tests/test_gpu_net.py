"""The learned-guess network on the GPU (MFMA BF16 kernels, through the C
ABI) against its CPU oracle with the same BF16 rounding points: forward
outputs and parameter gradients, and an Adam training run that lowers the
loss.

Tolerance.  Both sides round every stored activation to BF16, the GPU from
an FP32 sum, the oracle from an FP64 sum.  A sum that falls within FP32
rounding of a BF16 rounding boundary (about one value in 2^15) can round
the other way; that flips the activation by one BF16 ulp (2^-8 relative)
and the change propagates through the later layers of that image.  Small
images see no flip and agree to FP32 rounding (1e-6); larger batches are
held to 1e-2 relative L2 (a few flips), gradients likewise."""
import numpy as np
import pytest

from oracle import net as onet
from workloads.netinit import init_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def gnet():
    from paper_2606_17636_amd import smg
    return smg.Net(levels=4, channels=32)


@pytest.mark.parametrize("shape,tol", [((1, 8, 8), 1e-6), ((2, 32, 16), 1e-2), ((3, 24, 40), 1e-2)])
def test_forward_matches_oracle(gnet, shape, tol):
    n, h, w = shape
    rng = np.random.default_rng(10 + h)
    p = init_params(11, zero_output=False)
    x = rng.normal(size=(n, h, w, 8))
    gnet.set_params(p)
    y = gnet.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
    ref, _ = onet.forward(p.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    print(shape, _rel(y, ref), [_rel(y[k], ref[k]) for k in range(n)], flush=True)
    assert _rel(y, ref) < tol


@pytest.mark.parametrize("shape", [(2, 16, 16), (2, 32, 24)])
def test_backward_matches_oracle(gnet, shape):
    n, h, w = shape
    rng = np.random.default_rng(20 + h)
    p = init_params(12, zero_output=False)
    x = rng.normal(size=(n, h, w, 8)).astype(np.float32)
    t = rng.normal(size=(n, h, w)).astype(np.float32)
    pp = p.astype(np.float32).astype(np.float64)
    ref_out, cache = onet.forward(pp, x.astype(np.float64))
    _, g = onet.loss(ref_out, t.astype(np.float64))
    ref = onet.backward(pp, cache, g)
    gnet.set_params(p)
    y = gnet.forward(torch.from_numpy(x).cuda())
    dy = (2.0 * (y - torch.from_numpy(t).cuda()) / y.numel()).contiguous()
    got = gnet.backward(dy).cpu().numpy().astype(np.float64)
    per_layer = []
    for (W, b), (Wr, br) in zip(onet.unpack(got), onet.unpack(ref)):
        per_layer.append(max(_rel(W.ravel(), Wr.ravel()), _rel(b, br) if np.linalg.norm(br) > 0 else 0.0))
    print(shape, ["%.1e" % v for v in per_layer], flush=True)
    assert _rel(got, ref) < 1e-2
    assert max(per_layer) < 3e-2


def test_training_lowers_loss(gnet):
    """A fixed linear map (a smoothing of channel 1) is learned: Adam steps
    through smg_net_train_step lower the loss by an order of magnitude."""
    rng = np.random.default_rng(30)
    n, h, w = 64, 16, 16
    x = rng.normal(size=(n, h, w, 8)).astype(np.float32)
    t = 0.5 * x[..., 1] + 0.25 * np.roll(x[..., 1], 1, axis=1)
    samples = np.concatenate([x.reshape(n, -1), t.reshape(n, -1)], axis=1).astype(np.float32)
    st = torch.from_numpy(samples).cuda().contiguous()
    gnet.set_params(init_params(13))
    losses = []
    for step in range(300):
        idx = rng.choice(n, 8, replace=False)
        losses.append(gnet.train_step(st, idx, h, w, 2e-3))
    print(losses[0], np.mean(losses[-20:]), flush=True)
    assert np.mean(losses[-20:]) < 0.1 * losses[0]
