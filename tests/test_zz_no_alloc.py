"""The weight gradient entry point that allocates nothing
(smg_net_conv3_wgrad_noalloc, partial sums in the library's static device
array) against the entry point with a caller work buffer
(smg_net_conv3_wgrad): two calls in a row, the second on a smaller layer,
so the second reuses the array the first left behind.  dW is bit-identical
(same kernels, same pixel chunks, partials reduced in chunk order); db is
summed with FP32 atomics in block order, so it is held to the FP32
summation bound (P + 1) 2^-24 sum|g| of the other entry point's value."""
import numpy as np
import pytest

from oracle import net as onet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bits(v):
    return (np.asarray(v, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def test_noalloc_wgrad_matches_work_buffer_entry_point():
    from paper_2606_17636_amd import smg
    rng = np.random.default_rng(77)
    for shape in [(4, 64, 48, 64), (1, 20, 12, 8)]:          # second call smaller
        n, h, w, cin = shape
        print(f"[case] no-alloc wgrad {shape}", flush=True)
        x = torch.from_numpy(_bits(onet.bf16(rng.normal(size=(n, h, w, cin))))).cuda()
        gv = onet.bf16(rng.normal(size=(n, h, w, 32)))
        g = torch.from_numpy(_bits(gv)).cuda()
        dw_ref, db_ref = smg.conv3_wgrad(g, x)
        dw, db = smg.conv3_wgrad_noalloc(g, x)
        torch.cuda.synchronize()
        assert torch.equal(dw, dw_ref), shape
        P = n * h * w
        bound = (P + 1) * 2.0**-24 * np.abs(gv).sum(axis=(0, 1, 2))
        assert np.all(np.abs(db.cpu().numpy().astype(np.float64) - db_ref.cpu().numpy()) <= bound), shape
