"""The mesh-segment accuracy test (Sec. 6.1.2, Table of source and domain
parameters; convergence study of Sec. 6.1.3): a uniform grid-aligned
segment on the four grids of the paper (spherical / cylindrical x
logarithmic / uniform radius), solved by the HIP path (FP64, rel. residual
1e-10) at N = 32, 64, 128 and compared at sampled cell centres with the
oracle's reference potential (oracle/segment.py, the volume integral as a
surface integral, pinned by closed forms).  The error must fall at second
order (about 4x per doubling; > 3x is required) and at N = 256 (the paper's
resolution; uniform-radius grids) stay below the paper's 0.05% maximum
pointwise relative error.
Parity to the paper's exact reference formulas (which the paper cites but
does not print) is unpinned."""
import math

import numpy as np
import pytest

from oracle.segment import segment_density, segment_potential
from workloads import segment as W
from workloads.densities import to_cartesian

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _errors(name, N, n_sample, seed):
    from paper_2606_17636_amd import smg
    g = W.grid(name, N)
    geom, _, seg, _ = W.CONFIGS[name]
    print(f"[case] mesh segment {name} N={N}", flush=True)
    plan = smg.Plan(**g, precision="fp64", coarse_cells=2048).setup()
    a, b, p, _ = plan.geometry()
    from oracle.geometry import GridSpec, b_face, radial_face
    spec = GridSpec(**g)
    rho = segment_density(geom, seg, radial_face(spec, np.arange(N + 1)), b_face(spec, np.arange(N + 1)), 2 * N)
    phi, info = plan.solve(torch.from_numpy(rho).cuda(), tol=1e-10)
    assert info["converged"]
    phi = phi.cpu().numpy()
    rng = np.random.default_rng(seed)
    # a third of the sample inside the segment, the rest anywhere
    inside = np.argwhere(rho > 0)
    anyw = np.stack([rng.integers(0, s, n_sample) for s in rho.shape], axis=1)
    cells = np.concatenate([inside[rng.choice(len(inside), n_sample // 3, replace=False)], anyw[: n_sample - n_sample // 3]])
    x, y, z = to_cartesian(geom, a, b, p)
    pts = np.stack([x[tuple(cells.T)], y[tuple(cells.T)], z[tuple(cells.T)]], axis=1)
    ref = segment_potential(geom, seg, pts)
    eps = np.abs((phi[tuple(cells.T)] - ref) / ref)
    return float(np.sqrt(np.mean(eps**2))), float(eps.max())


@pytest.mark.parametrize("name", list(W.CONFIGS))
def test_mesh_segment_second_order(name):
    errs = [_errors(name, N, 36, 7) for N in (32, 64, 128)]
    print(name, "rms / max relative error at N = 32, 64, 128:", errs, flush=True)
    for (r0, _), (r1, _) in zip(errs[:-1], errs[1:]):
        assert r0 / r1 > 3.0, errs
    assert errs[-1][1] < 2e-3, errs


# N = 256 on the uniform-radius grids only: their DGF tables come from
# 33 x 33 auxiliary boxes; on the logarithmic grids every one of the 1024
# boundary sources of each of the 257 modes needs a solve on a 496 x 512
# extended domain, which takes far longer than a test may (there the N = 128
# maxima above, falling at second order, bound the N = 256 error).
@pytest.mark.parametrize("name", ["sph-uni", "cyl-uni"])
def test_mesh_segment_paper_bound(name):
    rms, mx = _errors(name, 256, 45, 11)
    print(name, "N = 256: rms", rms, "max", mx, flush=True)
    assert mx < 5e-4
