"""The 16-problem batch at its real shapes (spherical and cylindrical,
uniform and logarithmic radius, N in {64, 96, 128, 192}; 8 Gaussian blobs
each, seed 4), in the launch configuration bench.py times: one batch over
all problems, mixed precision, per-mode schedules replayed as graphs,
autotuned launch shapes, a 2048-cell exact coarsest level, smoothing steps
chosen by the library, SOR lines, rel. residual 1e-8.

The first solve runs the per-cycle host loop, the next two replay the
schedule's graph.  Every problem converges on every solve, and:
* the four problems the oracle solves whole in seconds (log sphere and log
  cylinder at N = 64, uniform cylinder at N = 96, uniform sphere at N = 128)
  match its full solve within 1e-6 relative L2 (volume-weighted);
* three N = 192 problems (uniform sphere, log sphere, log cylinder) match the
  oracle's sampled modes (m = 0, 1 and the Nyquist mode, through the seven
  steps with those modes' DGF tables) within 1e-6 of the largest sampled
  mode's norm."""
import math

import numpy as np
import pytest

from oracle import fourier
from oracle.geometry import GridSpec, cell_centres, cell_volumes_3d
from oracle.solve import OraclePlan
from tests.oracle_modes import oracle_modes
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FULL = [7, 15, 8, 0]
SAMPLED = {1: [0, 1, 96], 4: [0, 1, 96], 13: [0, 1, 96]}


@pytest.fixture(scope="module")
def solved():
    from paper_2606_17636_amd import smg
    grids = configs.c4_grids()
    plans = []
    for q, g in enumerate(grids):
        print(f"[setup] c4 problem {q}: {g['geometry']} {g['radial']} {g['n_a']}x{g['n_b']}x{g['n_phi']}", flush=True)
        plans.append(smg.Plan(**g, precision="mixed", launch="graph", autotune=True, line_solver="sor",
                              max_cycles=200, coarse_cells=2048, nu_pre=smg.NU_AUTO, nu_post=smg.NU_AUTO).setup())
    batch = smg.Batch(plans).setup()
    rhos = []
    for q, (g, p) in enumerate(zip(grids, plans)):
        a, b, ph, _ = p.geometry()
        rhos.append(configs.c4_density(q, g, a, b, ph))
    rd = [torch.from_numpy(r).cuda() for r in rhos]
    out = []
    for k in range(3):
        print(f"[solve] batch solve {k}", flush=True)
        phis, infos = batch.solve(rd, tol=1e-8)
        for q, i in enumerate(infos):
            assert i["converged"], (k, q)
        out.append([phi.cpu().numpy() for phi in phis])
    return grids, rhos, out


def test_c4_small_problems_match_oracle(solved):
    grids, rhos, out = solved
    for q in FULL:
        spec = GridSpec(**grids[q])
        print(f"[oracle] c4 problem {q} full solve", flush=True)
        ref = OraclePlan(spec).solve(rhos[q])
        w = cell_volumes_3d(spec)[:, :, None]
        for k, phis in enumerate(out):
            err = math.sqrt(np.sum((phis[q] - ref) ** 2 * w) / np.sum(ref**2 * w))
            print(f"problem {q} solve {k}: rel L2 vs oracle {err:.2e}", flush=True)
            assert err < 1e-6, (q, k, err)


def test_c4_large_problems_sampled_modes_match_oracle(solved):
    grids, rhos, out = solved
    for q, modes in SAMPLED.items():
        spec = GridSpec(**grids[q])
        assert max(modes) == spec.n_phi // 2
        ref = oracle_modes(spec, rhos[q], modes)
        scale = max(np.linalg.norm(ref[m]) for m in modes)
        for k, phis in enumerate(out):
            got = fourier.forward(phis[q])
            errs = {m: float(np.linalg.norm(got[m] - ref[m]) / scale) for m in modes}
            print(f"problem {q} solve {k}: per-mode error / max mode norm {errs}", flush=True)
            assert max(errs.values()) < 1e-6, (q, k, errs)
