"""Parity at full plane sizes, where the fused V-cycle keeps every level in
LDS with the coarser levels stored over the first level's right-hand side
(the layout used when the plain one exceeds 64 KiB), against the FP64 oracle.

* FP64 V-cycle on 64x32 planes: the plain fused layout needs about 92 KiB,
  so the whole cycle runs fused from the finest level in the overlaid
  layout; compared with the oracle's V-cycle at 1e-9 (the bar of the small
  V-cycle tests).
* FP64 V-cycle on the 129 modes of 128x64 planes: the finest level is
  smoothed by tiles of 16 radial lines (512 blocks over 129 planes), so the
  first post-smoothing launch applies the prolonged coarse correction while
  it loads its tile; sampled modes against the oracle's V-cycle at 1e-9.
* Cylindrical 256x128 planes (mixed, V(1,1) chosen by the library): sampled
  modes against the oracle's direct solve at 1e-8.
* Mixed-precision multigrid solves of the 65 modes of the 128x64 planes of
  the spherical log grid of the headline workload (rel. residual 1e-10),
  compared with the oracle's direct solve of every mode: relative L2 error
  below 1e-8 -- with the default hierarchy, with a 64x32 coarsest level
  solved exactly by fast diagonalisation, and with that level and the
  smoothing steps left to the library (V(1,1) here).
"""
import math

import numpy as np
import pytest

from oracle.geometry import GridSpec
from oracle.multigrid import Hierarchy
from oracle.solve import OraclePlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _random_modes(spec, seed):
    rng = np.random.default_rng(seed)
    shp = (spec.n_modes, spec.n_a, spec.n_b)
    x = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    x[0].imag = 0.0
    return x


def test_fused_overlaid_vcycle_fp64():
    from paper_2606_17636_amd import smg
    spec = GridSpec("spherical", "log", 64, 32, 8, 0.05, 5.0, 0.0, math.pi)
    print(f"[setup] {spec}", flush=True)
    gp = smg.grid_from_spec(spec, n_pad=8, precision="fp64", launch="dynamic").setup()
    f = _random_modes(spec, 21)
    ud = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    gp.mg_vcycle(_dev(f), ud)
    h = Hierarchy(spec)
    ref = np.zeros_like(f)
    for m in range(spec.n_modes):
        h.vcycle(ref[m], f[m], m)
    err = np.abs(ud.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-9, err


def test_vcycle_correction_applied_by_smoother_fp64():
    from paper_2606_17636_amd import smg
    spec = GridSpec("spherical", "log", 128, 64, 256, 0.05, 5.0, 0.0, math.pi)
    print(f"[setup] {spec}", flush=True)
    gp = smg.grid_from_spec(spec, n_pad=8, precision="fp64", launch="dynamic").setup()
    f = _random_modes(spec, 23)
    ud = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    gp.mg_vcycle(_dev(f), ud)
    u = ud.cpu().numpy()
    h = Hierarchy(spec)
    for m in (0, 1, 64, spec.n_modes - 1):
        ref = np.zeros_like(f[m])
        h.vcycle(ref, f[m], m)
        err = np.abs(u[m] - ref).max() / np.abs(ref).max()
        assert err < 1e-9, (m, err)


@pytest.mark.parametrize("coarse_cells,nu", [(0, 2), (2048, 2), (2048, -1)])
def test_headline_planes_mixed_solve(coarse_cells, nu):
    from paper_2606_17636_amd import smg
    from workloads import configs
    g = configs.GRIDS["c2"]
    spec = GridSpec(g["geometry"], g["radial"], g["n_a"], g["n_b"], g["n_phi"], g["a_min"], g["a_max"], g["b_min"],
                    g["b_max"], g.get("G", 1.0))
    print(f"[setup] {spec} coarse_cells {coarse_cells} nu {nu}", flush=True)
    # nu -1 = smg.NU_AUTO: the finest 128x64 level does not fit the fused
    # kernel, so the engine takes one smoothing step each way
    gp = smg.Plan(**g, precision="mixed", launch="dynamic", coarse_cells=coarse_cells, nu_pre=nu,
                  nu_post=nu).setup("cuda:0")
    a, b, p, _ = gp.geometry()
    op = OraclePlan(spec, dgf=0)   # only the per-mode direct solves are used
    f = op.source_modes(configs.density("c2", a, b, p))
    ud = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    cycles, res = gp.mg_solve(_dev(f), ud, 1e-10)
    print(f"[solve] cycles m=0 {cycles[0]}, max {cycles.max()}", flush=True)
    ref = op.solve_modes(f)
    u = ud.cpu().numpy()
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert err < 1e-8, err
    assert np.all(res <= 1e-10)


def test_cylindrical_full_planes_auto_smoothing():
    """256x128 cylindrical planes (the C3 grid with 17 modes): the finest
    level is smoothed by whole-grid launches, so the library takes V(1,1) and
    starts each correction cycle from zero without reading it; a mixed
    solve to 1e-10 against the oracle's direct solve of sampled modes."""
    from paper_2606_17636_amd import smg
    from workloads import configs
    g = dict(configs.GRIDS["c3"], n_phi=32)
    spec = GridSpec(g["geometry"], g["radial"], g["n_a"], g["n_b"], g["n_phi"], g["a_min"], g["a_max"], g["b_min"],
                    g["b_max"], g.get("G", 1.0))
    print(f"[setup] {spec}", flush=True)
    gp = smg.Plan(**g, precision="mixed", launch="dynamic", coarse_cells=2048, nu_pre=smg.NU_AUTO,
                  nu_post=smg.NU_AUTO).setup("cuda:0")
    f = _random_modes(spec, 31)
    ud = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    cycles, res = gp.mg_solve(_dev(f), ud, 1e-10)
    print(f"[solve] cycles m=0 {cycles[0]}, max {cycles.max()}", flush=True)
    assert np.all(res <= 1e-10)
    u = ud.cpu().numpy()
    op = OraclePlan(spec, dgf=0)
    for m in (0, 7, spec.n_modes - 1):
        lu = op.lu(m)
        r = f[m].reshape(-1)
        ref = (lu.solve(r.real.copy()) + 1j * lu.solve(r.imag.copy())).reshape(spec.n_a, spec.n_b)
        err = np.linalg.norm(u[m] - ref) / np.linalg.norm(ref)
        assert err < 1e-8, (m, err)
