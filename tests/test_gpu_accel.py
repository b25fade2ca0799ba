"""Parity of the face acceleration (smg_acceleration, through the C ABI) with
the oracle (oracle/acceleration.py, itself pinned in test_accel_oracle.py).

* Kernel parity: the same seeded potential and screening potential Theta on
  both sides, every face array compared element by element at rounding
  level (1e-13 of the array maximum), on grids with poles, a partial theta
  range (Dirichlet theta edges), cylindrical and log-radial spacing, and
  N_phi with a radix-3 factor.
* After a solve: the GPU acceleration of the GPU solution (Theta of the same
  solve) against the oracle acceleration of the oracle's direct solution,
  within the solve tolerance (1e-9 relative).
* Without Theta and before any solve the call fails with SMG_ESTATE.
"""
import math

import numpy as np
import pytest

from oracle import acceleration as acc
from oracle.geometry import GridSpec, cell_centres
from oracle.james import GhostSet
from oracle.solve import OraclePlan
from workloads.densities import gaussian_blobs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPECS = {
    "sph-uni": (GridSpec("spherical", "uniform", 32, 16, 32, 0.1, 1.0, 0.0, math.pi), 16),
    "sph-log": (GridSpec("spherical", "log", 48, 24, 24, 0.05, 5.0, 0.0, math.pi), 16),
    "cyl-uni": (GridSpec("cylindrical", "uniform", 24, 20, 12, 0.2, 2.0, -0.5, 0.5), 8),
    "cyl-log": (GridSpec("cylindrical", "log", 40, 12, 12, 0.05, 5.0, -2.5, 2.5), 16),
    "sph-part": (GridSpec("spherical", "uniform", 16, 24, 8, 1.9, 3.5, 0.34 * math.pi, 0.66 * math.pi), 6),
}

_plans = {}


def _plan(key):
    if key not in _plans:
        from paper_2606_17636_amd import smg
        spec, npad = SPECS[key]
        print(f"[setup] {key} {spec}", flush=True)
        _plans[key] = smg.grid_from_spec(spec, n_pad=npad).setup()
    return _plans[key]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _close(gpu, ref, tol):
    ref = np.asarray(ref)
    return float(np.abs(gpu.cpu().numpy() - ref).max() / max(np.abs(ref).max(), 1e-300)) < tol


@pytest.mark.parametrize("key", list(SPECS))
def test_acceleration_kernel_parity(key):
    spec, _ = SPECS[key]
    gp = _plan(key)
    rng = np.random.default_rng(40)
    phi = rng.standard_normal((spec.n_a, spec.n_b, spec.n_phi))
    th = rng.standard_normal((spec.n_modes, gp.n_ghost)) + 1j * rng.standard_normal((spec.n_modes, gp.n_ghost))
    g_a, g_b, g_p = gp.acceleration(_dev(phi), _dev(th))
    gh = GhostSet(spec)
    assert gh.n == gp.n_ghost
    r_a, r_b, r_p = acc.face_acceleration(spec, phi, gh, acc.ghost_potential(spec, th))
    assert _close(g_a, r_a, 1e-13) and _close(g_b, r_b, 1e-13) and _close(g_p, r_p, 1e-13)


@pytest.mark.parametrize("key", ["sph-log", "cyl-uni", "sph-part"])
def test_acceleration_after_solve(key):
    from paper_2606_17636_amd import smg
    spec, npad = SPECS[key]
    gp = smg.grid_from_spec(spec, n_pad=npad).setup()
    a, b, p = cell_centres(spec)
    if spec.geometry == "spherical":
        amid = 0.5 * (spec.a_min + spec.a_max) if spec.radial == "uniform" else math.sqrt(spec.a_min * spec.a_max)
        cen = [(amid, 0.5 * (spec.b_min + spec.b_max) + 0.1, 0.3)]
    else:
        cen = [(0.5 * (spec.a_min + spec.a_max), 0.05, 0.3)]
    rho = gaussian_blobs(spec.geometry, a, b, p, cen, [0.2 * (spec.a_max - spec.a_min)], [1.0])
    phi, info = gp.solve(_dev(rho), tol=1e-12)
    assert info["converged"]
    g_a, g_b, g_p = gp.acceleration(phi)
    op = OraclePlan(spec, n_pad=npad)
    phi_o, parts = op.solve(rho, return_parts=True)
    gh = GhostSet(spec)
    r_a, r_b, r_p = acc.face_acceleration(spec, phi_o, gh, acc.ghost_potential(spec, parts["theta"]))
    assert _close(g_a, r_a, 1e-9) and _close(g_b, r_b, 1e-9) and _close(g_p, r_p, 1e-9)


def test_acceleration_needs_theta():
    from paper_2606_17636_amd import smg
    spec, npad = SPECS["cyl-uni"]
    gp = smg.grid_from_spec(spec, n_pad=npad).setup()
    phi = torch.zeros((spec.n_a, spec.n_b, spec.n_phi), dtype=torch.float64, device="cuda")
    with pytest.raises(smg.SmgError, match="SMG_ESTATE"):
        gp.acceleration(phi)
