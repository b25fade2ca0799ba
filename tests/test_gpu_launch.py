"""The launch machinery of the solve (device-side convergence lists, per-mode
cycle schedules replayed as HIP graphs, the setup-time autotuner) against the
plain per-cycle host loop and the FP64 oracle.

Every plane's V-cycles do not depend on which other planes share a launch,
so a scheduled solve that runs each mode for the same cycles as the host
loop gives the same bits."""
import math

import numpy as np
import pytest

from oracle.geometry import GridSpec, cell_centres, cell_volumes_3d
from oracle.solve import OraclePlan
from workloads.densities import gaussian_blobs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPEC = GridSpec("spherical", "log", 48, 24, 24, 0.05, 5.0, 0.0, math.pi)
SPEC_CYL = GridSpec("cylindrical", "uniform", 24, 20, 12, 0.2, 2.0, -0.5, 0.5)
SPEC_SPLIT = GridSpec("spherical", "log", 128, 64, 16, 0.05, 5.0, 0.0, math.pi)


def _blobs(spec, seed, axisymmetric=False):
    a, b, p = cell_centres(spec)
    rng = np.random.default_rng(seed)
    n = 3
    if spec.geometry == "spherical":
        cen = [(math.exp(rng.uniform(math.log(0.3), math.log(2.0))), rng.uniform(0.8, 2.3), rng.uniform(0, 2 * math.pi))
               for _ in range(n)]
    else:
        cen = [(rng.uniform(0.6, 1.6), rng.uniform(-0.3, 0.3), rng.uniform(0, 2 * math.pi)) for _ in range(n)]
    w = rng.uniform(0.15, 0.4, n)
    amp = rng.lognormal(0.0, 1.0, n)
    rho = gaussian_blobs(spec.geometry, a, b, p, cen, w, amp)
    if axisymmetric:
        rho = np.repeat(rho.mean(axis=2, keepdims=True), spec.n_phi, axis=2)
    return rho


def _plan(spec, **kw):
    from paper_2606_17636_amd import smg
    print(f"[setup] {spec} {kw}", flush=True)
    npad = 8 if spec.radial == "uniform" else 16
    return smg.grid_from_spec(spec, n_pad=npad, **kw).setup()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _l2(spec, x, ref):
    w = cell_volumes_3d(spec)[:, :, None]
    return math.sqrt(np.sum((x - ref) ** 2 * w) / np.sum(ref**2 * w))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_host_loop_bitwise(precision):
    dyn = _plan(SPEC, precision=precision, launch="dynamic")
    gra = _plan(SPEC, precision=precision, launch="graph")
    rho = _dev(_blobs(SPEC, 1))
    ref, info_d = dyn.solve(rho, tol=1e-9)
    for k in range(3):  # first solve: host loop; then the scheduled graph
        phi, info_g = gra.solve(rho, tol=1e-9)
        assert info_g["converged"]
        assert np.array_equal(info_g["cycles1"], info_d["cycles1"])
        assert np.array_equal(info_g["cycles2"], info_d["cycles2"])
        assert torch.equal(phi, ref), f"solve {k}"


def test_graph_replay_matches_host_loop_bitwise_split_levels():
    """128x64 planes: the finest level is smoothed by whole-grid launches
    (V(1,1) chosen by the library, zero start of the correction cycle, the
    coarse correction and the FP64 accumulation inside the smoothing
    launches); graph replay and host loop still give the same bits."""
    kw = dict(precision="mixed", nu_pre=-1, nu_post=-1, coarse_cells=2048)
    dyn = _plan(SPEC_SPLIT, launch="dynamic", **kw)
    gra = _plan(SPEC_SPLIT, launch="graph", **kw)
    rho = _dev(_blobs(SPEC_SPLIT, 5))
    ref, info_d = dyn.solve(rho, tol=1e-9)
    assert info_d["converged"]
    for k in range(3):
        phi, info_g = gra.solve(rho, tol=1e-9)
        assert np.array_equal(info_g["cycles1"], info_d["cycles1"])
        assert np.array_equal(info_g["cycles2"], info_d["cycles2"])
        assert torch.equal(phi, ref), f"solve {k}"



def test_profiled_solve_matches_graph_replay_bitwise():
    """A profiled solve enqueues the scheduled launches of the graph replay
    from the host, with events between them: the same kernels, shapes and
    plane counts, so the same bits as the replay.  The per-class statistics
    cover the finest-level smoothing with positive durations."""
    kw = dict(precision="mixed", nu_pre=-1, nu_post=-1, coarse_cells=2048)
    gra = _plan(SPEC_SPLIT, launch="graph", **kw)
    rho = _dev(_blobs(SPEC_SPLIT, 7))
    gra.solve(rho, tol=1e-9)  # host loop: learns the per-mode schedule
    ref, info = gra.solve(rho, tol=1e-9)  # graph replay
    gra.profile_begin()
    phi, info_p = gra.solve(rho, tol=1e-9)
    stats = gra.profile_end()
    assert info_p["converged"]
    assert np.array_equal(info_p["cycles1"], info["cycles1"])
    assert np.array_equal(info_p["cycles2"], info["cycles2"])
    assert torch.equal(phi, ref)
    for cls in ("smooth_radial_lines_l0", "smooth_polar_lines_l0", "lds_coarse_cycle", "defect_norm"):
        assert stats[cls]["launches"] > 0, cls
        assert stats[cls]["total_ms"] > 0.0 and stats[cls]["bytes"] > 0.0, cls
    # and a later replay still gives the same bits
    phi2, _ = gra.solve(rho, tol=1e-9)
    assert torch.equal(phi2, ref)


def test_schedule_shortfall_is_finished():
    """A schedule learnt on an axisymmetric density (no cycles for m > 0)
    applied to a general one: the modes it starves are finished after the
    replay and the result meets the FP64 tolerance."""
    gra = _plan(SPEC, launch="graph")
    op = OraclePlan(SPEC, n_pad=16)
    sym = _blobs(SPEC, 2, axisymmetric=True)
    for _ in range(2):
        gra.solve(_dev(sym), tol=1e-12)
    rho = _blobs(SPEC, 3)
    phi, info = gra.solve(_dev(rho), tol=1e-12)
    assert info["converged"]
    assert int(info["cycles1"][1:].sum()) > 0
    assert _l2(SPEC, phi.cpu().numpy(), op.solve(rho)) < 1e-10
    # and the schedule adapts: the same density again replays without a shortfall
    phi2, info2 = gra.solve(_dev(rho), tol=1e-12)
    assert np.array_equal(info2["cycles1"], info["cycles1"])
    assert _l2(SPEC, phi2.cpu().numpy(), op.solve(rho)) < 1e-10


@pytest.mark.parametrize("spec", [SPEC, SPEC_CYL], ids=["sph-log", "cyl-uni"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_plan_matches_oracle(spec, precision):
    tuned = _plan(spec, precision=precision, autotune=True)
    rep = tuned.tune_report()
    assert "planes <=" in rep
    op = OraclePlan(spec, n_pad=8 if spec.radial == "uniform" else 16)
    rho = _blobs(spec, 4)
    ref = op.solve(rho)
    for _ in range(2):
        phi, info = tuned.solve(_dev(rho), tol=1e-12)
        assert info["converged"]
        assert _l2(spec, phi.cpu().numpy(), ref) < 1e-10


def test_warm_start_schedule():
    """Warm-started solves keep their own schedule: a slowly changing density
    sequence solved with SMG_WARM_PREV through the graph path meets the
    oracle like the host loop does."""
    dyn = _plan(SPEC, launch="dynamic")
    gra = _plan(SPEC, launch="graph")
    op = OraclePlan(SPEC, n_pad=16)
    base = _blobs(SPEC, 5)
    rng = np.random.default_rng(6)
    for k in range(4):
        rho_h = base * (1.0 + 0.01 * k) + 1e-3 * rng.random(base.shape)
        rho = _dev(rho_h)
        a, ia = dyn.solve(rho, tol=1e-11, warm=True)
        b, ib = gra.solve(rho, tol=1e-11, warm=True)
        assert ia["converged"] and ib["converged"]
        ref = op.solve(rho_h)
        assert _l2(SPEC, a.cpu().numpy(), ref) < 1e-9, k
        assert _l2(SPEC, b.cpu().numpy(), ref) < 1e-9, k
