"""The learned-guess step inside a solve (smg_net_guess_step) against its
oracle (oracle/net.py guess_images, the network forward, guess_candidate,
guess_judge), and a trained-network trajectory against the oracle's exact
solves.

* Inputs: the GPU forms them in FP64 and stores FP32, the oracle in FP64;
  they agree to one FP32 rounding (2^-24 relative, 2^-23 allowed for the
  RMS computed in another order).
* Network output: both sides round every stored activation to BF16 (the
  GPU from an FP32 sum, the oracle from an FP64 sum); a sum within FP32
  rounding of a BF16 rounding boundary can round the other way and the
  flipped ulp propagates, so the output is held to 1e-2 relative L2 (the
  layers themselves are checked element by element in test_gpu_layers).
* Candidate and judge: with a network whose output is a constant (zero
  output weights, a bias), both sides build the same candidate to FP64
  rounding and the judge's decisions are clear-cut; each mode's start
  must then equal the oracle's choice element by element (1e-12), and a
  mode that keeps the previous solution must return it bit for bit."""
import math

import numpy as np
import pytest

from oracle import net as onet
from oracle.geometry import GridSpec, cell_centres, cell_volumes_3d
from oracle.multigrid import MGLevel
from oracle.solve import OraclePlan
from workloads import configs
from workloads.densities import keplerian_snapshot
from workloads.netinit import init_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPEC = GridSpec("spherical", "log", 64, 32, 16, 0.05, 5.0, 0.0, math.pi)
M_MAX = 4

_cache = {}


def _setup():
    if "p" not in _cache:
        from paper_2606_17636_amd import smg
        print(f"[setup] {SPEC}", flush=True)
        plan = smg.grid_from_spec(SPEC, precision="mixed").setup()
        net = smg.Net()
        plan.attach_net(net, M_MAX)
        op = OraclePlan(SPEC, dgf=np.zeros((SPEC.n_modes, 1, 1)))
        a, b, p = cell_centres(SPEC)
        blobs = configs.c5_blobs(5)
        dt = 0.5 * (2 * math.pi / SPEC.n_phi) / (blobs[0].min() ** -1.5)
        f0 = op.source_modes(keplerian_snapshot(a, b, p, blobs, 0.0))
        f1 = op.source_modes(keplerian_snapshot(a, b, p, blobs, dt))
        fm = op.source_modes(keplerian_snapshot(a, b, p, blobs, -dt))
        u0 = op.solve_modes(f0)
        u1 = op.solve_modes(f1)
        um = op.solve_modes(fm)
        _cache.update(p=plan, net=net, op=op, f0=f0, f1=f1, u0=u0, u1=u1, um=um)
    return _cache


def _dev(z):
    return torch.from_numpy(np.ascontiguousarray(z[:M_MAX + 1])).cuda()


def test_guess_inputs_and_network_output_match_oracle():
    c = _setup()
    params = init_params(21, zero_output=False)
    c["net"].set_params(params)
    for t, u2 in ((0, None), (1, c["um"])):
        print(f"[case] inputs and output, t={t}, two steps back: {u2 is not None}", flush=True)
        guess, x, y, used = c["p"].net_guess_step(t, _dev(c["f1"]), _dev(c["f0"]), _dev(c["u0"]),
                                                  None if u2 is None else _dev(u2))
        x = x.cpu().numpy().astype(np.float64)
        y = y.cpu().numpy().astype(np.float64)
        xo, sc = onet.guess_images(c["f1"], c["f0"], c["u0"], M_MAX, uprev2=u2)
        err = np.abs(x - xo)
        bound = 2.0**-23 * np.abs(xo) + 2.0**-126      # one FP32 rounding; FP32 underflow
        bad = np.argwhere(err > bound)
        for k, i, j, ch in bad[:8]:
            print("mismatch at image", k, "cell", (i, j), "channel", ch, "gpu", x[k, i, j, ch], "oracle",
                  xo[k, i, j, ch], "scales", sc[k], flush=True)
        assert len(bad) == 0
        yo, _ = onet.forward(params.astype(np.float32).astype(np.float64), xo.astype(np.float32).astype(np.float64))
        rel = np.linalg.norm(y - yo) / np.linalg.norm(yo)
        print("network output rel L2", rel, flush=True)
        assert rel < 1e-2
        assert used.shape == (M_MAX + 1,)


def _constant_output_params(bias):
    p = init_params(22, zero_output=True)
    p[-1] = bias                         # the output layer's bias: y = bias everywhere
    return p


def test_guess_candidate_and_judge_match_oracle():
    c = _setup()
    bias = 2.0
    c["net"].set_params(_constant_output_params(bias))
    lev = MGLevel(SPEC, 0)
    rng = np.random.default_rng(24)
    for t, (f, fp, ut) in enumerate(((c["f1"], c["f0"], c["u1"]), (c["f1"] * 0.7, c["f0"] * 0.7, c["u1"] * 0.7))):
        # previous solutions: the exact solution of f for modes 1 and 3; for
        # modes 0, 2, 4 the exact solution minus what the candidate adds back,
        # so the candidate is the better start there and the worse one
        # elsewhere.  t = 0: no solution two steps back, the candidate adds
        # s_o(uprev) * bias (a fixed point in uprev); t = 1: uprev2 = uprev -
        # delta, the candidate adds delta + RMS(delta) * bias
        up = np.array(ut[:M_MAX + 1])
        up2 = None
        if t == 1:
            delta = 1e-3 * np.abs(ut).max() * (rng.standard_normal(up.shape) + 1j * rng.standard_normal(up.shape))
            delta[0] = delta[0].real
            rms = lambda v: float(np.sqrt(np.mean(v * v)))
            for m in (0, 2, 4):
                up[m] = ut[m] - delta[m] - bias * rms(delta[m].real)
                if m:
                    up[m] -= 1j * bias * rms(delta[m].imag)
            up2 = up - delta
        else:
            for _ in range(30):
                _, sc = onet.guess_images(f, fp, up, M_MAX)
                for m in (0, 2, 4):
                    kr = 0 if m == 0 else 2 * m - 1
                    shift = sc[kr, 3] * bias + (1j * sc[2 * m, 3] * bias if m else 1j * 0.0)
                    up[m] = ut[m] - shift
                    if m == 0:
                        up[0] = up[0].real + 1j * ut[0].imag
        print(f"[case] candidate and judge, t={t}", flush=True)
        guess, _, y, used = c["p"].net_guess_step(t, _dev(f), _dev(fp), _dev(up), None if up2 is None else _dev(up2))
        assert np.all(y.cpu().numpy() == np.float32(bias))
        _, sc = onet.guess_images(f, fp, up, M_MAX, uprev2=up2)
        cand = onet.guess_candidate(up, np.full((2 * M_MAX + 1,) + up.shape[1:], bias), sc, M_MAX, uprev2=up2)
        base = onet.guess_base(up, sc, M_MAX, uprev2=up2)
        uo, nc, nu = onet.guess_judge(lev, f, cand, base, M_MAX)
        margin = np.abs(nc - nu) / np.maximum(nc, nu)
        print("oracle judge", list(uo), "margins", margin, "gpu", list(used), flush=True)
        assert list(uo) == [1, 0, 1, 0, 1] and np.all(margin > 0.1)
        assert list(used) == list(uo)
        g = guess.cpu().numpy()
        for m in range(M_MAX + 1):
            ref = cand[m] if uo[m] else base[m]
            assert np.abs(g[m] - ref).max() <= 1e-12 * np.abs(ref).max(), m


def test_untrained_network_extrapolates():
    """With a zero output layer the candidate is the judge's baseline, the
    linear extrapolation of the last two solutions 2 u_{t-1} - u_{t-2}
    (u_{t-1} on static parts: m = 0 of the orbiting blobs does not change);
    on a smooth trajectory it is a better start than u_{t-1} for the modes
    that change (m >= 1 here), and the step returns it to FP64 rounding."""
    c = _setup()
    c["net"].set_params(init_params(23, zero_output=True))
    lev = MGLevel(SPEC, 0)
    print("[case] untrained network, extrapolation", flush=True)
    guess, _, y, used = c["p"].net_guess_step(0, _dev(c["f1"]), _dev(c["f0"]), _dev(c["u0"]), _dev(c["um"]))
    assert np.all(y.cpu().numpy() == 0.0)
    _, sc = onet.guess_images(c["f1"], c["f0"], c["u0"], M_MAX, uprev2=c["um"])
    cand = onet.guess_candidate(c["u0"], np.zeros((2 * M_MAX + 1,) + c["u0"].shape[1:]), sc, M_MAX, uprev2=c["um"])
    base = onet.guess_base(c["u0"], sc, M_MAX, uprev2=c["um"])
    assert np.array_equal(cand, base)
    g = guess.cpu().numpy()
    for m in range(M_MAX + 1):
        assert np.abs(g[m] - cand[m]).max() <= 1e-13 * np.abs(cand[m]).max(), m
    # the extrapolation against the previous solution, after one smoothing step of each
    uo, nc, nu = onet.guess_judge(lev, c["f1"], cand, c["u0"][:M_MAX + 1], M_MAX)
    print("extrapolation vs previous solution", list(uo), "norms", nc, nu, "gpu", list(used), flush=True)
    assert list(uo[1:]) == [1] * M_MAX


def test_trained_trajectory_matches_oracle():
    """A network trained on recorded trajectories, then a held-out trajectory
    solved warm with SMG_NET_GUESS (chosen form: mixed precision, graphs):
    every snapshot's Phi agrees with the oracle's exact solve of that
    snapshot's density within the mixed-precision bound (1e-6 relative L2 at
    rel. residual 1e-8), whichever start each mode took."""
    from paper_2606_17636_amd import learn, smg
    from workloads.densities import keplerian_snapshot_device
    spec = GridSpec("spherical", "log", 64, 32, 32, 0.05, 5.0, 0.0, math.pi)
    a, b, p = cell_centres(spec)
    dt = 0.5 * (2 * math.pi / spec.n_phi) / (configs.c5_blobs(5)[0].min() ** -1.5)

    def traj(seed, steps, t0=0.0):
        blobs = configs.c5_blobs(seed)
        return [keplerian_snapshot_device(a, b, p, blobs, t0 + k * dt) for k in range(steps)]

    net = smg.Net()
    net.set_params(init_params(2))
    print(f"[setup] trajectory {spec}", flush=True)
    rec = smg.grid_from_spec(spec, precision="fp64").setup().attach_net(net, M_MAX)
    steps = 16
    cap = 3 * (steps - 2) * learn.samples_per_step(M_MAX)
    buf = learn.sample_buffer(rec, cap)
    n, _ = learn.record_trajectories(rec, [traj(s, steps) for s in (50, 51, 52)], 1e-10, buf, cap)
    learn.train(net, buf, n, spec.n_a, spec.n_b, steps=300, batch=16, lr=1e-3, seed=3)
    plan = smg.grid_from_spec(spec, precision="mixed", launch="graph", coarse_cells=2048,
                              nu_pre=smg.NU_AUTO, nu_post=smg.NU_AUTO).setup().attach_net(net, M_MAX)
    op = OraclePlan(spec)
    blobs = configs.c5_blobs(5)
    w = cell_volumes_3d(spec)[:, :, None]
    used = 0
    for k in range(10):
        rho = keplerian_snapshot(a, b, p, blobs, 0.3 + k * dt)
        phi, info = plan.solve(torch.from_numpy(rho).cuda(), tol=1e-8, warm=k > 0, net=True)
        assert info["converged"], k
        if k >= 2:
            used += int(plan.net_used().sum())
        if k in (2, 5, 9):
            ref = op.solve(rho)
            err = math.sqrt(np.sum((phi.cpu().numpy() - ref) ** 2 * w) / np.sum(ref**2 * w))
            print(f"snapshot {k}: rel L2 vs oracle {err:.2e}", flush=True)
            assert err < 1e-6, k
    print("modes taking the network's guess", used, flush=True)
