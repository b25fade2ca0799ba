"""Training the learned initial guess on solves the method itself produces.

All arithmetic runs in the HIP library: the plan records training samples
(network inputs and target changes of the low-m mode planes) while it
solves a sequence of densities warm-started from the previous step, and the
network's own forward/backward kernels and Adam update train on them
(smg_net_train_step).  This module only sequences those calls and holds the
sample buffer (a torch tensor).
"""
import math

import numpy as np

from . import smg


def samples_per_step(m_max):
    """Samples one warm-started solve records (from the third solve of a
    sequence on): 2 multigrid solves x (2 m_max + 1) real images."""
    return 2 * (2 * m_max + 1)


def sample_buffer(plan, capacity, device="cuda"):
    import torch
    return torch.empty(capacity * plan.n_a * plan.n_b * 9, dtype=torch.float32, device=device)


def record_trajectories(plan, trajectories, tol, samples, capacity):
    """Solve every density sequence in `trajectories` (an iterable of
    iterables of cuda float64 densities), the first step of each from zero
    and the rest warm-started, recording samples into `samples`.  Returns
    the number of samples stored and the per-step info dicts."""
    plan.record(samples, capacity)
    infos = []
    for traj in trajectories:
        for k, rho in enumerate(traj):
            _, info = plan.solve(rho, tol=tol, warm=k > 0)
            infos.append(info)
    n = plan.recorded()
    plan.record(None, 0)
    return n, infos


def train(net, samples, n_samples, h, w, steps=1000, batch=16, lr=1e-3, seed=0, log_every=0, log=print):
    """Adam on random minibatches with a cosine learning-rate decay; returns
    the per-step losses."""
    rng = np.random.default_rng(seed)
    losses = []
    for k in range(steps):
        idx = rng.choice(n_samples, size=min(batch, n_samples), replace=False)
        lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps))
        losses.append(net.train_step(samples, idx, h, w, lr_k))
        if log_every and (k + 1) % log_every == 0:
            log(f"train step {k + 1}/{steps}: loss {np.mean(losses[-log_every:]):.3e}")
    return losses


def evaluate(net, samples, n_samples, h, w, count=64, batch=16):
    """Mean training loss over the first `count` samples (fixed batches),
    through the library's training step at learning rate 0; resets the Adam
    moments afterwards (the parameters are unchanged)."""
    count = min(count, n_samples)
    total, k = 0.0, 0
    for q in range(0, count - batch + 1, batch):
        total += net.train_step(samples, np.arange(q, q + batch), h, w, 0.0)
        k += 1
    net.set_params(net.params())
    return total / max(k, 1)


def low_mode_cycles(info, m_max):
    """V-cycles of modes 0..m_max in both multigrid solves of one step."""
    return int(info["cycles1"][: m_max + 1].sum() + info["cycles2"][: m_max + 1].sum())


__all__ = ["samples_per_step", "sample_buffer", "record_trajectories", "train", "evaluate", "low_mode_cycles", "smg"]
