"""Seeded initial parameters of the learned-guess network (He-normal 3x3
weights, zero biases, zero output layer) in the packed layer order: weights
(c_out, 9, c_in) then biases per layer, the 1x1 output layer last.  Random
numbers only; the network arithmetic lives in the oracle and the HIP
library."""
import math

import numpy as np


def layer_shapes(levels=4, ch=32, in_ch=8):
    shapes = []
    cin = in_ch
    for _ in range(levels):
        shapes += [("conv3", cin, ch), ("conv3", ch, ch)]
        cin = ch
    for _ in range(levels - 1):
        shapes += [("conv3", 2 * ch, ch), ("conv3", ch, ch)]
    shapes.append(("conv1", ch, 1))
    return shapes


def init_params(seed, levels=4, ch=32, in_ch=8, zero_output=True):
    rng = np.random.default_rng(seed)
    parts = []
    for kind, ci, co in layer_shapes(levels, ch, in_ch):
        fan_in = ci * (9 if kind == "conv3" else 1)
        nw = co * fan_in
        if kind == "conv1" and zero_output:
            w = np.zeros(nw)
        else:
            w = rng.normal(0.0, math.sqrt(2.0 / fan_in), nw)
        parts += [w, np.zeros(co)]
    return np.concatenate(parts)
