"""Seeded initial parameters for the 8-64-64-3 cost-model network (input data only).

Glorot-uniform weights (Glorot and Bengio, 2010): W ~ U(-a, a) with
a = sqrt(6 / (fan_in + fan_out)); biases start at zero.  Draws come from
SplitMix64 in parameter order.  Flat layout: W1[8][64], b1[64], W2[64][64],
b2[64], W3[64][3], b3[3] (4931 values).
"""

from __future__ import annotations

import math

import numpy as np

from .brickwork import SplitMix64

LAYERS = [(8, 64), (64, 64), (64, 3)]


def glorot_params(seed: int) -> np.ndarray:
    rng = SplitMix64(seed)
    parts = []
    for fan_in, fan_out in LAYERS:
        a = math.sqrt(6.0 / (fan_in + fan_out))
        w = np.array([(2.0 * rng.uniform() - 1.0) * a for _ in range(fan_in * fan_out)])
        parts += [w, np.zeros(fan_out)]
    return np.concatenate(parts)
