"""Seeded initial parameters of the tolerance network (input preparation).

A 6 -> 64 -> 64 -> 1 network whose parameter vector is laid out as
W1 [64][6], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1].  Weights are
drawn uniformly in +-sqrt(6 / fan_in) (He-uniform, suited to ReLU layers),
hidden biases start at zero, and the output bias starts so that the initial
tolerance is about `eps0` px (b3 = log(exp(eps0) - 1)).
"""

import numpy as np

SHAPES = ((64, 6), (64,), (64, 64), (64,), (64,), (1,))
NPARAM = 4673


def mlp_init(seed, eps0=2.0):
    rng = np.random.default_rng(seed)
    parts = []
    for shape in SHAPES:
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape))
        else:
            parts.append(np.zeros(shape))
    w3_lim = np.sqrt(6.0 / 64.0) * 0.1
    parts[4] = rng.uniform(-w3_lim, w3_lim, size=64)
    parts[5] = np.array([np.log(np.expm1(eps0))])
    theta = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert theta.size == NPARAM
    return theta
