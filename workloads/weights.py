"""Stencil weight recipes.  Each takes the caller's list of (dz, dy, dx)
offsets and returns one FP64 weight per offset, in the same order."""
import numpy as np


def const_weights(offsets, value):
    return np.full(len(offsets), float(value))


def centre_arm_weights(offsets, centre, arms):
    """centre for (0,0,0); arms[d-1] for a point at distance d along one axis."""
    w = []
    for o in offsets:
        d = max(abs(int(c)) for c in o)
        nonzero = sum(int(c) != 0 for c in o)
        if nonzero == 0:
            w.append(float(centre))
        elif nonzero == 1:
            w.append(float(arms[d - 1]))
        else:
            raise ValueError("centre/arm weights are for star stencils")
    return np.array(w)


def random_box_weights(offsets, seed):
    """w_raw = 0.5 + U[0,1) per offset (drawn in the given order from
    PCG64(seed)), normalised to sum 1 in FP64."""
    rng = np.random.default_rng(seed)
    raw = 0.5 + rng.random(len(offsets))
    return raw / raw.sum()


def perturbed(weights, seed, rel=0.01):
    """w * (1 + U[-rel, rel)) per weight from PCG64(seed); not renormalised."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)
    return w * (1.0 + rng.uniform(-rel, rel, w.shape))


def fp32_rounded(weights):
    """The weights as an FP32 kernel sees them, promoted back to FP64."""
    return np.asarray(weights, dtype=np.float64).astype(np.float32).astype(np.float64)
