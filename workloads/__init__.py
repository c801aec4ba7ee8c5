"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  This module holds no stencil arithmetic: it only draws fields and
weight values from documented recipes, so both the HIP path and the oracle can
consume the same inputs without sharing any of the method's code.

Weights are returned per offset: callers pass the list of (dz, dy, dx)
offsets of their stencil and get one weight per entry, in that order.

Recipes (one per workload; seeds are fixed per workload):
  * uniform [0, 1) fields from numpy's PCG64 generator;
  * a sum of 8 random Fourier modes (periodic x/y, sine in a Dirichlet z)
    plus Gaussian noise of standard deviation 0.01;
  * a Gaussian bump (centre of the grid, sigma = n/8) plus uniform
    [-1e-3, 1e-3) noise;
  * stencil weights: constant, centre/arm, random positive box normalised to
    sum 1, and a multiplicative perturbation for the adjoint target.
"""
from .fields import (  # noqa: F401
    uniform, uniform_into, fourier_modes, fourier_modes_into, gaussian_bump,
    gaussian_bump_into,
)
from .weights import (  # noqa: F401
    const_weights, centre_arm_weights, random_box_weights, perturbed, fp32_rounded,
)
from .configs import CONFIGS, Workload  # noqa: F401
