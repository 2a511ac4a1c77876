"""Random streams of the particle swarm search, drawn once on the host.

Algorithm 1 (steps 3-8) starts from a random swarm over (lambda, xi) and
moves each particle with random coefficients.  Both the oracle's PSO and the
library's PSO consume these pre-drawn arrays, so the two searches see the same
random numbers; neither side draws its own.
"""
from __future__ import annotations

import numpy as np


def pso_streams(seed, P, G, dims=2, v0_range=0.1):
    """Initial positions x0 ~ U[0,1)^dims, velocities v0 ~ U[-v0_range,
    v0_range)^dims, and per-generation coefficients r1, r2 ~ U[0,1) of shape
    (G, P, dims).  All float64."""
    rng = np.random.default_rng(seed)
    x0 = rng.random((P, dims))
    v0 = rng.uniform(-v0_range, v0_range, size=(P, dims))
    r1 = rng.random((G, P, dims))
    r2 = rng.random((G, P, dims))
    return dict(x0=x0, v0=v0, r1=r1, r2=r2)


def uniform_particles(seed, P):
    """P particles (lambda, xi) ~ U[0,1)^2 as float32, shape (P, 2)."""
    rng = np.random.default_rng(seed)
    return rng.random((P, 2)).astype(np.float32)
