"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This package only *draws* inputs: phantom volumes (raw, not normalised),
their ground-truth class maps, volume shapes for ragged batches, PSO particle
positions and the PSO random streams.  It holds none of the clustering
method's arithmetic (no normalisation, no memberships, no centres), so both
sides of every parity test can consume exactly the same bytes.
"""
from .phantoms import (  # noqa: F401
    nested_ellipsoids,
    random_ellipsoids,
    brain_shells,
    ragged_dims,
    ragged_batch,
    WORKLOADS,
)
from .streams import pso_streams, uniform_particles  # noqa: F401
