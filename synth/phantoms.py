"""Seeded phantom volumes that stand in for the paper's datasets.

The paper times its method on a synthetic "cube in a cube" set resized to
32x32 ... 854x854 (section 6.2) and on a Brainweb T1 volume of 181x217 slices
(section 6.3).  Neither dataset is available here, so these generators draw
volumes with the same shapes, class counts and noise model from a numpy PCG64
stream.  Every volume is returned *raw* (not normalised): min-max
normalisation is a step of the method (Algorithm 2, step 1) and lives on
each side of a parity test separately.

Arrays are float32 with shape (Z, Y, X), X fastest.  Coordinates of voxel
centres are mapped to the open cube (-1, 1)^3 with u = 2 (i + 1/2) / n - 1.
Each generator also returns the ground-truth class map (uint8, 0 = background).
"""
from __future__ import annotations

import numpy as np

CLASS_INTENSITY = np.array([0.0, 0.3, 0.6, 0.9], dtype=np.float64)


def _axes(shape):
    z, y, x = shape
    uz = (2.0 * (np.arange(z) + 0.5) / z - 1.0)[:, None, None]
    uy = (2.0 * (np.arange(y) + 0.5) / y - 1.0)[None, :, None]
    ux = (2.0 * (np.arange(x) + 0.5) / x - 1.0)[None, None, :]
    return uz, uy, ux


def _index_range(lo, hi, n):
    """Voxel indices whose centre coordinate u lies in [lo, hi]."""
    i0 = int(np.floor(((lo + 1.0) * n) / 2.0 - 0.5))
    i1 = int(np.ceil(((hi + 1.0) * n) / 2.0 - 0.5))
    return max(i0, 0), min(i1 + 1, n)


def nested_ellipsoids(shape=(8, 32, 32), seed=1, sigma=0.05):
    """Background 0 plus three nested ellipsoids (radii 0.8 / 0.55 / 0.3 in
    normalised coordinates, centred at 0) at intensities 0.3 / 0.6 / 0.9, with
    additive N(0, sigma^2) noise.  Returns (raw float32 volume, labels)."""
    rng = np.random.default_rng(seed)
    uz, uy, ux = _axes(shape)
    r2 = ux * ux + uy * uy + uz * uz
    labels = np.zeros(shape, dtype=np.uint8)
    for cls, rad in ((1, 0.8), (2, 0.55), (3, 0.3)):
        labels[np.broadcast_to(r2 <= rad * rad, shape)] = cls
    clean = CLASS_INTENSITY[labels]
    noise = rng.normal(0.0, sigma, size=shape)
    return (clean + noise).astype(np.float32), labels


def random_ellipsoids(shape=(16, 854, 854), seed=2, sigma=0.07, count=40):
    """Four-class random tissue map: background 0 plus `count` rotated
    ellipsoids painted in order (centres U(-0.9, 0.9)^3, in-plane semi-axes
    U(0.05, 0.3), z semi-axis U(0.3, 1.0), rotation about z U(0, pi), class
    uniform in {1, 2, 3}; the first three ellipsoids carry one class each so
    every class is drawn), plus N(0, sigma^2) noise."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.9, 0.9, size=(count, 3))        # (x, y, z)
    semi_xy = rng.uniform(0.05, 0.3, size=(count, 2))
    semi_z = rng.uniform(0.3, 1.0, size=count)
    theta = rng.uniform(0.0, np.pi, size=count)
    classes = rng.integers(1, 4, size=count)
    classes[:3] = rng.permutation([1, 2, 3])
    z, y, x = shape
    labels = np.zeros(shape, dtype=np.uint8)
    uz_all, uy_all, ux_all = _axes(shape)
    for e in range(count):
        cx, cy, cz = centres[e]
        a, b = semi_xy[e]
        c = semi_z[e]
        reach = max(a, b)
        x0, x1 = _index_range(cx - reach, cx + reach, x)
        y0, y1 = _index_range(cy - reach, cy + reach, y)
        z0, z1 = _index_range(cz - c, cz + c, z)
        if x0 >= x1 or y0 >= y1 or z0 >= z1:
            continue
        dx = ux_all[:, :, x0:x1] - cx
        dy = uy_all[:, y0:y1, :] - cy
        dz = uz_all[z0:z1, :, :] - cz
        ct, st = np.cos(theta[e]), np.sin(theta[e])
        px = ct * dx + st * dy
        py = -st * dx + ct * dy
        inside = (px / a) ** 2 + (py / b) ** 2 + (dz / c) ** 2 <= 1.0
        sub = labels[z0:z1, y0:y1, x0:x1]
        sub[inside] = classes[e]
    clean = CLASS_INTENSITY[labels]
    noise = rng.normal(0.0, sigma, size=shape)
    return (clean + noise).astype(np.float32), labels


def _smooth_direction_field(rng, nx, ny, nz):
    """Low-order function of the unit direction, scaled to max |s| = 1 on a
    fixed sample of directions."""
    coef = rng.normal(0.0, 1.0, size=9)

    def f(ax, ay, az):
        terms = (ax, ay, az, ax * ax - ay * ay, ay * ay - az * az,
                 ax * ay, ay * az, az * ax, ax * ay * az)
        return sum(k * t for k, t in zip(coef, terms))

    g = np.random.default_rng(12345).normal(size=(4096, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    scale = np.max(np.abs(f(g[:, 0], g[:, 1], g[:, 2])))
    return f(nx, ny, nz) / scale


def brain_shells(shape=(181, 217, 181), seed=3, noise_frac=0.05,
                 bias_amp=0.2, boundary_amp=0.05):
    """Brain-shaped nested shells: head ellipsoid (0.9, 0.9, 0.85) = CSF 0.25,
    (0.8, 0.8, 0.75) = GM 0.55, core (0.6, 0.6, 0.55) = WM 0.8, background 0.
    The GM and WM boundaries get a seeded low-order radial perturbation of
    relative amplitude `boundary_amp`; the clean image is multiplied by a
    smooth bias field 1 + bias_amp * p(u) / max|p| with p a degree-2
    polynomial with N(0, 1) coefficients; then N(0, (noise_frac * 0.8)^2)
    noise is added ("percent of the brightest clean tissue")."""
    rng = np.random.default_rng(seed)
    uz, uy, ux = _axes(shape)
    ux, uy, uz = np.broadcast_arrays(ux, uy, uz)
    rad = np.sqrt(ux * ux + uy * uy + uz * uz) + 1e-12
    nx, ny, nz = ux / rad, uy / rad, uz / rad
    s_gm = _smooth_direction_field(rng, nx, ny, nz)
    s_wm = _smooth_direction_field(rng, nx, ny, nz)

    def rho(axes):
        return np.sqrt((ux / axes[0]) ** 2 + (uy / axes[1]) ** 2 + (uz / axes[2]) ** 2)

    labels = np.zeros(shape, dtype=np.uint8)
    labels[rho((0.9, 0.9, 0.85)) <= 1.0] = 1
    labels[rho((0.8, 0.8, 0.75)) <= 1.0 + boundary_amp * s_gm] = 2
    labels[rho((0.6, 0.6, 0.55)) <= 1.0 + boundary_amp * s_wm] = 3
    intensity = np.array([0.0, 0.25, 0.55, 0.8])
    clean = intensity[labels]
    pc = rng.normal(0.0, 1.0, size=10)
    p = (pc[0] + pc[1] * ux + pc[2] * uy + pc[3] * uz + pc[4] * ux * ux
         + pc[5] * uy * uy + pc[6] * uz * uz + pc[7] * ux * uy
         + pc[8] * uy * uz + pc[9] * uz * ux)
    bias = 1.0 + bias_amp * p / np.max(np.abs(p))
    noise = rng.normal(0.0, noise_frac * 0.8, size=shape)
    return (clean * bias + noise).astype(np.float32), labels


def ragged_dims(seed=4, count=6, xy=(64, 256), z=(64, 128)):
    """Shapes (Z, Y, X) of a ragged batch: X, Y uniform in xy, Z uniform in z
    (inclusive bounds)."""
    rng = np.random.default_rng(seed)
    xs = rng.integers(xy[0], xy[1] + 1, size=count)
    ys = rng.integers(xy[0], xy[1] + 1, size=count)
    zs = rng.integers(z[0], z[1] + 1, size=count)
    return [(int(zz), int(yy), int(xx)) for xx, yy, zz in zip(xs, ys, zs)]


def ragged_batch(seed=4, count=6, sigma=0.07, dims=None):
    """A ragged batch of random-ellipsoid volumes.  Returns a list of
    (raw volume, labels) pairs."""
    if dims is None:
        dims = ragged_dims(seed, count)
    return [random_ellipsoids(shape=d, seed=seed * 1000 + b, sigma=sigma)
            for b, d in enumerate(dims)]


# The workloads, named by what they are.  Shapes are (Z, Y, X).
WORKLOADS = {
    "nested-32x32x8": dict(kind="nested", shape=(8, 32, 32), seed=1, sigma=0.05,
                           C=4, m=2.0, eps=1e-5, max_iter=50,
                           pso=dict(P=8, G=5, seed=101, w=0.7, c1=1.5, c2=1.5)),
    "ellipsoids-854x854x16": dict(kind="ellipsoids", shape=(16, 854, 854), seed=2,
                                  sigma=0.07, C=4, m=2.0, eps=1e-5, max_iter=100,
                                  pso=dict(P=20, G=20, seed=102, w=0.7, c1=1.5, c2=1.5)),
    "brain-181x217x181": dict(kind="brain", shape=(181, 217, 181), seed=3,
                              noise_frac=0.05, C=4, m=2.0, eps=1e-5, max_iter=100,
                              pso=dict(P=20, G=20, seed=103, w=0.7, c1=1.5, c2=1.5)),
    "ragged6-swarm64": dict(kind="ragged", seed=4, count=6, sigma=0.07, C=4, m=2.0,
                            eps=0.0, iters=20, particles=64, particle_seed=104),
    "adjoint-brain-K30": dict(kind="brain", shape=(181, 217, 181), seed=5,
                              noise_frac=0.05, C=4, m=2.0, K=30, ckpt=5,
                              points=((0.2, 0.3), (0.4, 0.1), (0.1, 0.6)),
                              pso=dict(P=32, G=10, seed=105, w=0.7, c1=1.5, c2=1.5)),
}
