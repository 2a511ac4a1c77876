"""The hand-written adjoint (ifcm_backward) against central finite
differences of the FP64 oracle.

J_K is the objective of eq (1) after exactly K iterations from a fixed U^0;
its gradient with respect to lambda, xi and the initial centres is compared
norm-wise (max component error over the largest component) with the
oracle's central differences at h = 1e-4.  All points keep lambda + xi <=
0.9, so the 1e-12 floor of the squared distance never engages and J_K is
smooth there.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    from paper_2002_01981_amd import Context
    c = Context(0)
    yield c
    c.close()


def _case(shape, C, seed, m=2.0):
    raw, _ = synth.random_ellipsoids(shape=shape, seed=seed, sigma=0.07)
    x = oracle.normalize(raw)
    c0, U0, _ = oracle.fcm_init(x, oracle.Params(C=C, m=m, eps=0.0, max_iter=8))
    # both sides start from the same float32 state
    return x, c0.astype(np.float32), U0.astype(np.float32)


def _gpu_grad(ctx, x, c0, U0, C, m, lam, xi, K, s):
    from paper_2002_01981_amd import Params
    g = ctx.ifcm_backward(dev(x), Params(C=C, m=m), lam, xi, c0, dev(U0), K, s)
    return g["J"], np.concatenate([[g["dlam"], g["dxi"]], g["dc"]])


def _fd(x, c0, U0, C, m, lam, xi, K):
    J, g = oracle.fd_grad(x, c0.astype(np.float64), U0.astype(np.float64),
                          oracle.Params(C=C, m=m), lam, xi, K=K, step=1e-4)
    return J, g


@pytest.mark.parametrize("lam,xi", [(0.2, 0.3), (0.4, 0.1), (0.1, 0.6)])
@pytest.mark.parametrize("K", [1, 5, 12])
def test_gradient_matches_finite_differences(ctx, lam, xi, K):
    C = 4
    x, c0, U0 = _case((10, 14, 22), C, seed=50)
    Jg, gg = _gpu_grad(ctx, x, c0, U0, C, 2.0, lam, xi, K, max(1, K // 3))
    Jo, go = _fd(x, c0, U0, C, 2.0, lam, xi, K)
    assert abs(Jg - Jo) <= 1e-4 * abs(Jo)
    err = np.max(np.abs(gg - go)) / np.max(np.abs(go))
    assert err <= GRAD_TOL, (gg, go, err)


@pytest.mark.parametrize("K,strides", [(9, (1, 2, 4, 9)), (11, (1, 3, 4, 5, 11))])
def test_checkpoint_stride_does_not_change_the_gradient(ctx, K, strides):
    """Any checkpoint stride gives the same gradient bit for bit, including
    strides whose last segment is partial and holds several states (K = 11
    with strides 3, 4, 5: the forward pass leaves those states for the
    reverse sweep instead of their recomputation)."""
    C = 4
    x, c0, U0 = _case((8, 12, 20), C, seed=51)
    ref = None
    for s in strides:
        J, g = _gpu_grad(ctx, x, c0, U0, C, 2.0, 0.3, 0.2, K, s)
        if ref is None:
            ref = (J, g)
        else:
            assert J == ref[0], s
            assert np.array_equal(g, ref[1]), s


def test_gradient_partial_last_segment_against_oracle(ctx):
    """K = 11 with checkpoints every 4: segments of 4, 4 and 3 iterations,
    against central differences of the oracle."""
    C, K = 4, 11
    x, c0, U0 = _case((10, 14, 22), C, seed=53)
    Jg, gg = _gpu_grad(ctx, x, c0, U0, C, 2.0, 0.25, 0.35, K, 4)
    Jo, go = _fd(x, c0, U0, C, 2.0, 0.25, 0.35, K)
    assert abs(Jg - Jo) <= 1e-4 * abs(Jo)
    err = np.max(np.abs(gg - go)) / np.max(np.abs(go))
    assert err <= GRAD_TOL, (gg, go, err)


@pytest.mark.parametrize("C,m", [(3, 2.0), (4, 2.5)])
def test_gradient_other_cluster_counts_and_fuzziness(ctx, C, m):
    x, c0, U0 = _case((8, 10, 18), C, seed=52, m=m)
    Jg, gg = _gpu_grad(ctx, x, c0, U0, C, m, 0.25, 0.35, 6, 2)
    Jo, go = _fd(x, c0, U0, C, m, 0.25, 0.35, 6)
    assert abs(Jg - Jo) <= 1e-4 * abs(Jo)
    assert np.max(np.abs(gg - go)) / np.max(np.abs(go)) <= GRAD_TOL


def test_gradient_brain_crop(ctx):
    """The brain-shaped workload (a crop, so the oracle's twelve K-step solves
    stay quick): K = 30 with checkpoints every 5 iterations."""
    raw, _ = synth.brain_shells(shape=(24, 40, 36), seed=5, noise_frac=0.05)
    x = oracle.normalize(raw)
    c0, U0, _ = oracle.fcm_init(x, oracle.Params(C=4, m=2.0, eps=0.0, max_iter=10))
    c0, U0 = c0.astype(np.float32), U0.astype(np.float32)
    for lam, xi in ((0.2, 0.3), (0.4, 0.1), (0.1, 0.6)):
        Jg, gg = _gpu_grad(ctx, x, c0, U0, 4, 2.0, lam, xi, 30, 5)
        Jo, go = _fd(x, c0, U0, 4, 2.0, lam, xi, 30)
        assert abs(Jg - Jo) <= 1e-4 * abs(Jo)
        assert np.max(np.abs(gg - go)) / np.max(np.abs(go)) <= GRAD_TOL, (lam, xi, gg, go)


def test_gradient_flat_block_tiny_volume_and_more_clusters(ctx):
    """A constant block inside a noisy volume (its interior voxels have flat
    neighbourhoods: g_inv < 0, eq (5) becomes the mean), a volume smaller
    than one wave tile in every direction, and C = 6."""
    rng = np.random.default_rng(54)
    raw, _ = synth.random_ellipsoids(shape=(7, 11, 13), seed=54, sigma=0.07)
    raw[1:6, 2:8, 3:9] = 0.37
    for raw_c, C, s in ((raw, 4, 3), (rng.random((3, 2, 5)).astype(np.float32), 3, 2), (raw, 6, 2)):
        x = oracle.normalize(raw_c)
        c0, U0, _ = oracle.fcm_init(x, oracle.Params(C=C, m=2.0, eps=0.0, max_iter=8))
        c0, U0 = c0.astype(np.float32), U0.astype(np.float32)
        Jg, gg = _gpu_grad(ctx, x, c0, U0, C, 2.0, 0.3, 0.25, 6, s)
        Jo, go = _fd(x, c0, U0, C, 2.0, 0.3, 0.25, 6)
        assert abs(Jg - Jo) <= 1e-4 * abs(Jo), (raw_c.shape, C, Jg, Jo)
        assert np.max(np.abs(gg - go)) / np.max(np.abs(go)) <= GRAD_TOL, (raw_c.shape, C, gg, go)
