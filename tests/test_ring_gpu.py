"""General neighbourhoods on the GPU against the oracle: several Chebyshev
rings with the weights of eq (10) (V = 2, 3), rings by squared distance
(PIFCM_SHELL_SQDIST), both eq (7) weightings, other C and m, flat and tiny
volumes, the swarm modes, and the limits."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, check_labels, dev, host, random_memberships_f32, rel

pytestmark = pytest.mark.gpu

SHELL, Q2 = 1, 2


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    from paper_2002_01981_amd import Context
    c = Context(0)
    yield c
    c.close()


def _P(**kw):
    from paper_2002_01981_amd import Params
    return Params(**kw)


def _run(ctx, raw, C, V, h, flags, lam, xi, steps, m=2.0, seed=0):
    rng = np.random.default_rng(seed)
    xo = oracle.normalize(raw)
    xg = ctx.pifcm_normalize(dev(raw))
    assert np.array_equal(host(xg), xo)
    U0 = random_memberships_f32(rng, xo.size, C)
    c0 = np.linspace(0.1, 0.9, C).astype(np.float32)
    g = ctx.ifcm_solve(xg, _P(C=C, m=m, V=V, h=h, eps=0.0, max_iter=steps, flags=flags), lam, xi,
                       c0, U_in=dev(U0), labels=True, want_hist=True)
    o = oracle.solve(xo, c0.astype(np.float64),
                     oracle.Params(C=C, m=m, V=V, h=h, eps=0.0, max_iter=steps, flags=flags),
                     lam, xi, U0=U0.astype(np.float64), want_hist=True)
    assert g["iters"] == o["iters"] == steps
    assert rel(host(g["U"]), o["U"]) <= TOL
    assert rel(g["c"], o["c"]) <= TOL
    assert abs(g["J"] - o["J"]) <= TOL * abs(o["J"])
    assert rel(g["J_hist"], o["J_hist"]) <= TOL
    check_labels(host(g["labels"]), o["U"], C)
    return g, o


@pytest.mark.parametrize("V,h", [(2, 1.0), (2, 0.5), (3, 2.0)])
@pytest.mark.parametrize("lam,xi", [(0.3, 0.4), (0.6, 0.2)])
def test_chebyshev_rings(ctx, V, h, lam, xi):
    raw, _ = synth.random_ellipsoids(shape=(7, 13, 19), seed=90 + V, sigma=0.07)
    _run(ctx, raw, 4, V, h, 0, lam, xi, 4)


@pytest.mark.parametrize("V,flags", [(1, SHELL), (3, SHELL), (3, SHELL | Q2), (6, SHELL),
                                     (12, SHELL), (2, Q2)])
def test_squared_distance_rings_and_weights(ctx, V, flags):
    raw, _ = synth.random_ellipsoids(shape=(6, 11, 15), seed=95, sigma=0.07)
    _run(ctx, raw, 4, V, 1.5, flags, 0.35, 0.3, 4)


def test_sqdist_v3_one_ring_each_matches_weighted_cube(ctx):
    """With V = 3 squared-distance rings (faces, edges, corners of the 3x3x3
    cube) and a huge h, every ring weighs 1/3: a different operator from the
    single Chebyshev ring, and both must match the oracle."""
    raw, _ = synth.random_ellipsoids(shape=(5, 9, 12), seed=96, sigma=0.07)
    g1, _ = _run(ctx, raw, 4, 3, 1e6, SHELL, 0.4, 0.3, 3)
    g2, _ = _run(ctx, raw, 4, 1, 1.0, 0, 0.4, 0.3, 3)
    assert rel(host(g1["U"]), host(g2["U"])) > 1e-6


@pytest.mark.parametrize("C,m", [(3, 2.0), (5, 2.5), (2, 1.5)])
def test_rings_other_c_and_m(ctx, C, m):
    raw, _ = synth.random_ellipsoids(shape=(6, 10, 14), seed=97, sigma=0.07)
    _run(ctx, raw, C, 2, 1.0, 0, 0.3, 0.3, 3, m=m)


def test_two_rings_tiles_split_along_z(ctx):
    """A volume deeper than one tile (45 planes against 32 per tile): the
    planes at a tile's ends take their two planes of context from the
    neighbouring tile's planes."""
    raw, _ = synth.random_ellipsoids(shape=(45, 9, 21), seed=102, sigma=0.07)
    _run(ctx, raw, 4, 2, 1.0, 0, 0.35, 0.3, 3)
    _run(ctx, raw, 3, 2, 0.7, Q2, 0.5, 0.2, 2)


def test_two_rings_volumes_smaller_than_a_tile(ctx):
    """The fused two-ring kernel on a line, a 2 x 3 x 2 block and a single
    plane: most of each ring lies outside the volume."""
    for shape, C, seed in (((1, 1, 5), 2, 103), ((2, 3, 2), 3, 104), ((1, 6, 9), 4, 105)):
        raw = synth.random_ellipsoids(shape=shape, seed=seed, sigma=0.07)[0]
        _run(ctx, raw, C, 2, 1.0, 0, 0.45, 0.3, 3)


def test_rings_flat_and_tiny_volumes(ctx):
    raw = np.zeros((4, 6, 7), np.float32)
    raw[:, :, 4:] = 1.0
    raw[1, 2, 1] = 0.5
    _run(ctx, raw, 3, 2, 1.0, 0, 0.4, 0.4, 3)
    tiny = synth.random_ellipsoids(shape=(2, 2, 3), seed=98, sigma=0.07)[0]
    _run(ctx, tiny, 2, 3, 1.0, 0, 0.5, 0.3, 3)
    one = synth.random_ellipsoids(shape=(1, 1, 5), seed=99, sigma=0.07)[0]
    _run(ctx, one, 2, 2, 1.0, SHELL, 0.5, 0.3, 2)


def test_rings_swarm_modes_and_solve_agree(ctx):
    from paper_2002_01981_amd import PIFCM_SWARM_PLAIN
    shapes = [(6, 12, 20), (5, 17, 9)]
    xs, c0s, U0s = [], [], []
    for b, s in enumerate(shapes):
        raw, _ = synth.random_ellipsoids(shape=s, seed=100 + b, sigma=0.07)
        x = ctx.pifcm_normalize(dev(raw))
        c, U0, _ = ctx.pifcm_fcm_init(x, _P(C=4, m=2.0, eps=0.0, max_iter=5))
        xs.append(x)
        c0s.append(c)
        U0s.append(U0)
    c0s = np.stack(c0s)
    p = _P(C=4, m=2.0, V=2, h=1.0, eps=1e-5, max_iter=12)
    parts = synth.uniform_particles(101, 4)
    bat = ctx.swarm_evaluate(xs, p, parts, c0s, U0s)
    pla = ctx.swarm_evaluate(xs, p, parts, c0s, U0s, mode=PIFCM_SWARM_PLAIN)
    assert np.array_equal(bat["fitness"], pla["fitness"])
    assert np.array_equal(bat["iters"], pla["iters"])
    for b in range(2):
        for q in (0, 3):
            s = ctx.ifcm_solve(xs[b], p, float(parts[q, 0]), float(parts[q, 1]), c0s[b], U_in=U0s[b])
            assert s["J"] == bat["fitness"][b, q]
            assert np.array_equal(s["c"], bat["centres"][b, q])
    assert "nothing timed" in ctx.pifcm_tune(xs, p, 4)


def test_ring_limits(ctx):
    from paper_2002_01981_amd import PifcmError
    from paper_2002_01981_amd.abi import PIFCM_E_UNSUPPORTED
    raw, _ = synth.random_ellipsoids(shape=(4, 6, 8), seed=102, sigma=0.07)
    x = ctx.pifcm_normalize(dev(raw))
    c0 = np.linspace(0.1, 0.9, 4).astype(np.float32)
    for V, flags in ((4, 0), (16, SHELL)):
        with pytest.raises(PifcmError) as e:
            ctx.ifcm_solve(x, _P(C=4, V=V, flags=flags), 0.3, 0.3, c0)
        assert e.value.status == PIFCM_E_UNSUPPORTED
    U0 = dev(random_memberships_f32(np.random.default_rng(0), raw.size, 4))
    with pytest.raises(PifcmError) as e:
        ctx.ifcm_backward(x, _P(C=4, V=2), 0.3, 0.3, c0, U0, 3, 1)
    assert e.value.status == PIFCM_E_UNSUPPORTED


def test_confusion_counts_exact(ctx):
    """pifcm_confusion against numpy on random labels (integer counts: bit
    exact), and the FCM segmentation of the nested phantom against its
    classes."""
    import torch
    from paper_2002_01981_amd import PifcmError
    from paper_2002_01981_amd.quality import misclassification
    rng = np.random.default_rng(5)
    for n, C, K in ((1, 2, 2), (1000, 4, 4), (300001, 16, 5)):
        lab = rng.integers(0, C, n).astype(np.uint8)
        tru = rng.integers(0, K, n).astype(np.uint8)
        got = ctx.pifcm_confusion(dev(lab), dev(tru), C, K)
        ref = np.zeros((C, K), np.int64)
        np.add.at(ref, (lab.astype(int), tru.astype(int)), 1)
        assert np.array_equal(got, ref)
    with pytest.raises(PifcmError):
        ctx.pifcm_confusion(dev(np.array([0, 4], np.uint8)), dev(np.array([0, 1], np.uint8)), 4, 4)
    raw, truth = synth.nested_ellipsoids(shape=(8, 32, 32), seed=1, sigma=0.05)
    x = ctx.pifcm_normalize(dev(raw))
    c0, U0, _ = ctx.pifcm_fcm_init(x, _P(C=4, m=2.0, eps=1e-5, max_iter=50))
    fin = ctx.ifcm_solve(x, _P(C=4, m=2.0, eps=1e-5, max_iter=50), 0.0, 0.0, c0, U_in=U0,
                         labels=True)
    counts = ctx.pifcm_confusion(fin["labels"], dev(truth.reshape(-1)), 4, 4)
    ref = np.mean(host(fin["labels"]) != truth.reshape(-1))
    assert abs(misclassification(counts) - ref) < 1e-15
    assert misclassification(counts) < 0.1
    del torch
