"""Slab mode (Algorithm 1, step 1: one slice with its 3D neighbours) on the
GPU against the oracle: only planes [zbeg, zend) are iterated, the others
hold their initial memberships as context."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, check_labels, dev, host, random_memberships_f32, rel

pytestmark = pytest.mark.gpu


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


def _case(ctx, shape, seed, C=4):
    raw, _ = synth.random_ellipsoids(shape=shape, seed=seed, sigma=0.07)
    xo = oracle.normalize(raw)
    xg = ctx.pifcm_normalize(dev(raw))
    assert np.array_equal(host(xg), xo)
    U0 = random_memberships_f32(np.random.default_rng(seed), xo.size, C)
    return xo, xg, U0


@pytest.mark.parametrize("zbeg,zend", [(0, 1), (5, 6), (11, 12), (3, 9), (0, 12)])
@pytest.mark.parametrize("lam,xi,V", [(0.3, 0.4, 1), (0.0, 0.0, 1), (0.4, 0.2, 2)])
def test_slab_matches_oracle(ctx, zbeg, zend, lam, xi, V):
    xo, xg, U0 = _case(ctx, (12, 21, 37), 110 + zbeg)
    c0 = np.array([0.1, 0.35, 0.6, 0.9], np.float32)
    steps = 4
    g = ctx.ifcm_solve_slab(xg, zbeg, zend, _P(C=4, m=2.0, V=V, eps=0.0, max_iter=steps), lam, xi,
                            c0, dev(U0), labels=True, want_hist=True)
    o = oracle.solve_slab(xo, c0.astype(np.float64),
                          oracle.Params(C=4, m=2.0, V=V, eps=0.0, max_iter=steps), lam, xi,
                          U0.astype(np.float64), zbeg, zend, want_hist=True)
    Ug = host(g["U"])
    assert g["iters"] == o["iters"] == steps
    assert rel(Ug, o["U"]) <= TOL
    assert rel(g["c"], o["c"]) <= TOL
    assert abs(g["J"] - o["J"]) <= TOL * abs(o["J"])
    assert rel(g["J_hist"], o["J_hist"]) <= TOL
    check_labels(host(g["labels"]), o["U"], 4)
    keep = np.ones((12, 21 * 37), bool)
    keep[zbeg:zend] = False
    assert np.array_equal(Ug[keep.reshape(-1)], U0[keep.reshape(-1)])


def test_slab_of_whole_volume_is_the_solve(ctx):
    xo, xg, U0 = _case(ctx, (9, 14, 30), 120)
    c0 = np.array([0.1, 0.35, 0.6, 0.9], np.float32)
    p = _P(C=4, m=2.0, eps=1e-5, max_iter=15)
    a = ctx.ifcm_solve(xg, p, 0.3, 0.3, c0, U_in=dev(U0))
    b = ctx.ifcm_solve_slab(xg, 0, 9, p, 0.3, 0.3, c0, dev(U0))
    assert a["J"] == b["J"] and a["iters"] == b["iters"]
    assert np.array_equal(host(a["U"]), host(b["U"]))


def test_slab_rejects_bad_ranges(ctx):
    from paper_2002_01981_amd import PifcmError
    xo, xg, U0 = _case(ctx, (4, 6, 8), 121)
    c0 = np.array([0.1, 0.35, 0.6, 0.9], np.float32)
    for zb, ze in ((-1, 2), (2, 2), (3, 5)):
        with pytest.raises(PifcmError):
            ctx.ifcm_solve_slab(xg, zb, ze, _P(C=4), 0.3, 0.3, c0, dev(U0))
