"""Work decompositions of the fused step through the C ABI.

pifcm_set_decomposition picks waves per work group, planes per tile and
particles per work item by hand (the tuner picks among the same).  Two
particles per work item share the volume's intensities, g_inv and every
|x_i - x_k|, and do each particle's arithmetic in the same order as one
particle per item: results must not change by a single bit -- with a swarm
whose particle count is odd (a last item with one particle) and a stop rule
under which particles stop at different iterations (items with one live and
one stopped particle).  Lone solves with the same tiles are the reference,
and they in turn are held to the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, dev, host, rel

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


def _volumes(ctx):
    out = []
    for shape, seed in (((13, 37, 29), 501), ((20, 18, 45), 502)):
        raw, _ = synth.random_ellipsoids(shape=shape, seed=seed, sigma=0.07, count=12)
        xo = oracle.normalize(raw)
        xg = ctx.pifcm_normalize(dev(raw))
        assert np.array_equal(host(xg), xo)
        c0, U0, _ = ctx.pifcm_fcm_init(xg, _P(C=4, m=2.0, eps=1e-5, max_iter=50))
        out.append((xo, xg, c0, U0))
    return out


@pytest.mark.parametrize("nw,zc", [(4, 32), (2, 8), (1, 16), (4, 128)])
def test_two_particles_per_item_change_nothing(ctx, nw, zc):
    vols = _volumes(ctx)
    xg = [v[1] for v in vols]
    c0s = np.stack([v[2] for v in vols])
    U0s = [v[3] for v in vols]
    P = 5
    parts = np.ascontiguousarray(np.broadcast_to(synth.uniform_particles(77, P), (2, P, 2)))
    p = _P(C=4, m=2.0, eps=1e-4, max_iter=25)
    ctx.pifcm_set_decomposition(xg, p, nw, zc, 1)
    one = ctx.swarm_evaluate(xg, p, parts, c0s, U0s)
    ctx.pifcm_set_decomposition(xg, p, nw, zc, 2)
    two = ctx.swarm_evaluate(xg, p, parts, c0s, U0s)
    print(f"nw={nw} zc={zc} iterations per pair {two['iters'].tolist()}", flush=True)
    assert len(set(two["iters"].ravel().tolist())) > 1, "every pair stopped together"
    assert np.array_equal(one["fitness"], two["fitness"])
    assert np.array_equal(one["centres"], two["centres"])
    assert np.array_equal(one["iters"], two["iters"])
    for b in range(2):
        for q in range(P):
            lam, xi = (float(v) for v in parts[b, q])
            s = ctx.ifcm_solve(xg[b], p, lam, xi, c0s[b], U_in=U0s[b])
            assert s["J"] == two["fitness"][b, q] and s["iters"] == two["iters"][b, q]
            assert np.array_equal(s["c"], two["centres"][b, q])


def test_two_particles_per_item_memberships(ctx):
    """The memberships the two-particle items write, read back through the
    interleaved swarm (each particle carries its own state; a frozen swarm
    keeps its positions), equal lone solves bit for bit and the oracle to the
    bar."""
    vols = _volumes(ctx)
    xo, xg, c0, U0 = vols[0]
    P, G, steps = 4, 2, 3
    st = synth.pso_streams(91, P, G)
    st = dict(x0=np.array([[0.2, 0.3], [0.5, 0.1], [0.1, 0.6], [0.35, 0.35]]),
              v0=np.zeros_like(st["v0"]), r1=np.zeros_like(st["r1"]), r2=np.zeros_like(st["r2"]))
    p = _P(C=4, m=2.0, eps=0.0, max_iter=steps)
    ctx.pifcm_set_decomposition([xg], p, 4, 32, 2)
    out = ctx.pifcm_pso_interleaved([xg], p, st, c0[None], [U0], steps=steps)
    lam, xi = (float(v) for v in np.float32(out["best_pos"][0]))
    s = ctx.ifcm_solve(xg, _P(C=4, m=2.0, eps=0.0, max_iter=G * steps), lam, xi, c0, U_in=U0)
    assert np.array_equal(host(out["U_best"][0]), host(s["U"]))
    assert np.array_equal(out["centres_best"][0], s["c"])
    o = oracle.solve(xo, c0.astype(np.float64), oracle.Params(C=4, m=2.0, eps=0.0, max_iter=G * steps),
                     lam, xi, U0=host(U0).astype(np.float64))
    assert rel(host(s["U"]), o["U"]) <= TOL and rel(s["c"], o["c"]) <= TOL


def test_decomposition_arguments(ctx):
    from paper_2002_01981_amd import PifcmError
    from paper_2002_01981_amd.abi import PIFCM_E_INVALID, PIFCM_E_UNSUPPORTED
    x = _volumes(ctx)[0][1]
    for args, status in (((3, 32, 1), PIFCM_E_INVALID), ((4, -1, 1), PIFCM_E_INVALID),
                         ((4, 32, 3), PIFCM_E_INVALID)):
        with pytest.raises(PifcmError) as e:
            ctx.pifcm_set_decomposition([x], _P(C=4), *args)
        assert e.value.status == status
    with pytest.raises(PifcmError) as e:
        ctx.pifcm_set_decomposition([x], _P(C=3), 4, 32, 2)
    assert e.value.status == PIFCM_E_UNSUPPORTED


def test_default_depth_by_hand_is_the_default(ctx):
    """planes_per_tile = 0 sets the default depth: the same bits as a context
    that never chose a decomposition."""
    from paper_2002_01981_amd import Context
    xo, xg, c0, U0 = _volumes(ctx)[1]
    p = _P(C=4, m=2.0, eps=0.0, max_iter=6)
    fresh = Context(0)
    try:
        a = fresh.ifcm_solve(xg, p, 0.3, 0.2, c0, U_in=U0, want_hist=True)
    finally:
        fresh.close()
    ctx.pifcm_set_decomposition([xg], p, 4, 0, 1)
    b = ctx.ifcm_solve(xg, p, 0.3, 0.2, c0, U_in=U0, want_hist=True)
    assert np.array_equal(host(a["U"]), host(b["U"]))
    assert np.array_equal(a["c"], b["c"]) and np.array_equal(a["J_hist"], b["J_hist"])
