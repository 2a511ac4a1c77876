"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every comparison runs both sides on the same seeded inputs: the raw phantoms
of `synth` are normalised by each side separately (and checked bit-equal),
initial memberships are drawn in float32 and handed to both.  The bar is
1e-4 relative (norm-wise) on memberships and centres, labels bit-exact
outside the 1e-5 tie band, integers (iteration counts) exact.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import (SATURATED_TIE_BAND, TIE_BAND, TOL, check_labels, dev, host,
                      random_memberships_f32, rel, rel2, saturated)

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


def _both_normalised(ctx, raw):
    xo = oracle.normalize(raw)
    xg = ctx.pifcm_normalize(dev(raw))
    assert np.array_equal(host(xg), xo), "normalisation differs"
    return xo, xg


def _run_steps(ctx, raw, C, lam, xi, steps, m=2.0, flags=0, seed=0, c0=None):
    rng = np.random.default_rng(seed)
    xo, xg = _both_normalised(ctx, raw)
    U0 = random_memberships_f32(rng, xo.size, C)
    if c0 is None:
        c0 = np.linspace(0.1, 0.9, C).astype(np.float32)
    p = _P(C=C, m=m, eps=0.0, max_iter=steps, flags=flags)
    g = ctx.ifcm_solve(xg, p, lam, xi, c0, U_in=dev(U0), labels=True, want_hist=True)
    po = oracle.Params(C=C, m=m, eps=0.0, max_iter=steps, flags=flags)
    o = oracle.solve(xo, c0.astype(np.float64), po, lam, xi, U0=U0.astype(np.float64),
                     want_hist=True)
    return g, o


def _assert_close(g, o, C, lam, xi, tol=TOL):
    assert g["iters"] == o["iters"]
    sat = saturated(lam, xi)
    eu = (rel2 if sat else rel)(host(g["U"]), o["U"])
    ec = rel(g["c"], o["c"])
    ej = abs(g["J"] - o["J"]) / abs(o["J"])
    assert eu <= tol, f"memberships off by {eu:.3g}"
    assert ec <= tol, f"centres off by {ec:.3g}"
    assert ej <= tol, f"objective off by {ej:.3g}"
    if "J_hist" in g and len(o.get("J_hist", [])):
        eh = np.max(np.abs(g["J_hist"] - o["J_hist"]) / np.abs(o["J_hist"]))
        assert eh <= tol, f"objective history off by {eh:.3g}"
    check_labels(host(g["labels"]), o["U"], C, SATURATED_TIE_BAND if sat else TIE_BAND)
    return eu, ec, ej


# ------------------------------------------------------------ normalisation
def test_normalize_bit_exact(ctx):
    for raw in (synth.nested_ellipsoids()[0],
                synth.random_ellipsoids(shape=(6, 70, 90), seed=9)[0],
                synth.brain_shells(shape=(20, 31, 27), seed=4)[0]):
        _both_normalised(ctx, raw)


def test_normalize_in_place_and_constant(ctx):
    raw = synth.random_ellipsoids(shape=(4, 33, 65), seed=3)[0]
    t = dev(raw)
    ctx.pifcm_normalize(t, out=t)
    assert np.array_equal(host(t), oracle.normalize(raw))
    c = np.full((3, 4, 5), 2.5, np.float32)
    assert np.all(host(ctx.pifcm_normalize(dev(c))) == 0)


# ------------------------------------------------------------- step parity
@pytest.mark.parametrize("shape", [(70, 10, 150), (33, 9, 64), (5, 7, 65), (40, 3, 129),
                                   (2, 70, 20)])
@pytest.mark.parametrize("lam,xi", [(0.3, 0.4), (0.0, 0.0), (0.9, 0.7)])
def test_steps_span_tiles(ctx, shape, lam, xi):
    """Wave tiles are 16 x 4 columns by 32 planes (the default depth of
    these small volumes): these shapes cover several tiles in every
    direction with ragged tails."""
    raw = synth.random_ellipsoids(shape=shape, seed=sum(shape), sigma=0.07)[0]
    g, o = _run_steps(ctx, raw, 4, lam, xi, steps=3, seed=shape[0])
    _assert_close(g, o, 4, lam, xi)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 2), (2, 1, 1), (1, 3, 2), (3, 1, 64),
                                   (1, 1, 65), (2, 5, 129), (4, 4, 2)])
def test_tiny_and_degenerate_volumes(ctx, shape):
    rng = np.random.default_rng(sum(shape) + 7)
    raw = rng.random(shape).astype(np.float32)
    g, o = _run_steps(ctx, raw, 3, 0.5, 0.3, steps=4, seed=3)
    _assert_close(g, o, 3, 0.5, 0.3)


@pytest.mark.parametrize("C", [2, 3, 5, 8, 16])
def test_cluster_counts(ctx, C):
    raw = synth.random_ellipsoids(shape=(9, 11, 70), seed=C, sigma=0.07)[0]
    g, o = _run_steps(ctx, raw, C, 0.4, 0.3, steps=3, seed=C)
    _assert_close(g, o, C, 0.4, 0.3)


@pytest.mark.parametrize("m", [2.5, 1.5])
def test_general_fuzziness(ctx, m):
    raw = synth.random_ellipsoids(shape=(7, 9, 80), seed=11, sigma=0.07)[0]
    g, o = _run_steps(ctx, raw, 4, 0.35, 0.25, steps=3, m=m, seed=5)
    _assert_close(g, o, 4, 0.35, 0.25)


def test_q2_reading_flag(ctx):
    from paper_2002_01981_amd import PIFCM_Q2_SQDIST
    raw = synth.random_ellipsoids(shape=(6, 10, 70), seed=21, sigma=0.07)[0]
    g, o = _run_steps(ctx, raw, 4, 0.3, 0.6, steps=3, flags=PIFCM_Q2_SQDIST, seed=2)
    _assert_close(g, o, 4, 0.3, 0.6)


def test_flat_neighbourhoods(ctx):
    """Voxels whose neighbours all share their intensity take the mean
    branch of eq (5)."""
    raw = np.zeros((6, 8, 70), np.float32)
    raw[:, :, 35:] = 1.0
    raw[2:4, 3:5, 10:12] = 0.5
    g, o = _run_steps(ctx, raw, 3, 0.5, 0.4, steps=4, seed=9)
    _assert_close(g, o, 3, 0.5, 0.4)


def test_attraction_beyond_one_clamps(ctx):
    """lambda + xi > 1 drives the factor of eq (4) to <= 0: both sides floor
    the squared distance at 1e-12."""
    raw = synth.random_ellipsoids(shape=(8, 12, 70), seed=31, sigma=0.07)[0]
    g, o = _run_steps(ctx, raw, 4, 1.0, 1.0, steps=4, seed=4)
    _assert_close(g, o, 4, 1.0, 1.0)


# -------------------------------------------------------- solves end to end
def test_fcm_init_parity(ctx):
    raw, _ = synth.nested_ellipsoids()
    xo, xg = _both_normalised(ctx, raw)
    p = _P(C=4, m=2.0, eps=1e-5, max_iter=50)
    cg, Ug, itg = ctx.pifcm_fcm_init(xg, p)
    co, Uo, ito = oracle.fcm_init(xo, oracle.Params(C=4, m=2.0, eps=1e-5, max_iter=50))
    assert itg == ito
    assert rel(cg, co) <= TOL
    assert rel(host(Ug), Uo) <= TOL
    assert np.all(np.diff(cg) >= 0)


@pytest.mark.parametrize("lam,xi", [(0.25, 0.5), (0.6, 0.3), (0.05, 0.9)])
def test_solve_nested32_end_to_end(ctx, lam, xi):
    """The CPU-sized workload: each side computes its own FCM initial state
    and then the IFCM solve with the convergence rule."""
    raw, _ = synth.nested_ellipsoids()
    xo, xg = _both_normalised(ctx, raw)
    p = _P(C=4, m=2.0, eps=1e-5, max_iter=50)
    po = oracle.Params(C=4, m=2.0, eps=1e-5, max_iter=50)
    cg, Ug, _ = ctx.pifcm_fcm_init(xg, p)
    co, Uo, _ = oracle.fcm_init(xo, po)
    g = ctx.ifcm_solve(xg, p, lam, xi, cg, U_in=Ug, labels=True, want_hist=True)
    o = oracle.solve(xo, co, po, lam, xi, U0=Uo, want_hist=True)
    _assert_close(g, o, 4, lam, xi)


def test_determinism(ctx):
    raw = synth.random_ellipsoids(shape=(20, 30, 100), seed=5)[0]
    xg = ctx.pifcm_normalize(dev(raw))
    p = _P(C=4, m=2.0, eps=0.0, max_iter=6)
    c0 = np.array([0.1, 0.4, 0.6, 0.9], np.float32)
    a = ctx.ifcm_solve(xg, p, 0.3, 0.3, c0, labels=True)
    b = ctx.ifcm_solve(xg, p, 0.3, 0.3, c0, labels=True)
    assert np.array_equal(host(a["U"]), host(b["U"]))
    assert np.array_equal(a["c"], b["c"]) and a["J"] == b["J"]
    assert np.array_equal(host(a["labels"]), host(b["labels"]))


def test_constant_volume(ctx):
    raw = np.full((5, 6, 70), 3.0, np.float32)
    xg = ctx.pifcm_normalize(dev(raw))
    p = _P(C=4, m=2.0, eps=0.0, max_iter=5)
    c, U0, _ = ctx.pifcm_fcm_init(xg, p)
    assert np.all(c == 0)
    g = ctx.ifcm_solve(xg, p, 0.6, 0.3, c, U_in=U0, labels=True)
    np.testing.assert_allclose(host(g["U"]), 0.25, atol=1e-6)
    assert np.all(g["c"] == 0)
    assert np.all(host(g["labels"]) == 0)


# ------------------------------------------------------------------ swarm
def _swarm_case(ctx, shapes, P, eps, max_iter, seed):
    raws = [synth.random_ellipsoids(shape=s, seed=seed + b, sigma=0.07)[0]
            for b, s in enumerate(shapes)]
    p = _P(C=4, m=2.0, eps=eps, max_iter=max_iter)
    po = oracle.Params(C=4, m=2.0, eps=eps, max_iter=max_iter)
    xs, inits = [], []
    for raw in raws:
        xo, xg = _both_normalised(ctx, raw)
        xs.append((xo, xg))
        cg, Ug, _ = ctx.pifcm_fcm_init(xg, _P(C=4, m=2.0, eps=0.0, max_iter=10))
        inits.append((cg, Ug))
    parts = synth.uniform_particles(seed, P)
    return raws, p, po, xs, inits, parts


def test_swarm_batched_equals_plain_and_oracle(ctx):
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED, PIFCM_SWARM_PLAIN
    shapes = [(10, 20, 70), (7, 33, 40), (12, 9, 130)]
    raws, p, po, xs, inits, parts = _swarm_case(ctx, shapes, P=5, eps=1e-5, max_iter=15, seed=40)
    c0 = np.stack([c for c, _ in inits])
    U0 = [u for _, u in inits]
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
    pla = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_PLAIN)
    assert np.array_equal(bat["fitness"], pla["fitness"])
    assert np.array_equal(bat["centres"], pla["centres"])
    assert np.array_equal(bat["iters"], pla["iters"])
    again = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
    assert np.array_equal(bat["fitness"], again["fitness"])
    for b, (xo, _) in enumerate(xs):
        U0o = host(U0[b]).astype(np.float64)
        for q in range(parts.shape[0]):
            lam, xi = parts[q]
            o = oracle.solve(xo, c0[b].astype(np.float64), po, float(lam), float(xi), U0=U0o)
            assert bat["iters"][b, q] == o["iters"]
            assert abs(bat["fitness"][b, q] - o["J"]) <= TOL * abs(o["J"])
            assert rel(bat["centres"][b, q], o["c"]) <= TOL


def test_swarm_stop_rule_many_items_per_wave(ctx):
    """A batched swarm under the stop rule with several times more tile items
    than the grid has waves, so every wave walks a run of items: every pair
    against the oracle.  Where the two stop at different iterations (the
    largest membership change within rounding of eps), the pair is checked
    against the oracle run for the GPU's iteration count instead."""
    shapes = [(64, 96, 128), (40, 72, 100)]
    raws, p, po, xs, inits, parts = _swarm_case(ctx, shapes, P=48, eps=1e-3, max_iter=10, seed=70)
    c0 = np.stack([c for c, _ in inits])
    U0 = [u for _, u in inits]
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0)
    assert np.all(bat["iters"] >= 1)
    assert len(np.unique(bat["iters"])) > 1, "every pair stopped together: the stop rule is not exercised"
    ties = 0
    for b, (xo, _) in enumerate(xs):
        U0o = host(U0[b]).astype(np.float64)
        for q in range(parts.shape[0]):
            lam, xi = (float(v) for v in parts[q])
            o = oracle.solve(xo, c0[b].astype(np.float64), po, lam, xi, U0=U0o)
            n = int(bat["iters"][b, q])
            if n != o["iters"]:
                ties += 1
                assert abs(n - o["iters"]) == 1, (b, q, n, o["iters"])
                o = oracle.solve(xo, c0[b].astype(np.float64),
                                 oracle.Params(C=4, m=2.0, eps=0.0, max_iter=n), lam, xi, U0=U0o)
            assert abs(bat["fitness"][b, q] - o["J"]) <= TOL * abs(o["J"]), (b, q)
            assert rel(bat["centres"][b, q], o["c"]) <= TOL, (b, q)
    assert ties <= 3, f"{ties} pairs stopped at another iteration than the oracle's"


@pytest.mark.parametrize("C,m", [(2, 1.7), (3, 2.0), (4, 2.5), (6, 2.0)])
def test_swarm_other_cluster_counts_and_fuzziness(ctx, C, m):
    """Batched and plain swarm evaluation at cluster counts and fuzzifiers
    other than the benchmark's (one particle per work item, the general-m
    memberships of eq (2)), under the stop rule: the two modes bit-identical,
    every pair against the oracle (a pair that stops one iteration apart
    from the oracle, its largest change within rounding of eps, is checked
    at the GPU's iteration count)."""
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED, PIFCM_SWARM_PLAIN
    shapes = [(9, 21, 66), (14, 10, 37)]
    eps, T = 1e-5, 12
    p = _P(C=C, m=m, eps=eps, max_iter=T)
    po = oracle.Params(C=C, m=m, eps=eps, max_iter=T)
    xs, c0, U0 = [], [], []
    for b, shape in enumerate(shapes):
        raw = synth.random_ellipsoids(shape=shape, seed=80 + b, sigma=0.07)[0]
        xo, xg = _both_normalised(ctx, raw)
        cg, Ug, _ = ctx.pifcm_fcm_init(xg, _P(C=C, m=m, eps=0.0, max_iter=10))
        xs.append((xo, xg))
        c0.append(cg)
        U0.append(Ug)
    c0 = np.stack(c0)
    parts = synth.uniform_particles(81, 5)
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
    pla = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_PLAIN)
    assert np.array_equal(bat["fitness"], pla["fitness"])
    assert np.array_equal(bat["centres"], pla["centres"])
    assert np.array_equal(bat["iters"], pla["iters"])
    ties = 0
    for b, (xo, _) in enumerate(xs):
        U0o = host(U0[b]).astype(np.float64)
        for q in range(parts.shape[0]):
            lam, xi = (float(v) for v in parts[q])
            o = oracle.solve(xo, c0[b].astype(np.float64), po, lam, xi, U0=U0o)
            n = int(bat["iters"][b, q])
            if n != o["iters"]:
                ties += 1
                assert abs(n - o["iters"]) == 1, (b, q, n, o["iters"])
                o = oracle.solve(xo, c0[b].astype(np.float64), oracle.Params(C=C, m=m, eps=0.0, max_iter=n),
                                 lam, xi, U0=U0o)
            assert abs(bat["fitness"][b, q] - o["J"]) <= TOL * abs(o["J"]), (b, q)
            assert rel(bat["centres"][b, q], o["c"]) <= TOL, (b, q)
    assert ties <= 1


def test_swarm_counter_handout_matches_plain(ctx):
    """Without a stop rule a batched launch whose XCD ranges hold more items
    than the XCD has waves hands the last tenth of each range out by counter
    (here ≈ 46 000 items of 32-plane tiles, one particle per item, against
    ≈ 3000 resident waves): bit-identical to the plain
    mode, which runs each pair alone with no counter, on every pair; a second
    call (the counters reset by the first) bit-identical again; sampled pairs
    against the oracle."""
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED, PIFCM_SWARM_PLAIN
    shapes = [(128, 96, 64), (100, 80, 70), (90, 60, 50)]
    T = 5
    p = _P(C=4, m=2.0, eps=0.0, max_iter=T)
    xs, c0, U0 = [], [], []
    for b, shape in enumerate(shapes):
        raw = synth.random_ellipsoids(shape=shape, seed=90 + b, sigma=0.07)[0]
        xo, xg = _both_normalised(ctx, raw)
        cg, Ug, _ = ctx.pifcm_fcm_init(xg, _P(C=4, m=2.0, eps=0.0, max_iter=10))
        xs.append((xo, xg))
        c0.append(cg)
        U0.append(Ug)
    c0 = np.stack(c0)
    P = 48
    parts = synth.uniform_particles(91, P)
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
    again = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
    pla = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_PLAIN)
    for other in (again, pla):
        assert np.array_equal(bat["fitness"], other["fitness"])
        assert np.array_equal(bat["centres"], other["centres"])
        assert np.array_equal(bat["iters"], other["iters"])
    assert np.all(bat["iters"] == T)
    po = oracle.Params(C=4, m=2.0, eps=0.0, max_iter=T)
    for b, q in ((0, 0), (1, 23), (2, 47)):
        xo = xs[b][0]
        lam, xi = (float(v) for v in parts[q])
        o = oracle.solve(xo, c0[b].astype(np.float64), po, lam, xi, U0=host(U0[b]).astype(np.float64))
        assert abs(bat["fitness"][b, q] - o["J"]) <= TOL * abs(o["J"]), (b, q)
        assert rel(bat["centres"][b, q], o["c"]) <= TOL, (b, q)


def _tiny_batch(ctx, shapes, seed, C=4, m=2.0):
    xs, c0, U0 = [], [], []
    for b, shape in enumerate(shapes):
        raw = synth.random_ellipsoids(shape=shape, seed=seed + b, sigma=0.07)[0]
        xo, xg = _both_normalised(ctx, raw)
        cg, Ug, _ = ctx.pifcm_fcm_init(xg, _P(C=C, m=m, eps=0.0, max_iter=10))
        xs.append((xo, xg))
        c0.append(cg)
        U0.append(Ug)
    return xs, np.stack(c0), U0


def test_swarm_largest_batch_of_volumes(ctx):
    """32 ragged volumes in one call (the most a launch holds), a few of them
    a single plane or a single row, 3 particles: batched and plain
    bit-identical, every pair against the oracle."""
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED, PIFCM_SWARM_PLAIN
    rng = np.random.default_rng(95)
    shapes = [tuple(int(v) for v in rng.integers(2, 19, 3)) for _ in range(29)] + [(1, 7, 23), (6, 1, 19), (5, 9, 1)]
    xs, c0, U0 = _tiny_batch(ctx, shapes, 300)
    T = 4
    p = _P(C=4, m=2.0, eps=0.0, max_iter=T)
    parts = synth.uniform_particles(96, 3)
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
    pla = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_PLAIN)
    assert bat["fitness"].shape == (32, 3)
    assert np.array_equal(bat["fitness"], pla["fitness"])
    assert np.array_equal(bat["centres"], pla["centres"])
    po = oracle.Params(C=4, m=2.0, eps=0.0, max_iter=T)
    for b, (xo, _) in enumerate(xs):
        for q in range(3):
            lam, xi = (float(v) for v in parts[q])
            o = oracle.solve(xo, c0[b].astype(np.float64), po, lam, xi, U0=host(U0[b]).astype(np.float64))
            assert abs(bat["fitness"][b, q] - o["J"]) <= TOL * max(abs(o["J"]), 1e-30), (b, q)
            assert rel(bat["centres"][b, q], o["c"]) <= TOL, (b, q)


def test_swarm_largest_pair_count(ctx):
    """B x P = 65536 (volumes x particles, the most a call takes) on small
    volumes, one batched launch per iteration: sampled pairs equal a lone
    solve bit for bit and the oracle."""
    shapes = [(3, 5, 7), (2, 6, 9), (4, 4, 4), (5, 3, 8)] * 4
    xs, c0, U0 = _tiny_batch(ctx, shapes, 400)
    P = 65536 // len(shapes)
    T = 3
    p = _P(C=4, m=2.0, eps=0.0, max_iter=T)
    parts = synth.uniform_particles(97, P)
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0)
    assert bat["fitness"].shape == (len(shapes), P)
    assert np.all(np.isfinite(bat["fitness"]))
    po = oracle.Params(C=4, m=2.0, eps=0.0, max_iter=T)
    for b, q in ((0, 0), (5, P // 2), (15, P - 1), (9, 1234)):
        lam, xi = (float(v) for v in parts[q])
        s1 = ctx.ifcm_solve(xg[b], p, lam, xi, c0[b], U_in=U0[b])
        assert s1["J"] == bat["fitness"][b, q]
        assert np.array_equal(s1["c"], bat["centres"][b, q])
        o = oracle.solve(xs[b][0], c0[b].astype(np.float64), po, lam, xi, U0=host(U0[b]).astype(np.float64))
        assert abs(bat["fitness"][b, q] - o["J"]) <= TOL * abs(o["J"]), (b, q)
        assert rel(bat["centres"][b, q], o["c"]) <= TOL, (b, q)


def test_swarm_graph_cache_across_alternating_calls(ctx):
    """The batched mode replays a captured graph kept per context and keyed
    by the launch: swarms of different shapes, particle counts and stop
    rules called in turn (A, B, C, A, B, C) each repeat their first results
    bit for bit."""
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED
    cases = []
    for k, (shapes, P, eps, T) in enumerate((([(10, 20, 70), (7, 33, 40)], 5, 0.0, 6),
                                             ([(16, 24, 30)], 9, 1e-5, 20),
                                             ([(6, 9, 12), (11, 5, 8), (9, 9, 9)], 4, 0.0, 3))):
        xs, c0, U0 = _tiny_batch(ctx, shapes, 500 + 10 * k)
        cases.append(([x for _, x in xs], c0, U0, synth.uniform_particles(98 + k, P),
                      _P(C=4, m=2.0, eps=eps, max_iter=T)))
    first = [ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
             for xg, c0, U0, parts, p in cases]
    for _ in range(2):
        for (xg, c0, U0, parts, p), ref in zip(cases, first):
            r = ctx.swarm_evaluate(xg, p, parts, c0, U0, mode=PIFCM_SWARM_BATCHED)
            assert np.array_equal(r["fitness"], ref["fitness"])
            assert np.array_equal(r["centres"], ref["centres"])
            assert np.array_equal(r["iters"], ref["iters"])


def test_swarm_matches_solve(ctx):
    """A pair of the batched launch and a lone solve with the same tile
    shapes run the same arithmetic in the same order: bit-identical."""
    shapes = [(9, 17, 66), (5, 40, 33)]
    raws, p, po, xs, inits, parts = _swarm_case(ctx, shapes, P=3, eps=0.0, max_iter=5, seed=60)
    c0 = np.stack([c for c, _ in inits])
    U0 = [u for _, u in inits]
    xg = [x for _, x in xs]
    bat = ctx.swarm_evaluate(xg, p, parts, c0, U0)
    for b in range(len(shapes)):
        for q in range(3):
            s = ctx.ifcm_solve(xg[b], p, float(parts[q, 0]), float(parts[q, 1]), c0[b], U_in=U0[b])
            assert s["J"] == bat["fitness"][b, q]
            assert np.array_equal(s["c"], bat["centres"][b, q])


# ---------------------------------------------------------------- errors
def test_error_paths(ctx):
    import torch
    from paper_2002_01981_amd import PifcmError
    from paper_2002_01981_amd.abi import (PIFCM_E_INVALID, PIFCM_E_NONFINITE,
                                          PIFCM_E_UNSUPPORTED)
    x = ctx.pifcm_normalize(dev(synth.random_ellipsoids(shape=(4, 6, 70), seed=1)[0]))
    c0 = np.array([0.1, 0.4, 0.6, 0.9], np.float32)

    def status(fn):
        with pytest.raises(PifcmError) as e:
            fn()
        return e.value.status

    assert status(lambda: ctx.ifcm_solve(x, _P(C=1), 0.3, 0.3, c0[:1])) == PIFCM_E_INVALID
    assert status(lambda: ctx.ifcm_solve(x, _P(m=1.0), 0.3, 0.3, c0)) == PIFCM_E_INVALID
    assert status(lambda: ctx.ifcm_solve(x, _P(V=4), 0.3, 0.3, c0)) == PIFCM_E_UNSUPPORTED
    assert status(lambda: ctx.ifcm_solve(x, _P(), float("nan"), 0.3, c0)) == PIFCM_E_INVALID
    bad = x.clone()
    bad[1, 2, 3] = float("nan")
    assert status(lambda: ctx.ifcm_solve(bad, _P(), 0.3, 0.3, c0)) == PIFCM_E_NONFINITE
    raw_bad = torch.tensor([1.0, float("inf"), 2.0], device="cuda")
    assert status(lambda: ctx.pifcm_normalize(raw_bad)) == PIFCM_E_NONFINITE
    U = torch.full((x.numel(), 4), 0.3, device="cuda")  # rows sum to 1.2
    assert status(lambda: ctx.ifcm_solve(x, _P(), 0.3, 0.3, c0, U_in=U)) == PIFCM_E_INVALID
    Uok = torch.full((x.numel(), 4), 0.25, device="cuda")
    assert status(lambda: ctx.ifcm_solve(x, _P(), 0.3, 0.3, c0, U_in=Uok, U_out=Uok)) == PIFCM_E_INVALID
    big = torch.empty(x.numel() * 4 + 1, device="cuda")
    assert status(lambda: ctx.ifcm_solve(x, _P(), 0.3, 0.3, c0, U_out=big[1:])) == PIFCM_E_INVALID
    # planes whose three-plane tile would pass 2^31 bytes of U are refused
    # (the outputs are allocated at full size: nothing is written either way)
    wide = torch.zeros((1, 8192, 8192), device="cuda")
    assert status(lambda: ctx.ifcm_solve(wide, _P(), 0.3, 0.3, c0)) == PIFCM_E_INVALID
    Uw = torch.full((wide.numel(), 4), 0.25, device="cuda")
    assert status(lambda: ctx.swarm_evaluate([wide], _P(), np.array([[0.3, 0.3]]), c0[None],
                                             [Uw])) == PIFCM_E_INVALID
    assert status(lambda: ctx.ifcm_backward(wide, _P(), 0.3, 0.3, c0, Uw, 2, 1)) == PIFCM_E_INVALID
    del wide, Uw
    # the context still works after errors
    g = ctx.ifcm_solve(x, _P(max_iter=2, eps=0.0), 0.3, 0.3, c0)
    assert g["iters"] == 2 and np.isfinite(g["J"])
