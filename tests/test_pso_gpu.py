"""The native swarm driver (pifcm_pso, Algorithm 1 steps 3-9) and the tile
autotuner (pifcm_tune) on the GPU.

The swarm's fitnesses come from the same fused step as swarm_evaluate; what
is new here is the host-side bookkeeping (personal and global bests, the
velocity and position update, clipping) and batching B volumes into one
launch per generation.  The oracle's swarm is the reference whenever every
decision it takes is separated by more than the parity bar; the bookkeeping
itself is checked by replaying the rules on the GPU's own fitnesses.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, dev, host, pso_replay, rel

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


def _volume(ctx, shape, seed):
    raw, _ = synth.random_ellipsoids(shape=shape, seed=seed, sigma=0.07)
    xo = oracle.normalize(raw)
    xg = ctx.pifcm_normalize(dev(raw))
    assert np.array_equal(host(xg), xo)
    return xo, xg


def test_pso_matches_oracle(ctx):
    xo, xg = _volume(ctx, (10, 24, 30), 70)
    c0, U0, _ = oracle.fcm_init(xo, oracle.Params(C=4, m=2.0, eps=0.0, max_iter=10))
    c0, U0 = c0.astype(np.float32), U0.astype(np.float32)
    st = synth.pso_streams(85, 6, 4)
    o = oracle.pso(xo, c0.astype(np.float64), U0.astype(np.float64),
                   oracle.Params(C=4, m=2.0, eps=0.0, max_iter=8), st)
    _, _, _, margin = pso_replay(o["fit_hist"], st)
    assert margin > 1e-3  # the oracle's decisions are far apart: both sides must take them
    g = ctx.pifcm_pso([xg], _P(C=4, m=2.0, eps=0.0, max_iter=8), st, c0[None], [dev(U0)])
    assert np.max(np.abs(g["pos_hist"][0] - o["pos_hist"])) <= 1e-12
    assert rel(g["fit_hist"][0], o["fit_hist"]) <= TOL
    assert np.max(np.abs(g["best_pos"][0] - o["best_pos"])) <= 1e-12
    assert abs(g["best_fit"][0] - o["best_fit"]) <= TOL * abs(o["best_fit"])


def _multi(ctx, shapes, seed):
    xs, c0s, U0s = [], [], []
    for b, s in enumerate(shapes):
        xo, xg = _volume(ctx, s, seed + b)
        cg, Ug, _ = ctx.pifcm_fcm_init(xg, _P(C=4, m=2.0, eps=0.0, max_iter=10))
        xs.append(xg)
        c0s.append(cg)
        U0s.append(Ug)
    return xs, np.stack(c0s), U0s


def test_pso_bookkeeping_replays_on_gpu_fitness(ctx):
    """Positions and bests follow the swarm rules exactly, given the
    fitnesses the GPU computed; each recorded fitness is the swarm
    evaluation at the recorded (float32) position."""
    xs, c0, U0 = _multi(ctx, [(9, 20, 44), (6, 31, 27)], 71)
    p = _P(C=4, m=2.0, eps=1e-4, max_iter=12)
    st = synth.pso_streams(86, 10, 5)
    g = ctx.pifcm_pso(xs, p, st, c0, U0, w=0.6, c1=1.2, c2=1.8)
    for b in range(2):
        ph, gb, bf, _ = pso_replay(g["fit_hist"][b], st, w=0.6, c1=1.2, c2=1.8)
        assert np.max(np.abs(ph - g["pos_hist"][b])) <= 1e-12
        assert np.max(np.abs(gb - g["best_pos"][b])) <= 1e-12
        assert bf == g["best_fit"][b]
        assert np.all((g["pos_hist"][b] >= 0.0) & (g["pos_hist"][b] <= 1.0))
    for gen in (0, 4):
        parts = g["pos_hist"][:, gen].astype(np.float32)
        ev = ctx.swarm_evaluate(xs, p, parts, c0, U0)
        assert np.array_equal(ev["fitness"], g["fit_hist"][:, gen])


def test_pso_batch_equals_single_volume_runs(ctx):
    from paper_2002_01981_amd import PIFCM_SWARM_PLAIN
    xs, c0, U0 = _multi(ctx, [(8, 18, 50), (11, 13, 37), (5, 26, 26)], 72)
    p = _P(C=4, m=2.0, eps=0.0, max_iter=6)
    st = synth.pso_streams(87, 7, 3)
    allb = ctx.pifcm_pso(xs, p, st, c0, U0)
    for b in range(3):
        one = ctx.pifcm_pso([xs[b]], p, st, c0[b:b + 1], [U0[b]])
        assert np.array_equal(one["fit_hist"][0], allb["fit_hist"][b])
        assert np.array_equal(one["pos_hist"][0], allb["pos_hist"][b])
        assert np.array_equal(one["best_pos"][0], allb["best_pos"][b])
    plain = ctx.pifcm_pso(xs, p, st, c0, U0, mode=PIFCM_SWARM_PLAIN)
    assert np.array_equal(plain["fit_hist"], allb["fit_hist"])
    assert np.array_equal(plain["best_pos"], allb["best_pos"])


def test_pso_single_generation_and_particle(ctx):
    xs, c0, U0 = _multi(ctx, [(4, 9, 70)], 73)
    p = _P(C=4, m=2.0, eps=0.0, max_iter=3)
    st = synth.pso_streams(88, 1, 1)
    g = ctx.pifcm_pso(xs, p, st, c0, U0)
    assert np.array_equal(g["pos_hist"][0, 0], st["x0"])
    assert np.array_equal(g["best_pos"][0], st["x0"][0])
    assert g["best_fit"][0] == g["fit_hist"][0, 0, 0]


def test_pso_rejects_bad_arguments(ctx):
    from paper_2002_01981_amd import PifcmError
    xs, c0, U0 = _multi(ctx, [(4, 9, 70)], 74)
    p = _P(C=4, m=2.0, eps=0.0, max_iter=3)
    st = synth.pso_streams(89, 4, 2)
    with pytest.raises(PifcmError):
        ctx.pifcm_pso(xs, p, st, c0, U0, w=float("nan"))
    bad = dict(st, r1=np.zeros((0, 4, 2)), r2=np.zeros((0, 4, 2)))
    with pytest.raises(PifcmError):
        ctx.pifcm_pso(xs, p, bad, c0, U0)


def test_tune_keeps_results_and_reports_choice(ctx):
    xs, c0, U0 = _multi(ctx, [(12, 40, 52), (20, 17, 33)], 75)
    p = _P(C=4, m=2.0, eps=0.0, max_iter=6)
    parts = synth.uniform_particles(90, 6)
    before = ctx.swarm_evaluate(xs, p, parts, c0, U0)
    desc = ctx.pifcm_tune(xs, p, 8)
    assert desc.startswith("waves_per_group=") and "planes_per_tile=" in desc
    after = ctx.swarm_evaluate(xs, p, parts, c0, U0)
    assert np.max(np.abs(after["fitness"] - before["fitness"]) / np.abs(before["fitness"])) <= 1e-5
    assert rel(after["centres"], before["centres"]) <= 1e-5
    # tuned shapes still agree with the oracle
    xo = oracle.normalize(synth.random_ellipsoids(shape=(12, 40, 52), seed=75, sigma=0.07)[0])
    o = oracle.solve(xo, c0[0].astype(np.float64), oracle.Params(C=4, m=2.0, eps=0.0, max_iter=6),
                     float(parts[2, 0]), float(parts[2, 1]), U0=host(U0[0]).astype(np.float64))
    assert abs(after["fitness"][0, 2] - o["J"]) <= TOL * abs(o["J"])
    assert rel(after["centres"][0, 2], o["c"]) <= TOL


def test_tune_cache_file(ctx, tmp_path, monkeypatch):
    """With PIFCM_TUNE_CACHE naming a file, the first tuning stores its
    choice under the key of (device, C, m == 2, V, B, P, shape bucket); a new
    context reads it back without timing, reports it as cached, and runs the
    same decomposition: the same bits as the context that tuned."""
    import json
    from paper_2002_01981_amd import Context
    xs, c0, U0 = _multi(ctx, [(12, 40, 52), (20, 17, 33)], 76)
    p = _P(C=4, m=2.0, eps=0.0, max_iter=6)
    parts = synth.uniform_particles(91, 8)
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PIFCM_TUNE_CACHE", str(cache))
    desc = ctx.pifcm_tune(xs, p, 8)
    assert "candidates=" in desc and "cached" not in desc
    entries = [l for l in cache.read_text().splitlines() if '"' in l and "{" in l]
    assert len(entries) == 1
    key = entries[0].split('"')[1]
    assert key.split("|")[1:] == ["C4", "m2", "V1", "B2", "P8", "N2^16", "Z2^5"]
    chosen = json.loads("{" + entries[0].strip().rstrip(",") + "}")[key]
    assert set(chosen) == {"nw", "zc", "pt", "step_ms"}
    tuned = ctx.swarm_evaluate(xs, p, parts, c0, U0)
    other = Context(0)
    try:
        desc2 = other.pifcm_tune(xs, p, 8)
        assert "cached" in desc2 and key in desc2
        assert desc2.startswith(f"waves_per_group={chosen['nw']} ")
        assert f"particles_per_item={chosen['pt']} " in desc2
        again = other.swarm_evaluate(xs, p, parts, c0, U0)
    finally:
        other.close()
    assert np.array_equal(tuned["fitness"], again["fitness"])
    assert np.array_equal(tuned["centres"], again["centres"])
    assert len([l for l in cache.read_text().splitlines() if '"' in l and "{" in l]) == 1


def test_pso_interleaved_matches_oracle(ctx):
    """Particles carrying their own state, 2 iterations per generation."""
    from gpu_util import rel2, saturated
    xo, xg = _volume(ctx, (10, 24, 30), 70)
    c0, U0, _ = oracle.fcm_init(xo, oracle.Params(C=4, m=2.0, eps=0.0, max_iter=10))
    c0, U0 = c0.astype(np.float32), U0.astype(np.float32)
    st = synth.pso_streams(127, 6, 4)
    o = oracle.pso_interleaved(xo, c0.astype(np.float64), U0.astype(np.float64),
                               oracle.Params(C=4, m=2.0), st, steps=2)
    assert pso_replay(o["fit_hist"], st)[3] > 1e-3
    g = ctx.pifcm_pso_interleaved([xg], _P(C=4, m=2.0), st, c0[None], [dev(U0)], steps=2)
    assert np.max(np.abs(g["pos_hist"][0] - o["pos_hist"])) <= 1e-12
    assert rel(g["fit_hist"][0], o["fit_hist"]) <= TOL
    assert np.max(np.abs(g["best_pos"][0] - o["best_pos"])) <= 1e-12
    sat = saturated(*o["best_pos"])
    assert (rel2 if sat else rel)(host(g["U_best"][0]), o["U_best"]) <= TOL
    assert rel(g["centres_best"][0], o["c_best"]) <= TOL


def test_pso_interleaved_frozen_swarm_equals_long_solves(ctx):
    from paper_2002_01981_amd import PIFCM_SWARM_PLAIN
    xs, c0, U0 = _multi(ctx, [(7, 19, 33), (5, 12, 40)], 76)
    st = synth.pso_streams(128, 3, 3)
    st = dict(x0=st["x0"], v0=np.zeros_like(st["v0"]), r1=np.zeros_like(st["r1"]),
              r2=np.zeros_like(st["r2"]))
    steps = 2
    g = ctx.pifcm_pso_interleaved(xs, _P(C=4, m=2.0), st, c0, U0, steps=steps)
    gp = ctx.pifcm_pso_interleaved(xs, _P(C=4, m=2.0), st, c0, U0, steps=steps,
                                   mode=PIFCM_SWARM_PLAIN)
    assert np.array_equal(g["fit_hist"], gp["fit_hist"])
    parts = st["x0"].astype(np.float32)
    for gen in range(3):
        ev = ctx.swarm_evaluate(xs, _P(C=4, m=2.0, eps=0.0, max_iter=(gen + 1) * steps), parts,
                                c0, U0)
        assert np.array_equal(ev["fitness"], g["fit_hist"][:, gen])
    for b in range(2):
        k = int(np.argmin(g["fit_hist"][b].min(axis=0)))
        s = ctx.ifcm_solve(xs[b], _P(C=4, m=2.0, eps=0.0, max_iter=3 * steps), float(parts[k, 0]),
                           float(parts[k, 1]), c0[b], U_in=U0[b])
        assert np.array_equal(host(s["U"]), host(g["U_best"][b]))
        assert np.array_equal(s["c"], g["centres_best"][b])
