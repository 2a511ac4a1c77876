"""The differentiation workload end to end at full size: brain phantom
181x217x181 (5 % noise), K = 30 unrolled IFCM iterations, checkpoints every
5 iterations.

- The adjoint's gradient of J_K with respect to (lambda, xi, c^0) against
  central differences of the FP64 oracle's J_K (h = 1e-4) at (0.2, 0.3),
  (0.4, 0.1) and (0.1, 0.6).
- Algorithm 1 steps 4-9 followed by the gradient hand-off: a 32-particle,
  10-generation swarm whose fitness is J_K, then projected gradient steps
  from its global best (refine), checked against the oracle's J_K at the
  point reached.

Each oracle J_K at this size costs a few seconds of host time (about a
minute for the 13 of the central differences at each point)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, dev, host

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


@pytest.fixture(scope="module")
def brain(ctx):
    W = synth.WORKLOADS["adjoint-brain-K30"]
    raw, _ = synth.brain_shells(shape=W["shape"], seed=W["seed"], noise_frac=W["noise_frac"])
    xo = oracle.normalize(raw)
    xg = ctx.pifcm_normalize(dev(raw))
    assert np.array_equal(host(xg), xo)
    c0, U0, _ = ctx.pifcm_fcm_init(xg, _P(C=4, m=2.0, eps=0.0, max_iter=10))
    return W, xo, xg, c0, U0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("point", [0, 1, 2])
def test_adjoint_full_size_against_oracle_differences(ctx, brain, point):
    W, xo, xg, c0, U0 = brain
    K, s = W["K"], W["ckpt"]
    lam, xi = W["points"][point]
    print(f"adjoint vs oracle differences: {xo.shape}, K = {K}, ({lam}, {xi})", flush=True)
    g = ctx.ifcm_backward(xg, _P(C=4, m=2.0), lam, xi, c0, U0, K, s)
    po = oracle.Params(C=4, m=2.0, eps=0.0, max_iter=K)
    Jo, fd = oracle.fd_grad(xo, c0.astype(np.float64), host(U0).astype(np.float64), po, lam, xi, K,
                            step=1e-4)
    got = np.concatenate([[g["dlam"], g["dxi"]], g["dc"]])
    err = float(np.max(np.abs(got - fd)) / np.max(np.abs(fd)))
    print(f"J {g['J']:.9g} vs {Jo:.9g}; gradient {got} vs {fd}; rel {err:.2e}", flush=True)
    assert abs(g["J"] - Jo) <= TOL * abs(Jo)
    assert err <= 1e-3


@pytest.mark.timeout(600)
def test_refine_global_best_of_the_swarm(ctx, brain):
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED, refine
    W, xo, xg, c0, U0 = brain
    K, s = W["K"], W["ckpt"]
    ps = W["pso"]
    st = synth.pso_streams(ps["seed"], ps["P"], ps["G"])
    pk = _P(C=4, m=2.0, eps=0.0, max_iter=K)
    sw = ctx.pifcm_pso([xg], pk, st, c0[None], [U0], w=ps["w"], c1=ps["c1"], c2=ps["c2"],
                       mode=PIFCM_SWARM_BATCHED)
    assert np.all(sw["iters_hist"] == K)
    lam0, xi0 = (float(v) for v in sw["best_pos"][0])
    print(f"swarm {ps['P']} x {ps['G']}: best ({lam0:.4f}, {xi0:.4f}) J_K {sw['best_fit'][0]:.9g}",
          flush=True)
    r = refine(ctx, xg, _P(C=4, m=2.0), lam0, xi0, c0, U0, K, s, steps=8, lr=0.05)
    hist = r["history"]
    for h in hist:
        print("refine", [round(float(v), 6) for v in h], flush=True)
    Js = [h[2] for h in hist]
    # the starting J_K is the swarm's best fitness (same solve, same state)
    assert abs(Js[0] - sw["best_fit"][0]) <= 1e-6 * abs(Js[0])
    assert all(b < a for a, b in zip(Js, Js[1:]))
    pos = r["pos"]
    on_edge = bool(np.any((pos == 0.0) | (pos == 1.0)))
    assert len(Js) >= 2 or on_edge, "no descent step from an interior point"
    assert np.all((pos >= 0.0) & (pos <= 1.0))
    # J_K at the point reached, from the oracle
    lam, xi = (float(v) for v in np.float32(pos))
    o = oracle.solve(xo, c0.astype(np.float64), oracle.Params(C=4, m=2.0, eps=0.0, max_iter=K), lam, xi,
                     U0=host(U0).astype(np.float64))
    print(f"refined ({lam:.6f}, {xi:.6f}): J_K {r['J']:.9g} vs oracle {o['J']:.9g}", flush=True)
    assert abs(r["J"] - o["J"]) <= TOL * abs(o["J"])
