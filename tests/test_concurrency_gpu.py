"""Separate contexts used from two host threads at once (each context has its
own stream and workspace; the library's only shared state is its occupancy
caches and the no-allocation scratch array, whose calls it serialises):
every result equals, bit for bit, the same call run alone."""
import threading

import numpy as np
import pytest

import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu


def _P(**kw):
    from paper_2002_01981_amd import Params
    return Params(**kw)


def _calls(ctx, seed):
    """A batched swarm, a backward pass and a no-allocation solve on one
    context; returns their host results."""
    shapes = [(40, 48, 36), (24, 30, 52)]
    xs, c0, U0 = [], [], []
    for b, shape in enumerate(shapes):
        raw = synth.random_ellipsoids(shape=shape, seed=seed + b, sigma=0.07)[0]
        x = ctx.pifcm_normalize(dev(raw))
        c, U, _ = ctx.pifcm_fcm_init(x, _P(C=4, m=2.0, eps=0.0, max_iter=10))
        xs.append(x)
        c0.append(c)
        U0.append(U)
    parts = synth.uniform_particles(seed, 16)
    sw = ctx.swarm_evaluate(xs, _P(C=4, m=2.0, eps=0.0, max_iter=6), parts, np.stack(c0), U0)
    g = ctx.ifcm_backward(xs[0], _P(C=4, m=2.0), 0.3, 0.2, c0[0], U0[0], 7, 3)
    import torch
    Uo = torch.empty_like(U0[1])
    na = ctx.ifcm_solve_noalloc(xs[1], _P(C=4, m=2.0, eps=0.0, max_iter=5), 0.4, 0.1, c0[1], U_in=U0[1],
                                U_out=Uo)
    torch.cuda.synchronize()
    return dict(fit=sw["fitness"].copy(), cen=sw["centres"].copy(), J=g["J"],
                grad=np.concatenate([[g["dlam"], g["dxi"]], g["dc"]]), naJ=na["J"], nac=na["c"].copy(),
                naU=Uo.cpu().numpy())


def _run(seed, out, key):
    from paper_2002_01981_amd import Context
    ctx = Context(0)
    try:
        out[key] = _calls(ctx, seed)
    except Exception as e:  # reported by the main thread
        out[key] = e
    finally:
        ctx.close()


def test_two_threads_two_contexts():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    alone = {}
    for seed in (11, 12):
        _run(seed, alone, seed)
    together = {}
    ts = [threading.Thread(target=_run, args=(seed, together, seed)) for seed in (11, 12)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in ts), "a thread did not finish"
    for seed in (11, 12):
        a, b = alone[seed], together[seed]
        for r in (a, b):
            if isinstance(r, Exception):
                raise r
        assert np.array_equal(a["fit"], b["fit"]) and np.array_equal(a["cen"], b["cen"])
        assert a["J"] == b["J"] and np.array_equal(a["grad"], b["grad"])
        assert a["naJ"] == b["naJ"] and np.array_equal(a["nac"], b["nac"])
        assert np.array_equal(a["naU"], b["naU"])
