"""ifcm_solve_noalloc -- the solve whose workspace is the library's
per-device scratch array -- through the C ABI against ifcm_solve on the
same context: two calls in a row, the second on a smaller volume (the
scratch still holds the first call's contents), bit-identical outputs; the
first call also against the FP64 oracle; requests beyond the scratch
refused before any work."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, check_labels, dev, host, rel

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


def _same(a, b):
    """Every output of two solves bit for bit."""
    assert a["iters"] == b["iters"]
    assert a["J"] == b["J"]
    assert np.array_equal(a["c"], b["c"])
    assert np.array_equal(a["J_hist"], b["J_hist"])
    assert np.array_equal(host(a["U"]), host(b["U"]))
    assert np.array_equal(host(a["labels"]), host(b["labels"]))


def test_noalloc_equals_solve_on_two_calls(ctx):
    # First call: 40 x 96 x 112, C = 4, m = 2, from the FCM initial state,
    # stop rule on.
    print("noalloc case 1: shape (40, 96, 112), C = 4, (0.3, 0.4)", flush=True)
    raw, _ = synth.random_ellipsoids(shape=(40, 96, 112), seed=61, sigma=0.07)
    x = ctx.pifcm_normalize(dev(raw))
    p = _P(C=4, m=2.0, eps=1e-5, max_iter=30)
    c0, U0, _ = ctx.pifcm_fcm_init(x, p)
    a = ctx.ifcm_solve_noalloc(x, p, 0.3, 0.4, c0, U_in=U0, labels=True, want_hist=True)
    b = ctx.ifcm_solve(x, p, 0.3, 0.4, c0, U_in=U0, labels=True, want_hist=True)
    _same(a, b)
    xo = oracle.normalize(raw)
    o = oracle.solve(xo, c0.astype(np.float64), oracle.Params(C=4, m=2.0, eps=1e-5, max_iter=30),
                     0.3, 0.4, U0=host(U0).astype(np.float64))
    assert a["iters"] == o["iters"]
    assert rel(host(a["U"]), o["U"]) <= TOL
    assert rel(a["c"], o["c"]) <= TOL
    assert abs(a["J"] - o["J"]) <= TOL * abs(o["J"])
    check_labels(host(a["labels"]), o["U"], 4)

    # Second call: a smaller volume, C = 3, m = 2.5, memberships from eq (2)
    # (no U_in), a fixed iteration count.
    print("noalloc case 2: shape (9, 20, 33), C = 3, m = 2.5, (0.5, 0.2)", flush=True)
    raw2, _ = synth.random_ellipsoids(shape=(9, 20, 33), seed=62, sigma=0.07)
    x2 = ctx.pifcm_normalize(dev(raw2))
    p2 = _P(C=3, m=2.5, eps=0.0, max_iter=7)
    c2 = np.array([0.2, 0.5, 0.8], np.float32)
    a2 = ctx.ifcm_solve_noalloc(x2, p2, 0.5, 0.2, c2, labels=True, want_hist=True)
    b2 = ctx.ifcm_solve(x2, p2, 0.5, 0.2, c2, labels=True, want_hist=True)
    _same(a2, b2)
    assert a2["iters"] == 7


def test_noalloc_refuses_what_the_scratch_cannot_hold(ctx):
    import torch
    from paper_2002_01981_amd.abi import PIFCM_E_INVALID, PIFCM_E_UNSUPPORTED, PifcmError
    # C = 16: 4 (g_inv) + 64 (memberships) bytes per voxel; 64 x 256 x 256
    # voxels need about 285 MB, more than the 256 MiB array.
    print("noalloc case 3: shape (64, 256, 256), C = 16, refused", flush=True)
    x = torch.zeros((64, 256, 256), dtype=torch.float32, device="cuda")
    Uo = torch.empty((x.numel(), 16), dtype=torch.float32, device="cuda")
    c = np.linspace(0.05, 0.95, 16).astype(np.float32)
    with pytest.raises(PifcmError) as e:
        ctx.ifcm_solve_noalloc(x, _P(C=16, m=2.0, eps=0.0, max_iter=2), 0.3, 0.4, c, U_out=Uo)
    assert e.value.status == PIFCM_E_INVALID and "scratch" in str(e.value)
    del x, Uo
    # general neighbourhoods are not covered
    x = torch.zeros((4, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(PifcmError) as e:
        ctx.ifcm_solve_noalloc(x, _P(C=4, m=2.0, V=2, eps=0.0, max_iter=2), 0.3, 0.4,
                               np.array([0.1, 0.4, 0.6, 0.9], np.float32))
    assert e.value.status == PIFCM_E_UNSUPPORTED
    # the context still works after a refusal
    raw, _ = synth.random_ellipsoids(shape=(5, 12, 17), seed=63, sigma=0.07)
    xs = ctx.pifcm_normalize(dev(raw))
    p = _P(C=4, m=2.0, eps=0.0, max_iter=3)
    c0 = np.array([0.1, 0.4, 0.6, 0.9], np.float32)
    a = ctx.ifcm_solve_noalloc(xs, p, 0.2, 0.1, c0, labels=True, want_hist=True)
    b = ctx.ifcm_solve(xs, p, 0.2, 0.1, c0, labels=True, want_hist=True)
    _same(a, b)
