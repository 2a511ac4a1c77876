"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares it with an
independent formulation (an all-pairs set-builder scan of eq (9), textbook
FCM, a closed form of a degenerate volume) or with an invariant that a
dropped term, a wrong sign, index or transposed operand would break.
"""
import math

import numpy as np
import pytest

from pins import (all_flips, bruteforce_hf, bruteforce_step, random_memberships,
                  textbook_fcm_step)


def _rand_vol(rng, shape):
    return rng.random(shape).astype(np.float32)


# ---------------------------------------------------------------- eq (1)-(8)
def test_two_voxel_closed_form(orc):
    """A 1x1x2 volume: each voxel has exactly one neighbour, so eq (5) gives
    H_1j = u_2j and eq (7) gives F_1j = u_2j^2 whatever g and q are."""
    x = np.array([0.2, 0.8], np.float32).reshape(2, 1, 1)
    U0 = np.array([[0.9, 0.1], [0.2, 0.8]])
    c0 = np.array([0.3, 0.7])
    lam, xi = 0.5, 0.3
    p = orc.Params(C=2, m=2.0)
    Un, cn, J, H, F = orc.step(x, U0, c0, p, lam, xi, want_hf=True)
    xv = x.reshape(-1).astype(np.float64)
    Hx = U0[::-1]
    Fx = U0[::-1] ** 2
    a = 1 - lam * Hx - xi * Fx
    d2 = (xv[:, None] - c0[None, :]) ** 2 * a
    Jx = float((U0 ** 2 * d2).sum())
    inv = 1 / d2
    Ux = inv / inv.sum(1, keepdims=True)
    cx = (Ux ** 2 * xv[:, None]).sum(0) / (Ux ** 2).sum(0)
    np.testing.assert_allclose(H, Hx, rtol=0, atol=1e-15)
    np.testing.assert_allclose(F, Fx, rtol=0, atol=1e-15)
    assert abs(J - Jx) <= 1e-15
    np.testing.assert_allclose(Un, Ux, rtol=1e-13)
    np.testing.assert_allclose(cn, cx, rtol=1e-13)
    # the same numbers worked by hand on paper (1e-6)
    np.testing.assert_allclose(a.reshape(-1), [0.888, 0.408, 0.307, 0.947], atol=1e-6)
    assert abs(J - 0.0173436) < 1e-6
    np.testing.assert_allclose(Un, [[0.919913, 0.080087], [0.109835, 0.890165]], atol=1e-6)
    np.testing.assert_allclose(cn, [0.208433, 0.795182], atol=1e-6)


@pytest.mark.parametrize("m", [2.0, 2.5, 1.7])
def test_reduces_to_textbook_fcm(orc, m):
    """lambda = xi = 0: the attraction factor is 1 and one IFCM step is one
    step of plain FCM (eqs (1)-(3))."""
    rng = np.random.default_rng(7)
    x = _rand_vol(rng, (4, 5, 6))
    U = random_memberships(rng, x.size, 4)
    c = np.array([0.1, 0.35, 0.6, 0.9])
    p = orc.Params(C=4, m=m)
    Un, cn, J = orc.step(x, U, c, p, 0.0, 0.0)
    Ut, ctb, Jt = textbook_fcm_step(x, U, c, m)
    np.testing.assert_allclose(Un, Ut, rtol=1e-12)
    np.testing.assert_allclose(cn, ctb, rtol=1e-12)
    assert abs(J - Jt) <= 1e-12 * abs(Jt)


@pytest.mark.parametrize("shape", [(2, 4, 4), (3, 3, 3), (3, 4, 5), (1, 1, 5)])
def test_bruteforce_setbuilder(orc, shape):
    """Eq (9) with L = 3 (0 < |d|^2 < 4) is the 26-voxel cube; the oracle's
    offset walk must equal the literal all-pairs scan, borders included."""
    rng = np.random.default_rng(11 + sum(shape))
    x = _rand_vol(rng, shape)
    U = random_memberships(rng, x.size, 3)
    c = np.array([0.2, 0.5, 0.8])
    lam, xi = 0.37, 0.41
    p = orc.Params(C=3, m=2.0)
    Un, cn, J, H, F = orc.step(x, U, c, p, lam, xi, want_hf=True)
    Ub, cb, Jb, Hb, Fb = bruteforce_step(x, U, c, lam, xi, 2.0, rings="setbuilder", L=3)
    np.testing.assert_allclose(H, Hb, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(F, Fb, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Un, Ub, rtol=1e-12)
    np.testing.assert_allclose(cn, cb, rtol=1e-12)
    assert abs(J - Jb) <= 1e-12 * abs(Jb)


def test_bruteforce_flat_region(orc):
    """A voxel whose whole neighbourhood has its own intensity takes the
    equal-weight mean in eq (5)."""
    rng = np.random.default_rng(3)
    x = np.full((3, 3, 3), 0.5, np.float32)
    x[0, 0, 0] = 0.9  # one differing corner: most voxels still see g > 0
    x2 = np.full((3, 3, 3), 0.5, np.float32)  # fully flat: every sum of g is 0
    for vol in (x, x2):
        U = random_memberships(rng, vol.size, 2)
        c = np.array([0.3, 0.7])
        p = orc.Params(C=2, m=2.0)
        _, _, _, H, F = orc.step(vol, U, c, p, 0.3, 0.2, want_hf=True)
        Hb, Fb = bruteforce_hf(vol, U, rings="setbuilder", L=3)
        np.testing.assert_allclose(H, Hb, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(F, Fb, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("V,h", [(2, 1.0), (2, 0.4), (3, 2.0)])
def test_bruteforce_deeper_rings(orc, V, h):
    """Rings r = 1..V (Chebyshev) with the decay weights of eq (10)."""
    rng = np.random.default_rng(100 + V)
    x = _rand_vol(rng, (4, 5, 5))
    U = random_memberships(rng, x.size, 3)
    p = orc.Params(C=3, m=2.0, V=V, h=h)
    _, _, _, H, F = orc.step(x, U, [0.2, 0.5, 0.8], p, 0.3, 0.3, want_hf=True)
    Hb, Fb = bruteforce_hf(x, U, V=V, h=h, rings="chebyshev")
    np.testing.assert_allclose(H, Hb, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(F, Fb, rtol=1e-12, atol=1e-15)


def test_bruteforce_alternative_readings(orc):
    """Squared-distance shells and the q (not q^2) weight."""
    rng = np.random.default_rng(5)
    x = _rand_vol(rng, (3, 4, 4))
    U = random_memberships(rng, x.size, 2)
    p = orc.Params(C=2, m=2.0, V=3, h=1.5, flags=orc.OR_SHELL_SQDIST | orc.OR_Q2_SQDIST)
    _, _, _, H, F = orc.step(x, U, [0.3, 0.7], p, 0.3, 0.3, want_hf=True)
    Hb, Fb = bruteforce_hf(x, U, V=3, h=1.5, rings="sqdist", q2_literal=False)
    np.testing.assert_allclose(H, Hb, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(F, Fb, rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------- invariants
def test_memberships_and_attraction_bounds(orc):
    """Eq (2) rows sum to 1; H and F of eqs (5), (7) are convex combinations:
    H, F in [0, 1], sum_j H = 1, sum_j F <= 1."""
    rng = np.random.default_rng(9)
    x = _rand_vol(rng, (5, 6, 7))
    U = random_memberships(rng, x.size, 4)
    p = orc.Params(C=4, m=2.0)
    Un, _, _, H, F = orc.step(x, U, [0.1, 0.4, 0.6, 0.9], p, 0.6, 0.7, want_hf=True)
    np.testing.assert_allclose(Un.sum(1), 1.0, atol=1e-12)
    assert H.min() >= 0 and H.max() <= 1 + 1e-15
    assert F.min() >= 0 and F.max() <= 1 + 1e-15
    np.testing.assert_allclose(H.sum(1), 1.0, atol=1e-12)
    assert F.sum(1).max() <= 1 + 1e-12


def test_uniform_memberships_cancel_attraction(orc):
    """With U = 1/C everywhere, H = 1/C and F = 1/C^2 for every cluster, the
    factor of eq (4) does not depend on j, so memberships and centres equal
    the FCM step and J scales by that factor."""
    rng = np.random.default_rng(13)
    x = _rand_vol(rng, (3, 4, 5))
    C = 4
    U = np.full((x.size, C), 1.0 / C)
    c = np.array([0.15, 0.4, 0.65, 0.85])
    lam, xi = 0.45, 0.35
    p = orc.Params(C=C, m=2.0)
    Un, cn, J, H, F = orc.step(x, U, c, p, lam, xi, want_hf=True)
    np.testing.assert_allclose(H, 1.0 / C, atol=1e-15)
    np.testing.assert_allclose(F, 1.0 / C ** 2, atol=1e-15)
    Ut, ct, Jt = textbook_fcm_step(x, U, c, 2.0)
    np.testing.assert_allclose(Un, Ut, rtol=1e-12)
    np.testing.assert_allclose(cn, ct, rtol=1e-12)
    a = 1 - lam / C - xi / C ** 2
    assert abs(J - a * Jt) <= 1e-12 * Jt


def test_m2_identity(orc):
    """For m = 2, eq (2) gives sum_j u_j^2 d_j^2 = 1 / sum_j (1 / d_j^2)."""
    rng = np.random.default_rng(21)
    x = _rand_vol(rng, (3, 4, 4))
    U = random_memberships(rng, x.size, 3)
    c = np.array([0.25, 0.5, 0.75])
    lam, xi = 0.3, 0.2
    p = orc.Params(C=3, m=2.0)
    Un, _, _, H, F = orc.step(x, U, c, p, lam, xi, want_hf=True)
    xv = x.reshape(-1).astype(np.float64)
    d2 = np.maximum((xv[:, None] - c) ** 2 * (1 - lam * H - xi * F), 1e-12)
    np.testing.assert_allclose((Un ** 2 * d2).sum(1), 1 / (1 / d2).sum(1), rtol=1e-12)


def test_fcm_objective_never_increases(orc):
    """At lambda = xi = 0 the iteration is FCM's alternating minimisation, so
    J of successive states never increases."""
    import synth
    raw, _ = synth.nested_ellipsoids()
    x = orc.normalize(raw)
    p = orc.Params(C=4, m=2.0, eps=0.0, max_iter=25)
    out = orc.solve(x, [0.125, 0.375, 0.625, 0.875], p, 0.0, 0.0, want_hist=True)
    Jh = out["J_hist"]
    assert len(Jh) == 25
    assert np.all(Jh[1:] <= Jh[:-1] * (1 + 1e-12))


def test_constant_image(orc):
    """A constant image normalises to zeros; FCM then puts every centre at 0,
    memberships become uniform, and every label is cluster 0."""
    raw = np.full((3, 4, 5), 7.25, np.float32)
    x = orc.normalize(raw)
    assert np.all(x == 0)
    p = orc.Params(C=4, m=2.0, eps=0.0, max_iter=5)
    c, U, _ = orc.fcm_init(x, p)
    assert np.all(c == 0)
    np.testing.assert_allclose(U, 0.25, atol=1e-12)
    out = orc.solve(x, c, p, 0.6, 0.3, U0=U)
    assert np.all(out["c"] == 0)
    np.testing.assert_allclose(out["U"], 0.25, atol=1e-12)
    assert np.all(orc.labels(out["U"], 4) == 0)


def test_symmetries(orc):
    """Axis flips and the X<->Y transpose of a square volume commute with the
    solve; permuting the initial centres permutes the outputs."""
    rng = np.random.default_rng(17)
    x = _rand_vol(rng, (4, 5, 5))
    c0 = np.array([0.2, 0.5, 0.8])
    p = orc.Params(C=3, m=2.0, eps=0.0, max_iter=6)
    lam, xi = 0.4, 0.3
    base = orc.solve(x, c0, p, lam, xi)
    Ub = base["U"].reshape(x.shape + (3,))
    for axes in all_flips():
        xf = np.flip(x, axes).copy()
        o = orc.solve(xf, c0, p, lam, xi)
        np.testing.assert_allclose(o["U"].reshape(x.shape + (3,)), np.flip(Ub, axes), atol=1e-12)
        np.testing.assert_allclose(o["c"], base["c"], rtol=1e-12)
        assert abs(o["J"] - base["J"]) <= 1e-12 * base["J"]
    xt = np.ascontiguousarray(np.transpose(x, (0, 2, 1)))
    o = orc.solve(xt, c0, p, lam, xi)
    np.testing.assert_allclose(o["U"].reshape(x.shape + (3,)), np.transpose(Ub, (0, 2, 1, 3)),
                               atol=1e-12)
    perm = [2, 0, 1]
    o = orc.solve(x, c0[perm], p, lam, xi)
    np.testing.assert_allclose(o["U"], base["U"][:, perm], atol=1e-12)
    np.testing.assert_allclose(o["c"], base["c"][perm], rtol=1e-12)


# ------------------------------------------------------------- normalisation
def test_normalize(orc):
    rng = np.random.default_rng(2)
    k = rng.integers(-3000, 3000, size=(4, 5, 6))
    raw = (k / 1024.0).astype(np.float32)
    x = orc.normalize(raw)
    assert x.dtype == np.float32
    assert x.min() == 0.0 and x.max() == 1.0
    assert x.reshape(-1)[np.argmin(raw)] == 0.0 and x.reshape(-1)[np.argmax(raw)] == 1.0
    order = np.argsort(raw.reshape(-1), kind="stable")
    assert np.all(np.diff(x.reshape(-1)[order]) >= 0)
    # affine maps by powers of two are exact, so the result is bit-identical
    raw2 = (raw * np.float32(4.0) + np.float32(8.0)).astype(np.float32)
    assert np.array_equal(orc.normalize(raw2), x)
    bad = raw.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(ValueError):
        orc.normalize(bad)


# ------------------------------------------------------------------ init/labels
def test_fcm_init_sorted_and_consistent(orc):
    import synth
    raw, _ = synth.nested_ellipsoids()
    x = orc.normalize(raw)
    p = orc.Params(C=4, m=2.0, eps=1e-5, max_iter=50)
    c, U, it = orc.fcm_init(x, p)
    assert np.all(np.diff(c) >= 0)
    o = orc.solve(x, [0.125, 0.375, 0.625, 0.875], p, 0.0, 0.0)
    order = np.argsort(o["c"], kind="stable")
    np.testing.assert_allclose(c, o["c"][order], rtol=0, atol=0)
    np.testing.assert_allclose(U, o["U"][:, order], rtol=0, atol=0)
    assert it == o["iters"] and 2 <= it <= 50


def test_labels_first_maximum(orc):
    rng = np.random.default_rng(4)
    U = random_memberships(rng, 200, 4)
    U[:20] = 0.25                      # four-way ties
    U[20:40, 1] = U[20:40, 3] = 0.4    # two-way ties
    U[20:40, 0] = U[20:40, 2] = 0.1
    np.testing.assert_array_equal(orc.labels(U, 4), np.argmax(U, axis=1))


# ------------------------------------------------------------------ PSO
def _pso_case(orc, P=4, G=3, seed=5):
    import synth
    rng = np.random.default_rng(seed)
    x = _rand_vol(rng, (2, 4, 4))
    p = orc.Params(C=2, m=2.0, eps=1e-6, max_iter=8)
    c0, U0, _ = orc.fcm_init(x, p)
    st = synth.pso_streams(seed, P, G)
    return x, p, c0, U0, st


def test_pso_frozen_swarm(orc):
    """With zero velocity and zero random coefficients no particle moves."""
    x, p, c0, U0, st = _pso_case(orc)
    st = dict(x0=st["x0"], v0=np.zeros_like(st["v0"]), r1=np.zeros_like(st["r1"]),
              r2=np.zeros_like(st["r2"]))
    out = orc.pso(x, c0, U0, p, st)
    for g in range(3):
        np.testing.assert_array_equal(out["pos_hist"][g], st["x0"])
        np.testing.assert_array_equal(out["fit_hist"][g], out["fit_hist"][0])


def test_pso_one_generation_by_hand(orc):
    """Generation 1 positions follow the velocity rule from generation 0:
    pbest = x0, gbest = first particle with the lowest fitness."""
    x, p, c0, U0, st = _pso_case(orc, P=5, G=2)
    w, c1, c2 = 0.7, 1.5, 1.5
    out = orc.pso(x, c0, U0, p, st, w, c1, c2)
    f0 = out["fit_hist"][0]
    gbest = st["x0"][int(np.argmin(f0))]
    v = w * st["v0"] + c1 * st["r1"][0] * 0.0 + c2 * st["r2"][0] * (gbest - st["x0"])
    np.testing.assert_allclose(out["pos_hist"][1], np.clip(st["x0"] + v, 0, 1), rtol=0,
                               atol=1e-15)
    fits = out["fit_hist"].reshape(-1)
    assert out["best_fit"] == fits.min()


def test_pso_personal_best_pull(orc):
    """The personal-best term: with inertia 1, no global pull and c1 r1 = 2,
    a particle moves by v0 in the first update; in the second it returns to
    its start if that was no worse (pbest stays x0: x0 + 2 v0 - 2 v0 = x0),
    and otherwise moves on by v0 again (pbest is the current position).
    Starts and velocities are kept away from the box edges."""
    x, p, c0, U0, st = _pso_case(orc, P=8, G=3, seed=11)
    rng = np.random.default_rng(12)
    x0 = 0.3 + 0.4 * rng.random((8, 2))
    v0 = 0.05 * (2 * rng.random((8, 2)) - 1)
    st = dict(x0=x0, v0=v0, r1=np.ones_like(st["r1"]), r2=np.zeros_like(st["r2"]))
    out = orc.pso(x, c0, U0, p, st, w=1.0, c1=2.0, c2=0.0)
    ph, fh = out["pos_hist"], out["fit_hist"]
    np.testing.assert_allclose(ph[1], x0 + v0, rtol=0, atol=1e-15)
    improved = fh[1] < fh[0]
    expect = np.where(improved[:, None], x0 + 2 * v0, x0)
    np.testing.assert_allclose(ph[2], expect, rtol=0, atol=1e-15)
    assert improved.any() and not improved.all()


def test_pso_global_best_pull(orc):
    """The global-best term alone (w = c1 = 0, c2 r2 = 1) puts every particle
    on the best position of the previous generations after each update."""
    x, p, c0, U0, st = _pso_case(orc, P=6, G=3, seed=13)
    st = dict(x0=st["x0"], v0=st["v0"], r1=np.zeros_like(st["r1"]), r2=np.ones_like(st["r2"]))
    out = orc.pso(x, c0, U0, p, st, w=0.0, c1=0.0, c2=1.0)
    ph, fh = out["pos_hist"], out["fit_hist"]
    best = ph[0][int(np.argmin(fh[0]))]
    np.testing.assert_allclose(ph[1], np.broadcast_to(best, ph[1].shape), rtol=0, atol=1e-15)


def test_pso_best_is_reevaluated_fitness(orc):
    x, p, c0, U0, st = _pso_case(orc, P=6, G=4, seed=8)
    out = orc.pso(x, c0, U0, p, st)
    lam, xi = out["best_pos"]
    o = orc.solve(x, c0, p, lam, xi, U0=U0)
    assert o["J"] == out["best_fit"]
    assert out["best_fit"] == out["fit_hist"].min()
    assert np.all((out["pos_hist"] >= 0) & (out["pos_hist"] <= 1))


# ------------------------------------------------------------------ gradient
def test_fd_gradient_closed_form_at_K0(orc):
    """At K = 0 the fitness is J(U0, c0) = sum u^m (x - c)^2 a, so
    dJ/dlambda = -sum u^m (x-c)^2 H, dJ/dxi = -sum u^m (x-c)^2 F and
    dJ/dc_j = -2 sum_i u_ij^m (x_i - c_j) a_ij (no floor active)."""
    rng = np.random.default_rng(31)
    x = _rand_vol(rng, (3, 3, 4))
    C = 3
    U0 = random_memberships(rng, x.size, C)
    c0 = np.array([0.2, 0.5, 0.8])
    lam, xi = 0.3, 0.2
    p = orc.Params(C=C, m=2.0)
    J, g = orc.fd_grad(x, c0, U0, p, lam, xi, K=0, step=1e-5)
    H, F = bruteforce_hf(x, U0, rings="setbuilder", L=3)
    xv = x.reshape(-1).astype(np.float64)
    dx2 = (xv[:, None] - c0) ** 2
    a = 1 - lam * H - xi * F
    um = U0 ** 2
    exp = [-(um * dx2 * H).sum(), -(um * dx2 * F).sum()]
    exp += list(-2 * (um * (xv[:, None] - c0) * a).sum(0))
    np.testing.assert_allclose(g, exp, rtol=1e-7, atol=1e-10)
    assert abs(J - float((um * dx2 * a).sum())) <= 1e-13


def test_fd_gradient_step_agreement(orc):
    rng = np.random.default_rng(33)
    x = _rand_vol(rng, (3, 4, 4))
    p = orc.Params(C=3, m=2.0)
    c0, U0, _ = orc.fcm_init(x, orc.Params(C=3, m=2.0, eps=1e-6, max_iter=20))
    _, g1 = orc.fd_grad(x, c0, U0, p, 0.2, 0.3, K=3, step=1e-4)
    _, g2 = orc.fd_grad(x, c0, U0, p, 0.2, 0.3, K=3, step=5e-5)
    # truncation error is O(h^2): compare norm-wise against the gradient's scale
    assert np.max(np.abs(g1 - g2)) <= 1e-6 * np.max(np.abs(g1))


def test_thread_count_does_not_change_results(orc):
    rng = np.random.default_rng(41)
    x = _rand_vol(rng, (6, 5, 4))
    p = orc.Params(C=3, m=2.0, eps=0.0, max_iter=4)
    n0 = orc.get_threads()
    try:
        orc.set_threads(1)
        a = orc.solve(x, [0.2, 0.5, 0.8], p, 0.3, 0.4)
        orc.set_threads(3)
        b = orc.solve(x, [0.2, 0.5, 0.8], p, 0.3, 0.4)
    finally:
        orc.set_threads(n0)
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["c"], b["c"])
    assert a["J"] == b["J"]
    assert math.isfinite(a["J"])


def test_pso_interleaved_frozen_swarm_is_one_long_solve(orc):
    """With a frozen swarm each particle keeps its (lambda, xi), so after
    generation g its state is (g + 1) * steps iterations of one solve from
    (c0, U0): the carried state must reproduce a long solve exactly."""
    x, p, c0, U0, st = _pso_case(orc, P=3, G=4, seed=9)
    st = dict(x0=st["x0"], v0=np.zeros_like(st["v0"]), r1=np.zeros_like(st["r1"]),
              r2=np.zeros_like(st["r2"]))
    steps = 2
    out = orc.pso_interleaved(x, c0, U0, p, st, steps=steps)
    for g in range(4):
        np.testing.assert_array_equal(out["pos_hist"][g], st["x0"])
        for k in range(3):
            lam, xi = st["x0"][k]
            o = orc.solve(x, c0, orc.Params(C=p.C, m=p.m, eps=0.0, max_iter=(g + 1) * steps),
                          lam, xi, U0=U0)
            assert out["fit_hist"][g, k] == o["J"]
    k = int(np.argmin(out["fit_hist"].min(axis=0)))
    lam, xi = st["x0"][k]
    o = orc.solve(x, c0, orc.Params(C=p.C, m=p.m, eps=0.0, max_iter=4 * steps), lam, xi, U0=U0)
    np.testing.assert_array_equal(out["U_best"], o["U"])
    np.testing.assert_array_equal(out["c_best"], o["c"])


def test_pso_interleaved_first_generation_is_the_plain_swarm(orc):
    """Generation 0 starts every particle from (c0, U0): its fitnesses are the
    plain swarm's with max_iter = steps, and the first move is the same."""
    x, p, c0, U0, st = _pso_case(orc, P=5, G=2, seed=10)
    steps = 3
    a = orc.pso_interleaved(x, c0, U0, p, st, steps=steps)
    b = orc.pso(x, c0, U0, orc.Params(C=p.C, m=p.m, eps=0.0, max_iter=steps), st)
    np.testing.assert_array_equal(a["fit_hist"][0], b["fit_hist"][0])
    np.testing.assert_array_equal(a["pos_hist"][1], b["pos_hist"][1])
    # generation 1 continues from the carried states, so it differs from a
    # fresh solve at the same particles
    assert not np.array_equal(a["fit_hist"][1], b["fit_hist"][1])


# ------------------------------------------------------------------ slab mode
def _bruteforce_slab_step(x, U, c, lam, xi, zbeg, zend, m=2.0):
    """One step in which only the planes [zbeg, zend) change: H and F from the
    literal neighbourhood scan of the whole volume, eqs (4), (2) on the
    active voxels, eq (3) and eq (1) summed over the active voxels."""
    H, F = bruteforce_hf(x, U)
    nz, ny, nx = x.shape
    flat = np.asarray(x, np.float64).reshape(-1)
    U = np.asarray(U, np.float64).reshape(flat.size, -1)
    act = np.zeros((nz, ny, nx), bool)
    act[zbeg:zend] = True
    act = act.reshape(-1)
    a = 1.0 - lam * H - xi * F
    d2 = np.maximum((flat[:, None] - np.asarray(c)[None, :]) ** 2 * a, 1e-12)
    J = float((U[act] ** m * d2[act]).sum())
    w = (1.0 / d2) ** (1.0 / (m - 1.0))
    Un = U.copy()
    Un[act] = (w / w.sum(1, keepdims=True))[act]
    um = Un[act] ** m
    cn = (um * flat[act, None]).sum(0) / um.sum(0)
    return Un, cn, J


def test_slab_of_the_whole_volume_is_the_solve(orc):
    rng = np.random.default_rng(21)
    x = _rand_vol(rng, (4, 5, 6))
    U0 = random_memberships(rng, x.size, 3)
    p = orc.Params(C=3, m=2.0, eps=0.0, max_iter=4)
    c0 = np.array([0.2, 0.5, 0.8])
    a = orc.solve(x, c0, p, 0.3, 0.4, U0=U0)
    b = orc.solve_slab(x, c0, p, 0.3, 0.4, U0, 0, 4)
    np.testing.assert_array_equal(a["U"], b["U"])
    np.testing.assert_array_equal(a["c"], b["c"])
    assert a["J"] == b["J"]


@pytest.mark.parametrize("zbeg,zend", [(0, 1), (2, 3), (4, 5), (1, 4)])
def test_slab_matches_bruteforce_with_fixed_context(orc, zbeg, zend):
    rng = np.random.default_rng(22 + zbeg)
    x = _rand_vol(rng, (5, 4, 6))
    U0 = random_memberships(rng, x.size, 3)
    c0 = np.array([0.15, 0.5, 0.85])
    lam, xi = 0.35, 0.25
    U1, c1, J0 = _bruteforce_slab_step(x, U0, c0, lam, xi, zbeg, zend)
    U2, c2, J1 = _bruteforce_slab_step(x, U1, c1, lam, xi, zbeg, zend)
    o = orc.solve_slab(x, c0, orc.Params(C=3, m=2.0, eps=0.0, max_iter=2), lam, xi, U0, zbeg,
                       zend, want_hist=True)
    np.testing.assert_allclose(o["U"], U2, rtol=0, atol=1e-13)
    np.testing.assert_allclose(o["c"], c2, rtol=1e-13)
    np.testing.assert_allclose(o["J_hist"], [J0, J1], rtol=1e-13)
    # the context planes never change
    keep = np.ones(x.shape, bool)
    keep[zbeg:zend] = False
    np.testing.assert_array_equal(o["U"][keep.reshape(-1)], U0[keep.reshape(-1)])


# ------------------------------------------------- loop control, fitness, U^(0)
def _nested_case(orc):
    import synth
    raw, _ = synth.nested_ellipsoids()
    return orc.normalize(raw), np.array([0.125, 0.375, 0.625, 0.875])


def _first_stop(Jh, eps, cap):
    """First iteration t >= 2 after which |J(t-1) - J(t-2)| <= eps |J(t-2)|,
    J(s) being the objective of state s; cap if none."""
    for t in range(2, cap + 1):
        if abs(Jh[t - 1] - Jh[t - 2]) <= eps * abs(Jh[t - 2]):
            return t
    return cap


@pytest.mark.parametrize("lam,xi", [(0.0, 0.0), (0.3, 0.2)])
def test_stop_rule_is_the_first_small_relative_change(orc, lam, xi):
    """Section 4 and Algorithm 2 end the iteration once the objective stops
    changing (reading R12: relative change of J, tested from t = 2).  A run
    with eps = 0 lists J of every state; for each eps the stopping iteration
    T is found from that list by hand, and the eps run must stop exactly
    there, returning the state of a plain T-iteration run bit for bit."""
    x, c0 = _nested_case(orc)
    cap = 40
    ref = orc.solve(x, c0, orc.Params(C=4, m=2.0, eps=0.0, max_iter=cap), lam, xi, want_hist=True)
    Jh = ref["J_hist"]
    assert len(Jh) == cap
    rel = sorted({abs(Jh[t - 1] - Jh[t - 2]) / abs(Jh[t - 2]) for t in range(2, cap + 1)})
    # eps = 0 means "run max_iter"; a converged FCM run may repeat J exactly
    rel = [r for r in rel if r > 0]
    # thresholds strictly between consecutive relative changes (no ties),
    # above the largest one (T = 2) and below the smallest positive one
    cuts = [rel[-1] * 2.0, rel[0] * 0.5]
    cuts += [math.sqrt(a * b) for a, b in zip(rel[:-1], rel[1:]) if a > 0 and b > a * (1 + 1e-6)]
    seen = set()
    for eps in cuts[:12]:
        T = _first_stop(Jh, eps, cap)
        seen.add(T)
        o = orc.solve(x, c0, orc.Params(C=4, m=2.0, eps=eps, max_iter=cap), lam, xi,
                      want_hist=True)
        assert o["iters"] == T, (eps, o["iters"], T)
        np.testing.assert_array_equal(o["J_hist"], Jh[:T])
        f = orc.solve(x, c0, orc.Params(C=4, m=2.0, eps=0.0, max_iter=T), lam, xi)
        assert np.array_equal(o["U"], f["U"]) and np.array_equal(o["c"], f["c"])
        assert o["J"] == f["J"]
    assert 2 in seen and len(seen) >= 3


@pytest.mark.parametrize("lam,xi", [(0.0, 0.0), (0.35, 0.25)])
def test_fitness_is_the_objective_of_the_final_state(orc, lam, xi):
    """Algorithm 1 step 4 ranks particles by J_m of eq (1), of the state the
    run ends in (reading R9).  A run of T iterations reports J(U^(T), c^(T)),
    which a run of T + 1 iterations lists as the objective of its last input
    state.  With no iteration the fitness is J of the initial state."""
    x, c0 = _nested_case(orc)
    for T in (0, 1, 2, 5):
        a = orc.solve(x, c0, orc.Params(C=4, m=2.0, eps=0.0, max_iter=T), lam, xi)
        b = orc.solve(x, c0, orc.Params(C=4, m=2.0, eps=0.0, max_iter=T + 1), lam, xi,
                      want_hist=True)
        assert a["iters"] == T
        assert a["J"] == b["J_hist"][T], (T, a["J"], b["J_hist"][T])
        if lam == 0.0 and xi == 0.0:
            # plain FCM: the objective of the returned (U, c) by the textbook formula
            _, _, Jt = textbook_fcm_step(x, a["U"], a["c"], 2.0)
            assert abs(a["J"] - Jt) <= 1e-12 * Jt


@pytest.mark.parametrize("m", [2.0, 2.5, 1.7])
def test_initial_memberships_are_fcm_memberships_of_the_centres(orc, m):
    """Without a given U^(0) the run starts from eq (2) with the attraction
    factor 1: the textbook FCM memberships of the initial centres.  A solve
    with no iteration must hand that state back, and a one-step solve from it
    must equal the one-step solve given the textbook memberships."""
    rng = np.random.default_rng(61)
    x = _rand_vol(rng, (4, 5, 6))
    c = np.array([0.1, 0.35, 0.6, 0.9])
    Ut, _, _ = textbook_fcm_step(x, random_memberships(rng, x.size, 4), c, m)
    p = orc.Params(C=4, m=m, eps=0.0, max_iter=0)
    np.testing.assert_allclose(orc.init_memberships(x, c, p), Ut, rtol=1e-12, atol=1e-15)
    z = orc.solve(x, c, p, 0.4, 0.3)
    np.testing.assert_allclose(z["U"], Ut, rtol=1e-12, atol=1e-15)
    p1 = orc.Params(C=4, m=m, eps=0.0, max_iter=1)
    a = orc.solve(x, c, p1, 0.4, 0.3)
    b = orc.solve(x, c, p1, 0.4, 0.3, U0=Ut)
    np.testing.assert_allclose(a["U"], b["U"], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(a["c"], b["c"], rtol=1e-11)
