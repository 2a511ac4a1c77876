"""Helpers of the GPU parity tests (comparison rules, device copies)."""
import numpy as np

# Parity bar: memberships and centres within 1e-4 relative, measured
# norm-wise (max |gpu - oracle| / max |oracle| per array) because the
# element-wise relative error of a membership near 0 carries no meaning.
TOL = 1e-4
# Labels must match except where the oracle's two largest memberships are
# closer than this (both precisions may then pick either cluster).
TIE_BAND = 1e-5


# For lambda + xi > 1 the attraction factor 1 - lambda H - xi F of eq (4)
# changes sign on a data-dependent set of voxels and the 1e-12 floor of the
# squared distance engages there; the membership map is ill-conditioned at
# those voxels (a plain float32 emulation of the step in numpy differs from
# float64 by up to 2e-3 max-norm after a few iterations while the 2-norm
# stays below 4e-5).  In that saturated regime memberships are held to the
# 2-norm relative error and labels to a wider tie band; centres and J keep
# the max-norm bar.
SATURATED_TIE_BAND = 1e-2


def saturated(lam, xi):
    return lam + xi > 1.0


# One step from a given state is held to the max-norm bar on every voxel
# whose attraction factor a_ij = 1 - lambda H_ij - xi F_ij (eq (4)) is at
# least A_MIN away from zero for every cluster.  Float32 rounding of a
# (about 1e-6 after the 26-term sums of eqs (5), (7)) then moves a positive
# d^2 by at most ~2e-5 relative, and cannot flip the sign of a negative one,
# whose d^2 is the 1e-12 floor on both sides: a membership moves by less
# than 1e-5.  Voxels with a factor near zero are ill-conditioned in either
# precision (whether the floor engages, and by how much d^2 exceeds it,
# depends on rounding; a float32 restatement of the step shows errors of
# 1e-2 there, see test_fp32_conditioning.py): they are checked for valid
# memberships and labels within the wide tie band.
A_MIN = 0.05


def regular_voxels(H, F, lam, xi, a_min=A_MIN):
    """Per voxel: True where every cluster's eq (4) factor a satisfies
    |a| >= a_min."""
    a = 1.0 - lam * np.asarray(H) - xi * np.asarray(F)
    return np.all(np.abs(a) >= a_min, axis=1)


def check_step_memberships(Ug, lab_g, Uo, H, F, lam, xi, C, tol=TOL):
    """One step from the same state on both sides: max-norm bar and the
    narrow tie band on regular voxels; on the others (a factor of eq (4)
    within A_MIN of zero) valid memberships and the wide tie band.  Returns
    the number of irregular voxels."""
    Ug = np.asarray(Ug, np.float64).reshape(-1, C)
    Uo = np.asarray(Uo, np.float64).reshape(-1, C)
    reg = regular_voxels(H, F, lam, xi)
    scale = float(np.max(np.abs(Uo)))
    if reg.any():
        e = float(np.max(np.abs(Ug[reg] - Uo[reg]))) / scale
        assert e <= tol, f"max-norm error {e:.3g} on regular voxels"
    assert np.all(Ug >= 0.0) and np.all(Ug <= 1.0 + 1e-6)
    assert np.max(np.abs(Ug.sum(1) - 1.0)) <= 1e-5
    if lab_g is not None:
        lab = np.asarray(lab_g).reshape(-1)
        check_labels(lab[reg], Uo[reg], C, TIE_BAND)
        if (~reg).any():
            check_labels(lab[~reg], Uo[~reg], C, SATURATED_TIE_BAND)
    return int((~reg).sum())


def rel2(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm((a - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = float(np.max(np.abs(ref))) if ref.size else 1.0
    return float(np.max(np.abs(a - ref))) / max(scale, 1e-300)


def check_labels(lab_gpu, U_ref, C, band=TIE_BAND):
    U = np.asarray(U_ref, np.float64).reshape(-1, C)
    srt = np.sort(U, axis=1)
    gap = srt[:, -1] - srt[:, -2]
    ref = np.argmax(U, axis=1)
    ok = gap >= band
    lab = np.asarray(lab_gpu).reshape(-1)
    bad = np.nonzero(lab[ok] != ref[ok])[0]
    assert bad.size == 0, f"{bad.size} labels differ outside the tie band"
    return int((~ok).sum())


def random_memberships_f32(rng, n, C):
    a = rng.random((n, C)) + 0.05
    return (a / a.sum(1, keepdims=True)).astype(np.float32)


def pso_replay(fit_hist, streams, w=0.7, c1=1.5, c2=1.5):
    """Re-run the global-best swarm rules on given fitnesses (G, P).
    Returns (pos_hist (G, P, 2), best_pos, best_fit, margin), where margin is
    the smallest relative gap of any comparison the swarm decided: a
    trajectory fed with fitnesses perturbed by less than that takes the
    same decisions."""
    G, P = fit_hist.shape
    pos = np.array(streams["x0"], np.float64)
    vel = np.array(streams["v0"], np.float64)
    pb = pos.copy()
    pbf = np.zeros(P)
    margin = np.inf
    ph = np.empty((G, P, 2))
    gb = None
    for g in range(G):
        ph[g] = pos
        for q in range(P):
            f = fit_hist[g, q]
            if g:
                margin = min(margin, abs(f - pbf[q]) / abs(pbf[q]))
            if g == 0 or f < pbf[q]:
                pbf[q] = f
                pb[q] = pos[q]
        if P > 1:
            o = np.sort(pbf)
            margin = min(margin, (o[1] - o[0]) / abs(o[0]))
        k = int(np.argmin(pbf))  # lowest index among equal minima
        gb = pb[k].copy()
        if g + 1 == G:
            break
        for q in range(P):
            for d in range(2):
                v = (w * vel[q, d] + c1 * streams["r1"][g, q, d] * (pb[q, d] - pos[q, d])
                     + c2 * streams["r2"][g, q, d] * (gb[d] - pos[q, d]))
                vel[q, d] = v
                pos[q, d] = min(max(pos[q, d] + v, 0.0), 1.0)
    return ph, gb, float(pbf.min()), margin
