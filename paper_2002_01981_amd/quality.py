"""Segmentation quality readouts and the speed/quality trade-off of eq (11).

The counting runs on the GPU (pifcm_confusion); the functions here reduce
the small count matrices and timing tables on the host.

    python -m paper_2002_01981_amd.quality   # FCM vs 3DPIFCM on brain phantoms

runs the comparison of section 6 on the synthetic brain phantom at 3, 5 and
9 % noise: misclassification against the phantom's classes and wall time of
plain FCM and of the full method (FCM start, swarm over (lambda, xi), final
solve), and the trade-off cost of eq (11) for several alpha.
"""
from __future__ import annotations

import itertools

import numpy as np


def misclassification(counts) -> float:
    """1 - (voxels on the diagonal) / (all voxels) of a confusion matrix
    [cluster][class]: cluster j read as class j (centres sorted ascending,
    classes numbered by intensity)."""
    c = np.asarray(counts, np.float64)
    n = c.sum()
    return float(1.0 - np.trace(c[: min(c.shape), : min(c.shape)]) / n) if n else 0.0


def best_map_misclassification(counts) -> float:
    """Misclassification under the best one-to-one map of clusters to
    classes (brute force; for up to 8 clusters)."""
    c = np.asarray(counts, np.float64)
    C, K = c.shape
    if C > 8 or K > 8:
        raise ValueError("brute force over maps is limited to 8 clusters")
    n = c.sum()
    best = 0.0
    for perm in itertools.permutations(range(K), min(C, K)):
        best = max(best, sum(c[j, perm[j]] for j in range(len(perm))))
    return float(1.0 - best / n) if n else 0.0


def tradeoff_cost(incS, S, alpha):
    """Eq (11): for algorithms a and images i, the mean over images of
    alpha * (incS - min) / (max - min) + (1 - alpha) * (S - min) / (max - min),
    minima and maxima taken over the algorithms for each image.  incS and S
    are [algorithms][images] (misclassification, seconds).  An image on which
    every algorithm has the same value contributes 0 for that term.
    Returns [algorithms]."""
    q = np.asarray(incS, np.float64)
    s = np.asarray(S, np.float64)

    def norm(v):
        lo, hi = v.min(axis=0, keepdims=True), v.max(axis=0, keepdims=True)
        span = hi - lo
        return np.where(span > 0, (v - lo) / np.where(span > 0, span, 1.0), 0.0)

    return (alpha * norm(q) + (1.0 - alpha) * norm(s)).mean(axis=1)


def _study():  # pragma: no cover - needs a GPU
    import time

    import torch

    import synth
    from . import Context, Params, segment

    ctx = Context(0)
    p = Params(C=4, m=2.0, eps=1e-5, max_iter=100)
    W = synth.WORKLOADS["brain-181x217x181"]
    ps = W["pso"]
    rows = []
    for f in (0.03, 0.05, 0.09):
        raw, truth = synth.brain_shells(shape=W["shape"], seed=W["seed"], noise_frac=f)
        tr = torch.from_numpy(truth.reshape(-1)).cuda()
        x = ctx.pifcm_normalize(torch.from_numpy(raw).cuda())
        ctx.pifcm_fcm_init(x, p)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c0, U0, _ = ctx.pifcm_fcm_init(x, p)
        fcm = ctx.ifcm_solve(x, p, 0.0, 0.0, c0, U_in=U0, labels=True)
        torch.cuda.synchronize()
        t_fcm = time.perf_counter() - t0
        st = synth.pso_streams(ps["seed"], ps["P"], ps["G"])
        t0 = time.perf_counter()
        seg = segment(ctx, x, p, st, w=ps["w"], c1=ps["c1"], c2=ps["c2"])
        torch.cuda.synchronize()
        t_pifcm = time.perf_counter() - t0
        q_fcm = misclassification(ctx.pifcm_confusion(fcm["labels"], tr, 4, 4))
        q_pifcm = misclassification(ctx.pifcm_confusion(seg["labels"], tr, 4, 4))
        rows.append((f, q_fcm, t_fcm, q_pifcm, t_pifcm, seg["best_pos"]))
        print(f"noise {f:.0%}: FCM incS {q_fcm:.4f} in {t_fcm:.3f} s; 3DPIFCM incS {q_pifcm:.4f} "
              f"in {t_pifcm:.3f} s at (lambda, xi) = {seg['best_pos']}", flush=True)
    incS = np.array([[r[1] for r in rows], [r[3] for r in rows]])
    S = np.array([[r[2] for r in rows], [r[4] for r in rows]])
    for a in (0.0, 0.25, 0.5, 0.75, 1.0):
        J = tradeoff_cost(incS, S, a)
        print(f"eq (11) alpha={a:.2f}: FCM {J[0]:.3f}  3DPIFCM {J[1]:.3f}")
    ctx.close()


if __name__ == "__main__":  # pragma: no cover
    _study()
