"""Composition of the libpifcm entry points into the paper's procedure.

Nothing here computes on the data: every step is one C-ABI call of
libpifcm (see abi.py); this module only orders the calls and moves small
host arrays between them.

- segment(): Algorithm 1 -- FCM initial state (step 2), the particle swarm
  over (lambda, xi) (steps 3-9, pifcm_pso), then one IFCM solve at the best
  particle from the shared initial state with labels (steps 10-11).
- IFCMObjective: torch.autograd.Function whose forward is J_K, the objective
  of eq (1) after exactly K iterations, and whose backward is the adjoint of
  those iterations (ifcm_backward).
- refine(): projected gradient steps on (lambda, xi) in [0, 1]^2 from a
  starting particle, using that gradient.
"""
from __future__ import annotations

import numpy as np

from .abi import PIFCM_SWARM_BATCHED, Context, Params


def segment(ctx: Context, x, p: Params, streams, w=0.7, c1=1.5, c2=1.5, init: Params = None,
            mode=PIFCM_SWARM_BATCHED):
    """Algorithm 1 on one normalised volume x (device float32 (Z, Y, X)).

    streams: dict(x0, v0 (P, 2), r1, r2 (G, P, 2)) of the swarm's random
    numbers, drawn by the caller.  init: parameters of the FCM initial solve
    (default: p's eps and max_iter).  Returns dict(best_pos, best_fit,
    fit_hist, pos_hist, centres0, U, centres, labels, J, iters)."""
    c0, U0, init_iters = ctx.pifcm_fcm_init(x, init or p)
    sw = ctx.pifcm_pso([x], p, streams, c0[None], [U0], w=w, c1=c1, c2=c2, mode=mode)
    lam, xi = (float(v) for v in sw["best_pos"][0])
    fin = ctx.ifcm_solve(x, p, lam, xi, c0, U_in=U0, labels=True)
    return dict(best_pos=sw["best_pos"][0], best_fit=float(sw["best_fit"][0]),
                fit_hist=sw["fit_hist"][0], pos_hist=sw["pos_hist"][0], centres0=c0,
                init_iters=init_iters, U=fin["U"], centres=fin["c"], labels=fin["labels"],
                J=fin["J"], iters=fin["iters"])


def _autograd_function():
    import torch

    class IFCMObjective(torch.autograd.Function):
        """J_K(lambda, xi, c^0) with U^0 held constant.

        apply(ctx_, x, p, U0, K, ckpt_every, params) where params is a CPU
        float64 tensor [lambda, xi, c_1 .. c_C]; returns a 0-d float64 tensor.
        The gradient flows to `params` only."""

        @staticmethod
        def forward(fctx, lib_ctx, x, p, U0, K, ckpt_every, params):
            v = params.detach().cpu().numpy().astype(np.float64)
            g = lib_ctx.ifcm_backward(x, p, float(v[0]), float(v[1]), v[2:].astype(np.float32),
                                      U0, int(K), int(ckpt_every))
            grad = np.concatenate([[g["dlam"], g["dxi"]], g["dc"]])
            fctx.save_for_backward(torch.from_numpy(grad))
            return torch.tensor(g["J"], dtype=torch.float64)

        @staticmethod
        def backward(fctx, gout):
            (grad,) = fctx.saved_tensors
            return None, None, None, None, None, None, gout.to(torch.float64) * grad

    return IFCMObjective


_IFCM_OBJECTIVE = None


def ifcm_objective():
    """The torch.autograd.Function class of J_K (built on first use)."""
    global _IFCM_OBJECTIVE
    if _IFCM_OBJECTIVE is None:
        _IFCM_OBJECTIVE = _autograd_function()
    return _IFCM_OBJECTIVE


def refine(ctx: Context, x, p: Params, lam, xi, centres0, U0, K, ckpt_every, steps=10, lr=0.05):
    """Projected gradient descent on (lambda, xi) over [0, 1]^2 for J_K from
    (centres0, U0).  The step along the gradient is lr / max|grad| (a step of
    lr in the steepest coordinate), halved while J_K does not decrease (at
    most 8 halvings per step).  Returns dict(pos, J, history) with history a
    list of (lambda, xi, J_K, dJ/dlambda, dJ/dxi)."""
    c = np.ascontiguousarray(centres0, np.float32)
    pos = np.array([lam, xi], np.float64)
    g = ctx.ifcm_backward(x, p, float(pos[0]), float(pos[1]), c, U0, K, ckpt_every)
    hist = [(pos[0], pos[1], g["J"], g["dlam"], g["dxi"])]
    for _ in range(steps):
        d = np.array([g["dlam"], g["dxi"]])
        scale = float(np.max(np.abs(d)))
        if scale == 0.0:
            break
        t = lr / scale
        moved = False
        for _ in range(9):
            cand = np.clip(pos - t * d, 0.0, 1.0)
            if np.array_equal(cand, pos):
                break
            gc = ctx.ifcm_backward(x, p, float(cand[0]), float(cand[1]), c, U0, K, ckpt_every)
            if gc["J"] < g["J"]:
                pos, g, moved = cand, gc, True
                break
            t *= 0.5
        if not moved:
            break
        hist.append((pos[0], pos[1], g["J"], g["dlam"], g["dxi"]))
    return dict(pos=pos, J=g["J"], history=hist)
