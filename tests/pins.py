"""Independent references that pin the FP64 oracle.

Nothing here calls the oracle.  These are deliberately different
formulations of the same mathematics:

* `bruteforce_hf` / `bruteforce_step` scan *every* pair of voxels and keep a
  neighbour by the literal set-builder condition of eq (9)
  (0 < dX^2 + dY^2 + dZ^2 < 2^(L-1)), or by Chebyshev ring radius for deeper
  neighbourhoods, instead of walking a precomputed offset table.
* `textbook_fcm_step` is Bezdek's fuzzy c-means in its usual normalised
  form (memberships proportional to d^(-2/(m-1))), with no stencil at all.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _coords(shape):
    nz, ny, nx = shape
    return [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]


def bruteforce_hf(x, U, V=1, h=1.0, L=3, rings="chebyshev", q2_literal=True):
    """H and F of eqs (5), (7) for every voxel by an all-pairs scan.

    rings="setbuilder": one ring, k in NB(i) iff 0 < |d|^2 < 2^(L-1) (eq (9)).
    rings="chebyshev": ring r = max(|dX|, |dY|, |dZ|) for r = 1..V.
    rings="sqdist":    ring r = |d|^2 for r = 1..V.
    """
    xs = np.asarray(x, dtype=np.float64)
    shape = xs.shape
    flat = xs.reshape(-1)
    U = np.asarray(U, dtype=np.float64).reshape(flat.size, -1)
    C = U.shape[1]
    pts = _coords(shape)
    nrings = 1 if rings == "setbuilder" else V
    # eq (10) exactly as printed
    den = sum(math.exp(-r / h) for r in range(1, nrings + 1))
    W = [0.0] + [math.exp(-r / h) / den for r in range(1, nrings + 1)]
    H = np.zeros_like(U)
    F = np.zeros_like(U)
    for i, (zi, yi, xi) in enumerate(pts):
        members = {r: [] for r in range(1, nrings + 1)}
        for k, (zk, yk, xk) in enumerate(pts):
            d2 = (xi - xk) ** 2 + (yi - yk) ** 2 + (zi - zk) ** 2  # eq (8)
            if rings == "setbuilder":
                if 0 < d2 < 2 ** (L - 1):
                    members[1].append((k, d2))
            elif rings == "chebyshev":
                r = max(abs(xi - xk), abs(yi - yk), abs(zi - zk))
                if 1 <= r <= V:
                    members[r].append((k, d2))
            else:
                if 1 <= d2 <= V:
                    members[d2].append((k, d2))
        for r in range(1, nrings + 1):
            S = members[r]
            if not S:
                continue
            g = np.array([abs(flat[i] - flat[k]) for k, _ in S])  # eq (6)
            q = np.array([float(d2) for _, d2 in S])
            w = q * q if q2_literal else q
            u = np.array([U[k] for k, _ in S])  # (|S|, C)
            if g.sum() > 0:
                H[i] += W[r] * (g[:, None] * u).sum(0) / g.sum()
            else:
                H[i] += W[r] * u.mean(0)
            F[i] += W[r] * (w[:, None] * u * u).sum(0) / w.sum()
    return H, F


def bruteforce_step(x, U, c, lam, xi, m=2.0, floor=1e-12, **kw):
    """One IFCM step assembled from `bruteforce_hf`: returns
    (U_new, c_new, J_of_input, H, F)."""
    H, F = bruteforce_hf(x, U, **kw)
    flat = np.asarray(x, np.float64).reshape(-1)
    U = np.asarray(U, np.float64).reshape(flat.size, -1)
    c = np.asarray(c, np.float64)
    a = 1.0 - lam * H - xi * F                                  # eq (4)
    d2 = np.maximum((flat[:, None] - c[None, :]) ** 2 * a, floor)
    J = float((U ** m * d2).sum())                               # eq (1)
    w = (1.0 / d2) ** (1.0 / (m - 1.0))
    Un = w / w.sum(1, keepdims=True)                             # eq (2)
    um = Un ** m
    cn = (um * flat[:, None]).sum(0) / um.sum(0)                 # eq (3)
    return Un, cn, J, H, F


def textbook_fcm_step(x, U, c, m=2.0):
    """Bezdek FCM: J(U, c), then memberships of c, then centres."""
    flat = np.asarray(x, np.float64).reshape(-1)
    U = np.asarray(U, np.float64).reshape(flat.size, -1)
    c = np.asarray(c, np.float64)
    d2 = (flat[:, None] - c[None, :]) ** 2
    J = float((U ** m * d2).sum())
    w = d2 ** (-1.0 / (m - 1.0))
    Un = w / w.sum(1, keepdims=True)
    um = Un ** m
    cn = (flat @ um) / um.sum(0)
    return Un, cn, J


def random_memberships(rng, n, C):
    a = rng.random((n, C)) + 0.05
    return a / a.sum(1, keepdims=True)


def all_flips():
    return [ax for k in range(1, 4) for ax in itertools.combinations((0, 1, 2), k)]
