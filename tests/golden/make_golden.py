"""Write the oracle's regression fixtures into tests/golden/.

Calls only the FP64 oracle (and the shared seeded input generators).  The
fixtures freeze the oracle's outputs on the 32x32x8 nested-ellipsoid phantom
(the CPU-sized workload): the FCM initial state of Algorithm 1 step 2 and
IFCM solves at a few (lambda, xi) particles.  A later change of the oracle's
arithmetic that moves these numbers must regenerate them and say in its
commit which passage of the paper justifies the change.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402

PARTICLES = [(0.0, 0.0), (0.25, 0.5), (0.6, 0.3), (0.9, 0.8)]


def compute():
    raw, _ = synth.nested_ellipsoids(shape=(8, 32, 32), seed=1, sigma=0.05)
    x = oracle.normalize(raw)
    p = oracle.Params(C=4, m=2.0, V=1, h=1.0, eps=1e-5, max_iter=50)
    c0, U0, it0 = oracle.fcm_init(x, p)
    out = dict(workload="nested-32x32x8", seed=1, sigma=0.05, C=4, m=2.0, eps=1e-5,
               max_iter=50, x_sum=float(np.sum(x, dtype=np.float64)),
               fcm_init=dict(centres=c0.tolist(), iters=it0,
                             U_col_sums=U0.sum(0).tolist()),
               solves=[])
    for lam, xi in PARTICLES:
        o = oracle.solve(x, c0, p, lam, xi, U0=U0)
        lab = oracle.labels(o["U"], 4)
        out["solves"].append(dict(lam=lam, xi=xi, centres=o["c"].tolist(), J=o["J"],
                                  iters=o["iters"], U_col_sums=o["U"].sum(0).tolist(),
                                  label_counts=np.bincount(lab, minlength=4).tolist()))
    return out


if __name__ == "__main__":
    data = compute()
    path = os.path.join(HERE, "nested32_oracle.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", path)
