"""The pins of the FP64 oracle catch plausible mistakes in it.

Each case plants one mistake in a scratch copy of oracle/pifcm_oracle.c (a
dropped or wrong term, a wrong sign, index or exponent, a reading slipped to
another), builds it, and runs tests/test_oracle_pins.py against that build
(PIFCM_ORACLE_LIB): some pin must fail.  The frozen golden fixture is not in
that run, so every mistake has to be caught by a check built from the paper
or the mathematics.  Runs on the CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pifcm_oracle.c")

MUTATIONS = [
    ("stop rule from t = 3 (R12)", "p->eps > 0.0 && t >= 2 &&", "p->eps > 0.0 && t >= 3 &&"),
    ("fitness of the previous state (R9)",
     "step_range(x, nx, ny, nz, zbeg, zend, p, lambda, xi, Ua, ca, NULL, NULL, &Jf, NULL, NULL);",
     "step_range(x, nx, ny, nz, zbeg, zend, p, lambda, xi, Ub, ca, NULL, NULL, &Jf, NULL, NULL);"),
    ("initial memberships from |x - c| instead of (x - c)^2",
     "double e = ((double)x[i] - c[j]) * ((double)x[i] - c[j]);",
     "double e = fabs((double)x[i] - c[j]);"),
    ("eq (4): + lambda H", "1.0 - lambda * H - xi * F", "1.0 + lambda * H - xi * F"),
    ("eq (4): + xi F", "1.0 - lambda * H - xi * F", "1.0 - lambda * H + xi * F"),
    ("eq (4): distance not squared", "const double e = (xv - c[j]) * (xv - c[j]) * a;",
     "const double e = fabs(xv - c[j]) * a;"),
    ("eq (3): u instead of u^m", "const double w = pow(un_new[j], m);", "const double w = un_new[j];"),
    ("eq (1): u instead of u^m", "J += pow(U[i * C + j], m) * d2[j];", "J += U[i * C + j] * d2[j];"),
    ("eq (2): exponent 2/(m-1) on squared distances", "double e = 1.0 / (m - 1.0);",
     "double e = 2.0 / (m - 1.0);"),
    ("eq (5): not divided by the sum of g", "hn[r][j] / gs[r] : un[r][j]", "hn[r][j] : un[r][j]"),
    ("eq (5): flat neighbourhood gives 0", "hn[r][j] / gs[r] : un[r][j] / (double)cnt[r]",
     "hn[r][j] / gs[r] : 0.0"),
    ("eq (6): g = x_i - x_k without the absolute value", "const double g = fabs(xv - (double)x[k]);",
     "const double g = xv - (double)x[k];"),
    ("eq (7): weight q instead of q^2", "(double)s : (double)s * (double)s", "(double)s : (double)s"),
    ("eq (7): divided by the neighbour count", "const double fr = fn[r][j] / qs[r];",
     "const double fr = fn[r][j] / (double)cnt[r];"),
    ("eq (7): u instead of u^2", "fn[r][j] += u * u * off[o].q2;", "fn[r][j] += u * off[o].q2;"),
    ("eq (9): rings by the sum of offsets instead of the largest",
     "ring = ax > ay ? ax : ay;\n          ring = ring > az ? ring : az;", "ring = ax + ay + az;"),
    ("eq (10): weights not normalised", "W[r] = exp(-(double)(r - 1) / p->h) / total;",
     "W[r] = exp(-(double)(r - 1) / p->h);"),
    ("normalisation by the maximum", "out[i] = (float)(((double)raw[i] - mn) / (mx - mn));",
     "out[i] = (float)(((double)raw[i] - mn) / mx);"),
    ("swarm: pbest term with the wrong sign", "c1 * r1[s] * (pb[2 * q + d] - pos[2 * q + d])",
     "c1 * r1[s] * (pos[2 * q + d] - pb[2 * q + d])"),
    ("swarm: gbest term with the wrong sign", "c2 * r2[s] * (gb[d] - pos[2 * q + d])",
     "c2 * r2[s] * (pos[2 * q + d] - gb[d])"),
    ("swarm: no inertia", "double v = w * vel[2 * q + d] +", "double v = vel[2 * q + d] +"),
    ("swarm: no clipping to [0, 1]", "pos[2 * q + d] = np < 0.0 ? 0.0 : (np > 1.0 ? 1.0 : np);",
     "pos[2 * q + d] = np;"),
    ("central differences: half the step", "grad[0] = (Jp - Jm) / (2.0 * step);",
     "grad[0] = (Jp - Jm) / step;"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_a_planted_mistake(tmp_path, what, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {old}"
    mutated = src.replace(old, new, 1)
    (tmp_path / "pifcm_oracle.c").write_text(mutated)
    shutil.copy(os.path.join(ROOT, "oracle", "pifcm_oracle.h"), tmp_path / "pifcm_oracle.h")
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                    str(tmp_path / "pifcm_oracle.c"), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, PIFCM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "-p", "no:xdist"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{what}: no pin failed\n{r.stdout[-2000:]}\n{r.stderr[-2000:]}"
