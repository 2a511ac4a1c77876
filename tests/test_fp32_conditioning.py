"""Why the saturated regime (lambda + xi > 1) is compared the way it is.

Where 1 - lambda H - xi F of eq (4) is near zero, the floor of the squared
distance decides the memberships, and which side of it a voxel lands on
depends on rounding.  A float32 restatement of the IFCM step in numpy (no
GPU, no oracle code: shifted-array sums over the 26 offsets of eq (9)) is
compared here with the FP64 oracle:

* one step from the same float32 state: on voxels whose factor is at least
  A_MIN away from zero for every cluster the two agree far inside the
  max-norm bar (what the GPU's one-step checks hold such voxels to); on the
  other voxels the error exceeds the bar in float32 as such, whatever the
  kernel;
* several steps: the errors of those voxels reach their neighbours through
  eqs (5) and (7), so after a few iterations the max-norm error exceeds the
  bar on regular voxels too (why multi-step comparisons in this regime are
  held to the 2-norm bar, and non-converging runs to validity).
"""
import numpy as np

from gpu_util import A_MIN, TOL, regular_voxels, rel2


def fp32_step(x, U, c, lam, xi):
    """One IFCM step of the 3x3x3 neighbourhood, every operation in float32:
    eqs (5)-(9) as sums over the 26 offsets, eq (4) with the 1e-12 floor,
    eq (2) at m = 2."""
    f = np.float32
    nz, ny, nx = x.shape
    C = U.shape[1]
    X = x.astype(f)
    U3 = U.reshape(nz, ny, nx, C).astype(f)
    Hn = np.zeros((nz, ny, nx, C), f)
    Fn = np.zeros((nz, ny, nx, C), f)
    Um = np.zeros((nz, ny, nx, C), f)
    Gs = np.zeros((nz, ny, nx), f)
    Qs = np.zeros((nz, ny, nx), f)
    cnt = np.zeros((nz, ny, nx), f)

    def rng_of(d, n):  # target indices i with i + d inside [0, n)
        return slice(max(0, -d), min(n, n - d)), slice(max(0, d), min(n, n + d))

    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dz == dy == dx == 0:
                    continue
                tz, sz = rng_of(dz, nz)
                ty, sy = rng_of(dy, ny)
                tx, sx = rng_of(dx, nx)
                tgt, src = (tz, ty, tx), (sz, sy, sx)
                g = np.abs(X[tgt] - X[src])                 # eq (6)
                u = U3[src]
                Hn[tgt] += g[..., None] * u
                Gs[tgt] += g
                q = f((dz * dz + dy * dy + dx * dx) ** 2)   # eq (8), squared in eq (7)
                Fn[tgt] += q * u * u
                Qs[tgt] += q
                Um[tgt] += u
                cnt[tgt] += f(1)
    with np.errstate(invalid="ignore", divide="ignore"):
        H = np.where(Gs[..., None] > 0, Hn / Gs[..., None],
                     np.where(cnt[..., None] > 0, Um / np.maximum(cnt, f(1))[..., None], f(0)))
        F = np.where(cnt[..., None] > 0, Fn / np.maximum(Qs, f(1e-30))[..., None], f(0))
    a = f(1) - f(lam) * H - f(xi) * F
    d2 = np.maximum((X[..., None] - c.astype(f)) ** 2 * a, f(1e-12))
    inv = f(1) / d2
    Un = inv / inv.sum(-1, keepdims=True)
    return Un.reshape(-1, C)


def _centres32(x, U):
    f = np.float32
    w = (U * U).astype(f)
    X = x.reshape(-1).astype(f)
    return (w * X[:, None]).sum(0) / w.sum(0)


def _start(orc):
    import synth
    raw, _ = synth.nested_ellipsoids(shape=(8, 32, 32), seed=1, sigma=0.05)
    x = orc.normalize(raw)
    c0, U0, _ = orc.fcm_init(x, orc.Params(C=4, m=2.0, eps=1e-5, max_iter=50))
    return x, c0, U0


def test_one_fp32_step_matches_oracle_off_the_floor(orc):
    x, c0, U0 = _start(orc)
    worst_irregular = 0.0
    for (lam, xi), t in [(pt, t) for pt in ((0.3, 0.4), (0.9, 0.7), (1.0, 1.0), (0.6, 0.6))
                         for t in (0, 5)]:
        st = orc.solve(x, c0, orc.Params(C=4, m=2.0, eps=0.0, max_iter=t), lam, xi, U0=U0)
        U32 = st["U"].astype(np.float32)
        c32 = st["c"].astype(np.float32)
        Uo, _, _, H, F = orc.step(x, U32.astype(np.float64), c32.astype(np.float64),
                                  orc.Params(C=4, m=2.0), lam, xi, want_hf=True)
        Ue = fp32_step(x, U32, c32, lam, xi)
        reg = regular_voxels(H, F, lam, xi)
        scale = np.max(np.abs(Uo))
        assert reg.sum() > 0.8 * reg.size
        e_reg = np.max(np.abs(Ue[reg] - Uo[reg])) / scale
        assert e_reg <= 0.1 * TOL, (lam, xi, e_reg)
        if lam + xi <= 1.0:
            assert reg.all() and np.max(np.abs(Ue - Uo)) / scale <= 0.1 * TOL
        if (~reg).any():
            worst_irregular = max(worst_irregular,
                                  float(np.max(np.abs(Ue[~reg] - Uo[~reg])) / scale))
    # float32 alone breaks the max-norm bar on the irregular voxels
    assert worst_irregular > TOL, worst_irregular
    assert A_MIN > 0


def test_fp32_errors_spread_over_iterations(orc):
    x, c0, U0 = _start(orc)
    worst = {}
    for lam, xi in ((0.3, 0.4), (1.0, 1.0)):
        U32, c32 = U0.astype(np.float32), c0.astype(np.float32)
        Uo, co = U0.copy(), c0.copy()
        worst[(lam, xi)] = 0.0
        for _ in range(6):
            Un, cn, _, H, F = orc.step(x, Uo, co, orc.Params(C=4, m=2.0), lam, xi, want_hf=True)
            U32 = fp32_step(x, U32, c32, lam, xi)
            c32 = _centres32(x, U32)
            Uo, co = Un, cn
            reg = regular_voxels(H, F, lam, xi)
            worst[(lam, xi)] = max(worst[(lam, xi)], float(np.max(np.abs(U32[reg] - Uo[reg]))))
    assert worst[(0.3, 0.4)] <= TOL          # off the floor the iteration stays on the bar
    assert worst[(1.0, 1.0)] > 10 * TOL      # at saturation the errors reach regular voxels
    assert rel2(U32, Uo) > 0
