"""Replays, on the CPU, the walk along z of the tiled kernels' planes.

Every tiled kernel (the fused 3x3x3 step k_ifcm_gather, the two-ring step
k_ifcm_ring2, and both adjoint kernels) gives one wavefront a column of
tiles and walks it plane by plane: a plane is prefetched into registers,
staged into one of a few LDS buffers, read for the neighbourhood sums of the
voxels above, in and below it, and a voxel is finalised (its results
stored) once its last neighbour plane has been read.  A mistake in that
schedule either reads a plane outside the volume (a GPU memory fault) or
finalises a voxel from a plane that was already overwritten (wrong results).

The functions below restate each kernel's loop structure plane by plane
(prologue, first planes, the unrolled interior, the last planes) and record
every global load and store, every LDS staging and read, and which plane each
register set holds.  The tests run them for every plane count up to 300, every
plane-per-tile depth the host or the tuner can choose, and slabs, and check:

* every load that is issued reads a plane in [0, nz), within the 32-bit
  offset range the host sizes tiles for;
* every voxel of the active planes is finalised exactly once, from its own
  tile;
* every LDS read finds the plane it expects, and every use of the prefetch
  registers finds the plane it expects;
* in the interior loops, where the kernels drop the per-plane tests, every
  one of those tests holds.

A replay of the discarded variant of the fused step (interior prefetches
without the plane-range test) must be caught, which shows the check has teeth.
"""
import pytest

ZC_CHOICES = (1, 2, 3, 4, 5, 7, 8, 16, 32, 64, 128)


class Walk:
    def __init__(self, nz, zlo, zhi, nbuf):
        self.nz, self.zlo, self.zhi = nz, zlo, zhi
        self.buf = [None] * nbuf
        self.reg = None            # plane held by the prefetch registers
        self.loads = []            # (plane, issued)
        self.stores = []           # planes finalised

    def load(self, q, range_test=True):
        pv = 0 <= q < self.nz
        self.loads.append((q, pv if range_test else True))
        self.reg = q

    def stage(self, b, q):
        assert self.reg == q, f"staging plane {q} from registers holding {self.reg}"
        self.buf[b] = q

    def read(self, b, q):
        assert self.buf[b] == q, f"LDS buffer {b} holds plane {self.buf[b]}, read as {q}"

    def finalize(self, z):
        self.stores.append(z)


def gather_walk(nz, zlo, zhi, interior_range_test=True, interior_margin=4):
    """k_ifcm_gather: three LDS buffers, plane q in buffer (q - zlo + 1) % 3."""
    w = Walk(nz, zlo, zhi, 3)
    bufof = lambda q: (q - zlo + 1) % 3  # noqa: E731

    def plane(p, gen, bp_const=None):
        if not gen:
            # the interior body assumes every per-plane test is true
            assert 0 <= p < nz and p - 1 >= zlo and zlo <= p < zhi and p + 1 < zhi
            assert p + 1 <= zhi and p + 2 <= zhi
            assert bufof(p) == bp_const
        pv = (not gen) or (0 <= p < nz)
        doA = (not gen) or p - 1 >= zlo
        doB = (not gen) or (zlo <= p < zhi)
        doC = (not gen) or p + 1 < zhi
        if pv:
            w.read(bufof(p), p)
            if doA:
                w.read(bufof(p - 1), p - 1)  # voxel p-1's own cell, finalised below
        if doC:
            assert w.reg == p + 1, "voxel p+1's centre value from the prefetch registers"
        if (not gen) or p + 1 <= zhi:
            w.stage(bufof(p + 1), p + 1)
            if (not gen) or p + 2 <= zhi:
                w.load(p + 2, range_test=gen or interior_range_test)
        if doA:
            w.read(bufof(p - 1), p - 1)
            w.finalize(p - 1)
        del doB

    w.load(zlo - 1)
    w.stage(0, zlo - 1)
    w.load(zlo)
    p = zlo - 1
    while p <= zlo and p <= zhi:
        plane(p, True)
        p += 1
    while p + interior_margin <= zhi:
        plane(p, False, 2)
        plane(p + 1, False, 0)
        plane(p + 2, False, 1)
        p += 3
    while p <= zhi:
        plane(p, True)
        p += 1
    return w


def adjoint_walk(nz, zlo, zhi):
    """k_adj_point and k_adj_transpose_tiled: the same three-buffer walk with
    the interior chosen per group inside one loop."""
    w = Walk(nz, zlo, zhi, 3)
    bufof = lambda q: (q - zlo + 1) % 3  # noqa: E731

    def plane(p):
        pv = 0 <= p < nz
        doA = p - 1 >= zlo
        if pv:
            w.read(bufof(p), p)
        if p + 1 < zhi:
            assert w.reg == p + 1
        if p + 1 <= zhi:
            w.stage(bufof(p + 1), p + 1)
            if p + 2 <= zhi:
                w.load(p + 2)
        if doA:
            w.read(bufof(p - 1), p - 1)
            w.finalize(p - 1)

    w.load(zlo - 1)
    w.stage(0, zlo - 1)
    w.load(zlo)
    p = zlo - 1
    while p <= zhi:
        if p > zlo and p + 4 <= zhi:
            plane(p)
            plane(p + 1)
            plane(p + 2)
            p += 3
        else:
            plane(p)
            p += 1
    return w


def ring2_walk(nz, zlo, zhi):
    """k_ifcm_ring2: four LDS buffers, plane q in buffer (q - zlo + 2) & 3;
    cells of plane p feed voxels p-2 .. p+2; the own values (intensity and
    ring invariants) of voxel q are prefetched separately, two planes before
    the voxel's slot opens."""
    w = Walk(nz, zlo, zhi, 4)
    own = {"q": None}
    own_loads = []
    bufof = lambda q: (q - zlo + 2) & 3  # noqa: E731

    def load_own(q):
        own_loads.append((q, 0 <= q < nz))
        own["q"] = q

    def plane(p, gen):
        if not gen:
            assert 0 <= p < nz and zlo <= p - 2 < zhi
            assert p + 1 <= zhi + 1 and p + 2 <= zhi + 1 and p + 3 <= zhi + 1
        if p + 2 < zhi:  # a slot past the tile is never finalised
            assert own["q"] == p + 2, "the slot of voxel p+2 opens from its prefetched own values"
        pv = (not gen) or (0 <= p < nz)
        if pv:
            w.read(bufof(p), p)
        if (not gen) or p + 1 <= zhi + 1:
            w.stage(bufof(p + 1), p + 1)
            if (not gen) or p + 2 <= zhi + 1:
                w.load(p + 2)
        if (not gen) or p + 3 <= zhi + 1:
            load_own(p + 3)
        if (not gen) or (zlo <= p - 2 < zhi):
            w.read(bufof(p - 2), p - 2)
            w.finalize(p - 2)

    w.load(zlo - 2)
    w.stage(bufof(zlo - 2), zlo - 2)
    w.load(zlo - 1)
    load_own(zlo)
    p = zlo - 2
    while p < zlo + 2:
        plane(p, True)
        p += 1
    while p + 4 <= zhi:
        plane(p, False)
        p += 1
    while p <= zhi + 1:
        plane(p, True)
        p += 1
    w.loads += own_loads
    return w


def tiles(zbeg, zend, zc):
    zc = max(1, min(zc, zend - zbeg))
    ntz = (zend - zbeg + zc - 1) // zc
    for t in range(ntz):
        zlo = zbeg + t * zc
        yield zlo, min(zlo + zc, zend), zc


def slabs(nz):
    out = {(0, nz)}
    for z in {0, nz // 2, nz - 1}:
        out.add((z, z + 1))
    if nz > 2:
        out.add((1, nz - 1))
    return sorted(out)


NZ_CHUNKS = [range(a, a + 50) for a in range(1, 301, 50)]


def check(walk_fn, nz, zbeg, zend, zc, offset_planes=None):
    done = []
    for zlo, zhi, zc_eff in tiles(zbeg, zend, zc):
        w = walk_fn(nz, zlo, zhi)
        zb = max(zlo - 1, 0)
        for q, issued in w.loads:
            if issued:
                assert 0 <= q < nz, (nz, zlo, zhi, q)
                if offset_planes is not None:
                    # 32-bit byte offsets from the tile's first staged plane
                    assert 0 <= q - zb <= zc_eff + offset_planes, (zlo, zhi, q)
        assert sorted(w.stores) == list(range(zlo, zhi)), (nz, zlo, zhi, w.stores)
        done += w.stores
    assert sorted(done) == list(range(zbeg, zend))


@pytest.mark.parametrize("nzs", NZ_CHUNKS, ids=lambda r: f"nz{r.start}-{r.stop - 1}")
def test_fused_step_walk(nzs):
    for nz in nzs:
        for zc in ZC_CHOICES + (nz,):
            for zbeg, zend in slabs(nz):
                check(gather_walk, nz, zbeg, zend, zc, offset_planes=1)


def test_fused_step_walk_every_depth():
    """The default depth of a volume is some ceil(nz / k) (and
    pifcm_set_decomposition takes any depth): every depth of a spread of
    plane counts."""
    for nz in list(range(1, 40)) + list(range(40, 320, 13)):
        for zc in range(1, nz + 1):
            check(gather_walk, nz, 0, nz, zc, offset_planes=1)


@pytest.mark.parametrize("nzs", NZ_CHUNKS, ids=lambda r: f"nz{r.start}-{r.stop - 1}")
def test_two_ring_walk(nzs):
    for nz in nzs:
        for zc in ZC_CHOICES + (nz,):
            for zbeg, zend in slabs(nz):
                check(ring2_walk, nz, zbeg, zend, zc)


@pytest.mark.parametrize("nzs", NZ_CHUNKS, ids=lambda r: f"nz{r.start}-{r.stop - 1}")
def test_adjoint_walk(nzs):
    """The adjoint kernels' depth is some ceil(nz / k) of at least
    min(nz, 32) planes, picked per launch from the kernel's occupancy."""
    for nz in nzs:
        depths = {(nz + k - 1) // k for k in range(1, nz + 1)}
        for zc in sorted(d for d in depths if d >= min(nz, 32)) + [64]:
            check(adjoint_walk, nz, 0, nz, zc)


def test_discarded_prefetch_variant_is_caught():
    """Interior prefetches without the plane-range test read plane p + 4 ==
    nz when a tile ends at the volume's last plane; with the interior loop
    held to p + 5 <= zhi that read never happens."""
    caught = 0
    for nz in range(1, 80):
        for zc in ZC_CHOICES:
            for zlo, zhi, _ in tiles(0, nz, zc):
                w = gather_walk(nz, zlo, zhi, interior_range_test=False)
                bad = [q for q, issued in w.loads if issued and not 0 <= q < nz]
                caught += bool(bad)
                if bad:
                    assert bad == [nz] and zhi == nz
                w = gather_walk(nz, zlo, zhi, interior_range_test=False, interior_margin=5)
                assert all(0 <= q < nz for q, issued in w.loads if issued)
    assert caught > 0
