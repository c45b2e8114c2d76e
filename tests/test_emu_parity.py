"""The library's traversal core (traverse.h) compiled for the CPU against the
oracle.  Same code as the HIP kernels, so indexing, termination, exactness
and accuracy are checked here before any GPU run; the GPU parity tests repeat
the comparison through the HIP library."""
import numpy as np
import pytest

import amrgen
import oracle
import paper_1210_8014_amd as amr
from tests import emu
from tests import parity
from tests.test_oracle_pins import degenerate_cams, rand_cams


class EmuRenderer:
    """Renders with all four descent modes (restart at the base level, at the
    common ancestor from a stack, register-cached, register-cached with an
    ancestor stack) and insists they are bit-identical."""

    def __init__(self, leaves, restrict=None):
        self.T = amr.Tree(leaves, restrict=restrict, host_only=True)
        self.E = emu.EmuTree(self.T)

    def camera(self, d):
        return amr.set_camera(d, self.T)

    def render(self, cam, op, field=0, weight=0, los=False, rays=None):
        a = self.E.render(cam, op, field, weight, los, rays, lca=2)
        for mode in (0, 1, 3):
            b = self.E.render(cam, op, field, weight, los, rays, lca=mode)
            for x, y in zip(a, b):
                assert np.array_equal(x.view(np.int32), y.view(np.int32)), f"descent mode {mode} differs"
        return a

    def trace(self, cam, rays):
        return self.E.trace(cam, rays)


@pytest.mark.parametrize("seed", range(4))
def test_random_trees_all_cameras(seed):
    rng = np.random.default_rng(seed)
    L = amrgen.random_tree(200 + seed, lmax=5, p_refine=0.45, nfields=4)
    L.fields[1:] -= 5.0
    R = EmuRenderer(L)
    OT = oracle.Tree(L)
    cams = rand_cams(rng, 8, W=9, H=7, inside=(seed % 2 == 1)) + degenerate_cams()
    for camd in cams:
        for ml in (OT.lmax, 2):
            d = dict(camd, max_level=ml)
            n = d["W"] * d["H"]
            parity.compare_all(R, OT, d, ops=("sum", "max", "wmean"), los_fields=(1, 0, True),
                               trace_rays=np.arange(n), what=f"seed{seed} {d['kind']} ml{ml}")


def test_tiny_scene_full_image():
    L = amrgen.scene("tiny")
    R = EmuRenderer(L)
    OT = oracle.Tree(L)
    res = parity.compare_all(R, OT, amrgen.tiny_camera(), ops=("sum", "max"),
                             trace_rays=np.arange(0, 65536, 7), what="tiny")
    assert res["sum"] < 5e-7


def test_tiny_scene_every_truncation_level():
    L = amrgen.scene("tiny")
    R = EmuRenderer(L)
    OT = oracle.Tree(L)
    for ml in range(0, 7):
        parity.compare_all(R, OT, amrgen.tiny_camera(64, 64, max_level=ml), ops=("sum", "max"),
                           trace_rays=np.arange(64 * 64), what=f"tiny L{ml}")


def test_small_disk_perspective_wmean():
    """Disk recipe at reduced depth (levels 7..11) with the three inclinations."""
    L = amrgen.disk(seed=3, lmax=11, m_thr=2e-4)
    assert 300_000 < L.n < 3_000_000
    R = EmuRenderer(L)
    OT = oracle.Tree(L)
    rays = np.random.default_rng(0).choice(128 * 128, 3000, replace=False)
    for cam in amrgen.disk_cameras(128, 128, max_level=11):
        parity.compare_all(R, OT, cam, ops=("sum", "max", "wmean"), rays=rays, los_fields=(1, 0, True),
                           trace_rays=rays[:300], what="disk")


def test_deep_levels_fp64_boundaries():
    """Cores refine to level 20; a camera inside the disk looks at core 0 with
    the automatic maximum level, so cells at levels >= 18 are crossed."""
    m_thr = 3e-3
    L = amrgen.generate(amrgen.DISK, 0, 7, 20, m_thr, True, False)
    assert L.lmax == 20
    R = EmuRenderer(L)
    OT = oracle.Tree(L)
    tgt = amrgen.core_position(0, 20, m_thr, 0)
    s = 2.0 ** -13
    cam = amrgen.camera("persp", (tgt[0], tgt[1] - 0.8 * s, tgt[2] + 0.6 * s), tgt, (0, 0.6, 0.8), 96, 96,
                        fov_y=0.9, max_level=-1)
    c = R.camera(cam)
    assert c.max_level >= 18
    rays = np.arange(96 * 96)
    offs, cells = R.trace(c, rays[::5])
    assert cells[:, 0].max() >= 18
    parity.compare_all(R, OT, cam, ops=("sum", "max"), trace_rays=rays[::5], what="deep")


class SplitRenderer(EmuRenderer):
    """The split-ray path (each ray cut into K spans at base-level planes,
    spans merged in order): cells concatenated over the spans must equal the
    oracle's cell sequence exactly, the maximum must be bit-identical to the
    unsplit walk, sums agree within the parity bars."""

    def __init__(self, leaves, K, restrict=None):
        super().__init__(leaves, restrict)
        self.K = K

    def render(self, cam, op, field=0, weight=0, los=False, rays=None):
        out, aux, cnt, _ = self.E.render_split(cam, op, self.K, field, weight, los, rays)
        plain = self.E.render(cam, op, field, weight, los, rays, lca=2)
        assert np.array_equal(cnt, plain[2]), "split changes the cell count"
        if op == oracle.MAX:
            assert np.array_equal(out.view(np.int32), plain[0].view(np.int32)), "split changes the maximum"
        return out, aux, cnt

    def trace(self, cam, rays):
        _, _, _, (offs, cells) = self.E.render_split(cam, oracle.MAX, self.K, rays=rays, with_cells=True)
        return offs, cells


@pytest.mark.parametrize("seed", range(4))
def test_split_rays_random_trees(seed):
    rng = np.random.default_rng(50 + seed)
    L = amrgen.random_tree(300 + seed, lmax=6, p_refine=0.4, nfields=4)
    L.fields[1:] -= 5.0
    OT = oracle.Tree(L)
    cams = rand_cams(rng, 6, W=9, H=7, inside=(seed % 2 == 1)) + degenerate_cams()
    for K in (2, 3, 4, 7):
        R = SplitRenderer(L, K)
        for camd in cams:
            for ml in (OT.lmax, 3, 1):
                d = dict(camd, max_level=ml)
                n = d["W"] * d["H"]
                parity.compare_all(R, OT, d, ops=("sum", "max", "wmean"), los_fields=(1, 0, True),
                                   trace_rays=np.arange(n), what=f"split{K} seed{seed} {d['kind']} ml{ml}")


def test_split_rays_disk_and_deep_levels():
    L = amrgen.disk(seed=3, lmax=11, m_thr=2e-4)
    OT = oracle.Tree(L)
    rays = np.random.default_rng(1).choice(128 * 128, 2000, replace=False)
    for K in (2, 4):
        R = SplitRenderer(L, K)
        for cam in amrgen.disk_cameras(128, 128, max_level=11):
            parity.compare_all(R, OT, cam, ops=("sum", "max", "wmean"), rays=rays, los_fields=(1, 0, True),
                               trace_rays=rays[:300], what=f"split{K} disk")
    m_thr = 3e-3
    L = amrgen.generate(amrgen.DISK, 0, 7, 20, m_thr, True, False)
    OT = oracle.Tree(L)
    tgt = amrgen.core_position(0, 20, m_thr, 0)
    s = 2.0 ** -13
    cam = amrgen.camera("persp", (tgt[0], tgt[1] - 0.8 * s, tgt[2] + 0.6 * s), tgt, (0, 0.6, 0.8), 48, 48,
                        fov_y=0.9, max_level=-1)
    R = SplitRenderer(L, 4)
    parity.compare_all(R, OT, cam, ops=("sum", "max"), trace_rays=np.arange(48 * 48)[::3], what="split deep")


def test_whole_box_end_test_matches_per_axis_end_test():
    """The fast walk ends a ray either by one comparison against the box
    (rays that stop at the box: render_pixel) or by the per-axis stop planes
    (spans: here one span per ray).  The two must give the same cells and
    bit-identical results, degenerate rays included."""
    rng = np.random.default_rng(77)
    for seed in (21, 22):
        L = amrgen.random_tree(seed, lmax=6, p_refine=0.45, nfields=4)
        L.fields[1:] -= 5.0
        T = amr.Tree(L, host_only=True)
        E = emu.EmuTree(T)
        for camd in rand_cams(rng, 4, W=33, H=29, inside=(seed % 2 == 1)) + degenerate_cams():
            cam = amr.set_camera(camd, T)
            for op, kw in ((0, {}), (1, {}), (2, dict(field=1, weight=0, los=True))):
                a, ax, ca = E.render(cam, op, lca=2, **kw)
                b, bx, cb, _ = E.render_split(cam, op, 1, **kw)
                assert np.array_equal(a.view(np.int32), b.view(np.int32)), (seed, camd, op)
                assert np.array_equal(ax.view(np.int32), bx.view(np.int32)), (seed, camd, op)
                assert np.array_equal(ca, cb), (seed, camd, op)
    # a disk refined to level 11: long rays, deep descents, sibling moves
    L = amrgen.disk(seed=3, lmax=11, m_thr=2e-4)
    T = amr.Tree(L, host_only=True)
    E = emu.EmuTree(T)
    rays = np.random.default_rng(5).choice(96 * 96, 1500, replace=False)
    for camd in amrgen.disk_cameras(96, 96, max_level=11):
        cam = amr.set_camera(camd, T)
        a, _, ca = E.render(cam, 0, lca=2, rays=rays)
        b, _, cb, _ = E.render_split(cam, 0, 1, rays=rays)
        assert ca.sum() > 10 * len(rays)
        assert np.array_equal(a.view(np.int32), b.view(np.int32)) and np.array_equal(ca, cb)


def _cells_per_ray(offs, cells):
    return [cells[offs[r]:offs[r + 1]].tobytes() for r in range(len(offs) - 1)]


def test_lod_cut_flag_is_exactly_the_rays_that_differ_from_full_depth():
    """The learned-LOD tile walk records whether a ray cut a cell (stopped
    descending at a cell that has children).  A ray that cut none must give
    the full-depth result bit for bit (the LOD render then copies it instead
    of walking the ray again for its audit); a ray that cut one must have a
    cell sequence different from the full-depth one."""
    rng = np.random.default_rng(91)
    seen = [0, 0]
    cases = []
    for seed in (31, 32, 33):
        L = amrgen.random_tree(seed, lmax=6, p_refine=0.45, nfields=4)
        L.fields[1:] -= 5.0
        cases.append((L, rand_cams(rng, 3, W=21, H=17, inside=(seed % 2 == 0)) + degenerate_cams()))
    cases.append((amrgen.disk(seed=3, lmax=11, m_thr=2e-4), amrgen.disk_cameras(40, 40, max_level=11)))
    for L, cams in cases:
        T = amr.Tree(L, host_only=True)
        E = emu.EmuTree(T)
        lmax = int(T.info.lmax)
        for camd in cams:
            cam = amr.set_camera(dict(camd, max_level=lmax), T)
            rays = np.arange(cam.W * cam.H)
            ref_cells = _cells_per_ray(*E.trace(cam, rays))
            for op, kw in ((0, {}), (1, {}), (2, dict(field=1, weight=0, los=True))):
                if op == 2 and T.info.nfields < 4:
                    continue
                full, full_aux, _, _ = E.render_split(cam, op, 2, **kw)
                for lv in range(0, lmax):
                    out, aux, cut = E.render_cut(cam, op, lv, **kw)
                    keep = ~cut
                    assert np.array_equal(out[keep].view(np.int32), full[keep].view(np.int32)), (lv, op)
                    assert np.array_equal(aux[keep].view(np.int32), full_aux[keep].view(np.int32)), (lv, op)
                    if op == 0:
                        cl = amr.set_camera(dict(camd, max_level=lv), T)
                        cells = _cells_per_ray(*E.trace(cl, rays))
                        differs = np.array([a != b for a, b in zip(cells, ref_cells)])
                        assert np.array_equal(cut, differs), (lv, np.flatnonzero(cut != differs)[:5])
                        seen[0] += int(cut.sum())
                        seen[1] += int(keep.sum())
    assert seen[0] > 1000 and seen[1] > 1000  # both kinds of ray occur


def test_exact_quotient_of_the_ray_setup():
    """The set-up's floor(num / d) (an fp64 estimate corrected once) against
    integer division, over its whole domain 0 <= num < 2^28 d, 0 < d < 2^31:
    random operands, exact multiples and their neighbours, the extremes."""
    rng = np.random.default_rng(17)
    d = np.concatenate([rng.integers(1, 2 ** 31, 200_000), rng.integers(1, 64, 20_000),
                        [1, 2, 3, 2 ** 31 - 1, 2 ** 30, 2 ** 31 - 2]]).astype(np.int64)
    q = rng.integers(0, 2 ** 28, len(d))
    q[-6:] = [0, 2 ** 28 - 1, 1, 2 ** 28 - 1, 2 ** 27, 12345]
    cases = []
    for off in (-1, 0, 1):  # just below, at and just above an exact multiple
        cases.append((q * d + off, d))
    cases.append((q * d + (rng.random(len(d)) * d).astype(np.int64), d))
    cases.append((d * (2 ** 28) - 1, d))  # the largest numerator
    for num, dd in cases:
        ok = (num >= 0) & (num < dd * 2 ** 28)
        num, dd = num[ok], dd[ok]
        got = emu.div_q28(num, dd.astype(np.int32))
        assert np.array_equal(got.astype(np.int64), num // dd)
