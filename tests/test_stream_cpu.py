"""Trees larger than the GPU, on the CPU: the stream plan's partition of a
host_only tree (checked cell by cell against the tree it came from) and the
streamed walk of the traversal core over the plan's chunk arrays (checked
against the oracle: every value, maximum and cell sequence, degenerate
rays and eyes inside chunks included).  The GPU tests repeat the comparison
through amr_render_streamed."""
import numpy as np
import pytest

import amrgen
import oracle
import paper_1210_8014_amd as amr
from tests import emu
from tests import parity
from tests.test_oracle_pins import degenerate_cams, rand_cams


def _morton(code):
    x = y = z = 0
    for b in range(10):
        x |= ((code >> (3 * b)) & 1) << b
        y |= ((code >> (3 * b + 1)) & 1) << b
        z |= ((code >> (3 * b + 2)) & 1) << b
    return x, y, z


def _code(x, y, z, level):
    c = 0
    for b in range(level):
        c |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return c


def _check_plan(T, P):
    child, vals, _ = T.host_arrays()
    off = list(T.info.level_offset)
    base = min(int(T.info.levelmin), 10)
    nf = int(T.info.nfields)
    I = P.info
    assert I.nchunks == P.nchunks >= 1
    # the cubes tile the box, in Morton order, each at a level <= base
    L = max(P.chunk(i)["level"] for i in range(P.nchunks))
    pos = 0
    ancestors = set()
    total = 0
    for i in range(P.nchunks):
        c = P.chunk(i)
        lc = c["level"]
        assert 0 <= lc <= base
        code = _code(c["ix"], c["iy"], c["iz"], lc)
        assert code << (3 * (L - lc)) == pos, "cubes out of Morton order or overlapping"
        pos += 1 << (3 * (L - lc))
        for a in range(lc):
            ancestors.add((a, code >> (3 * (lc - a))))
        total += c["ncells"]
        assert c["ncells"] <= I.max_chunk_cells
        # walk the chunk and the tree side by side from the cube's cell
        rec, cv = c["records"], c["values"]
        lchild = rec[:, 0]
        assert np.array_equal(rec[:, 1].view(np.float32), cv[0])
        seen = np.zeros(c["ncells"], bool)
        stack = [(off[lc] + code, 0, lc)]
        while stack:
            g, loc, l = stack.pop()
            assert c["level_start"][l] <= loc < c["level_start"][l + 1], "cell outside its level's range"
            assert not seen[loc]
            seen[loc] = True
            for f in range(nf):
                assert cv[f, loc].view(np.int32) == vals[f, g].view(np.int32)
            if c["packed"] is not None:
                assert np.array_equal(c["packed"][loc], vals[:4, g])
            if l <= base:
                assert c["off_local"][l] + (g - off[l]) == loc, "local offset of a complete level"
            if child[g] < 0:
                assert lchild[loc] == -1
            else:
                assert lchild[loc] >= 0
                for o in range(8):
                    stack.append((child[g] + o, lchild[loc] + o, l + 1))
        assert seen.all(), "chunk holds cells outside the cube's subtree"
    assert pos == 1 << (3 * L), "the cubes do not cover the box"
    assert total == I.cells and total + len(ancestors) == T.ncells


@pytest.mark.parametrize("cap", [10 ** 9, 5000, 1200])
def test_plan_partitions_the_tree_tiny(cap):
    T = amr.Tree(amrgen.scene("tiny"), host_only=True)
    P = amr.StreamPlan(T, cap, host_only=True)
    _check_plan(T, P)
    if cap == 10 ** 9:
        assert P.nchunks == 1 and P.info.max_chunk_level == 0


@pytest.mark.parametrize("seed", range(3))
def test_plan_partitions_random_trees(seed):
    L = amrgen.random_tree(400 + seed, lmax=6, p_refine=0.45, levelmin=3, nfields=4)
    T = amr.Tree(L, host_only=True)
    for cap in (T.ncells // 3, T.ncells // 20, 300):
        try:
            P = amr.StreamPlan(T, cap, host_only=True)
        except amr.AmrError as e:
            assert e.status == 5 and cap == 300  # a base-level subtree above the cap
            continue
        _check_plan(T, P)


def test_plan_rejects():
    L = amrgen.random_tree(3, lmax=5, p_refine=0.45, levelmin=2)
    Td = amr.Tree(L, host_only=True)
    with pytest.raises(amr.AmrError) as e:
        amr.StreamPlan(Td, 0, host_only=True)
    assert e.value.status == 1
    with pytest.raises(amr.AmrError) as e:
        amr.StreamPlan(Td, 8, host_only=True)  # 73+ cells under one level-2 cell
    assert e.value.status == 5
    P = amr.StreamPlan(Td, Td.ncells, host_only=True)
    cam = amr.set_camera(amrgen.tiny_camera(16, 16, 5))
    import torch

    out = torch.zeros(256)
    ws = torch.zeros(256 * 4)
    with pytest.raises(amr.AmrError) as e:
        P.render(cam, amr.SUM, out, ws, stream=0)  # a host_only plan cannot render
    assert e.value.status == 1


class ChunkedRenderer:
    """Streamed walk over a plan's chunks (tests/emu.EmuStream), checked
    against the whole-ray walk: identical cell counts and maximum."""

    def __init__(self, leaves, cap, restrict=None):
        self.T = amr.Tree(leaves, restrict=restrict, host_only=True)
        self.P = amr.StreamPlan(self.T, cap, host_only=True)
        self.S = emu.EmuStream(self.P, self.T)
        self.E = emu.EmuTree(self.T)

    @property
    def chunk_level(self):
        return int(self.P.info.max_chunk_level)

    def camera(self, d):
        return amr.set_camera(d, self.T)

    def render(self, cam, op, field=0, weight=0, los=False, rays=None):
        out, aux, cnt = self.S.render(cam, op, field, weight, los, rays)
        plain = self.E.render(cam, op, field, weight, los, rays, lca=2)
        assert np.array_equal(cnt, plain[2]), "chunks change the cell count"
        if op == oracle.MAX:
            assert np.array_equal(out.view(np.int32), plain[0].view(np.int32)), "chunks change the maximum"
        return out, aux, cnt

    def trace(self, cam, rays):
        return self.S.trace(cam, rays)


@pytest.mark.parametrize("seed", range(3))
def test_streamed_walk_random_trees(seed):
    rng = np.random.default_rng(60 + seed)
    L = amrgen.random_tree(500 + seed, lmax=6, p_refine=0.42, levelmin=3, nfields=4)
    L.fields[1:] -= 5.0
    OT = oracle.Tree(L)
    # few large chunks against degenerate rays; many small ones (levels up to
    # the base) against random cameras
    for frac, cams in ((8, degenerate_cams()), (40, rand_cams(rng, 4, W=11, H=9, inside=(seed % 2 == 1)))):
        R = ChunkedRenderer(L, max(len(L.level) // frac, 400))
        assert R.P.nchunks > 1
        for camd in cams:
            for ml in sorted({OT.lmax, R.chunk_level}):
                if ml < R.chunk_level:
                    continue
                d = dict(camd, max_level=ml)
                n = d["W"] * d["H"]
                parity.compare_all(R, OT, d, ops=("sum", "max", "wmean"), los_fields=(1, 0, True),
                                   trace_rays=np.arange(n), what=f"stream/{frac} seed{seed} {d['kind']} ml{ml}")


def test_streamed_walk_tiny_scene_and_eye_inside_chunks():
    L = amrgen.scene("tiny")
    OT = oracle.Tree(L)
    R = ChunkedRenderer(L, 1500)
    assert R.P.info.max_chunk_level >= 2
    parity.compare_all(R, OT, amrgen.tiny_camera(64, 64, 6), ops=("sum", "max"), trace_rays=np.arange(64 * 64)[::7],
                       what="stream tiny ortho")
    # perspective eyes inside the box: the eye's own chunk is met from inside,
    # the rectangles of the chunks around it span the whole image
    rng = np.random.default_rng(9)
    for _ in range(4):
        eye = rng.uniform(0.2, 0.8, 3)
        tgt = rng.uniform(0.0, 1.0, 3)
        d = amrgen.camera("persp", eye, tgt, rng.normal(size=3), 40, 30, fov_y=1.2, max_level=6)
        parity.compare_all(R, OT, d, ops=("sum", "max"), trace_rays=np.arange(40 * 30)[::3], what="stream inside")


def test_streamed_walk_disk_deep_levels():
    """A disk refined to level 11 with chunks at levels up to 4 (long rays
    crossing many cubes), and cores to level 20 (fp64 chords inside chunks)."""
    L = amrgen.disk(seed=3, lmax=11, m_thr=2e-4)
    OT = oracle.Tree(L)
    R = ChunkedRenderer(L, len(L.level) // 50)
    assert R.P.nchunks >= 30
    rays = np.random.default_rng(1).choice(96 * 96, 800, replace=False)
    for cam in amrgen.disk_cameras(96, 96, max_level=11):
        parity.compare_all(R, OT, cam, ops=("sum", "max", "wmean"), rays=rays, los_fields=(1, 0, True),
                           trace_rays=rays[:200], what="stream disk")
    m_thr = 3e-3
    L = amrgen.generate(amrgen.DISK, 0, 7, 20, m_thr, True, False)
    OT = oracle.Tree(L)
    R = ChunkedRenderer(L, len(L.level) // 15)
    tgt = amrgen.core_position(0, 20, m_thr, 0)
    s = 2.0 ** -13
    cam = amrgen.camera("persp", (tgt[0], tgt[1] - 0.8 * s, tgt[2] + 0.6 * s), tgt, (0, 0.6, 0.8), 40, 40,
                        fov_y=0.9, max_level=-1)
    parity.compare_all(R, OT, cam, ops=("sum", "max"), trace_rays=np.arange(40 * 40)[::3], what="stream deep")
