"""CPU build of the product's traversal core (tests only; see emu.cpp)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu.cpp")
HDR = os.path.join(HERE, "..", "..", "paper_1210_8014_amd", "csrc", "traverse.h")
LIB = os.path.join(HERE, "libamremu.so")
_lib = None


def build():
    if (not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(HDR))):
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
                               "-fsanitize=undefined", "-DAMR_BOUNDS_CHECK", SRC, "-o", LIB + ".tmp"])
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _cam_args(cam):
    k4 = np.array([cam.kind, cam.W, cam.H, cam.max_level], np.int32)
    ofuv = np.array(list(cam.O) + list(cam.F) + list(cam.U) + list(cam.V), np.int64)
    return k4, ofuv


def div_q28(num, d):
    """floor(num / d) by the traversal core's helper (0 <= num < 2^28 d)."""
    num = np.ascontiguousarray(num, np.int64)
    d = np.ascontiguousarray(d, np.int32)
    q = np.zeros(len(num), np.int32)
    _load().emu_div_q28(_p(num), _p(d), _p(q), ctypes.c_int64(len(num)))
    return q


class EmuTree:
    """Host arrays of a host_only library tree plus its layout constants."""

    def __init__(self, tree):
        self.child, self.vals, self.md = tree.host_arrays()
        self.vals = np.ascontiguousarray(self.vals)
        info = tree.info
        self.ncells = int(info.ncells)
        self.nfields = int(info.nfields)
        self.base = min(int(info.levelmin), 10)
        self.lmax = int(info.lmax)
        self.off = np.array(list(info.level_offset), np.int32)

    def _tree_args(self):
        return (_p(self.child), _p(self.vals), ctypes.c_int64(self.ncells), ctypes.c_int32(self.nfields),
                ctypes.c_int32(self.base), ctypes.c_int32(self.lmax), _p(self.off))

    def render(self, cam, op, field=0, weight=0, los=False, rays=None, max_level=None, lca=2):
        n = cam.W * cam.H if rays is None else len(rays)
        pix = np.arange(n, dtype=np.int64) if rays is None else np.ascontiguousarray(rays, np.int64)
        out = np.zeros(n, np.float32)
        aux = np.zeros(n, np.float32)
        cnt = np.zeros(n, np.int32)
        k4, ofuv = _cam_args(cam)
        ml = cam.max_level if max_level is None else max_level
        _load().emu_render(*self._tree_args(), _p(k4), _p(ofuv), ctypes.c_int32(op), ctypes.c_int32(field),
                           ctypes.c_int32(weight), ctypes.c_int32(int(los)), ctypes.c_int32(ml), _p(pix),
                           ctypes.c_int64(n), _p(out), _p(aux), _p(cnt), ctypes.c_int32(int(lca)))
        return out, aux, cnt

    def trace(self, cam, rays):
        rays = np.ascontiguousarray(rays, np.int64)
        _, _, cnt = self.render(cam, 1, rays=rays)
        offs = np.zeros(len(rays) + 1, np.int64)
        offs[1:] = np.cumsum(cnt)
        cells = np.zeros((max(int(offs[-1]), 1), 4), np.int32)
        k4, ofuv = _cam_args(cam)
        _load().emu_trace(*self._tree_args(), _p(k4), _p(ofuv), ctypes.c_int32(cam.max_level), _p(rays),
                          ctypes.c_int64(len(rays)), _p(offs), _p(cells))
        return offs, cells[:int(offs[-1])]

    def render_cut(self, cam, op, level, field=0, weight=0, los=False, rays=None):
        """The learned-LOD tile walk at `level` (two spans per ray): values,
        aux and whether each ray cut a cell."""
        n = cam.W * cam.H if rays is None else len(rays)
        pix = np.arange(n, dtype=np.int64) if rays is None else np.ascontiguousarray(rays, np.int64)
        out = np.zeros(n, np.float32)
        aux = np.zeros(n, np.float32)
        cut = np.zeros(n, np.int32)
        k4, ofuv = _cam_args(cam)
        _load().emu_render_cut(*self._tree_args(), _p(k4), _p(ofuv), ctypes.c_int32(op), ctypes.c_int32(field),
                               ctypes.c_int32(weight), ctypes.c_int32(int(los)), ctypes.c_int32(level), _p(pix),
                               ctypes.c_int64(n), _p(out), _p(aux), _p(cut))
        return out, aux, cut.astype(bool)

    def render_split(self, cam, op, K, field=0, weight=0, los=False, rays=None, with_cells=False):
        """Split-ray path (K spans per ray, merged in span order): values,
        aux, per-ray cell counts and, optionally, the concatenated cells."""
        n = cam.W * cam.H if rays is None else len(rays)
        pix = np.arange(n, dtype=np.int64) if rays is None else np.ascontiguousarray(rays, np.int64)
        out = np.zeros(n, np.float32)
        aux = np.zeros(n, np.float32)
        cnt = np.zeros(n, np.int32)
        k4, ofuv = _cam_args(cam)
        args = (_p(k4), _p(ofuv), ctypes.c_int32(op), ctypes.c_int32(field), ctypes.c_int32(weight),
                ctypes.c_int32(int(los)), ctypes.c_int32(cam.max_level), _p(pix), ctypes.c_int64(n))
        tail = (ctypes.c_int32(K),)
        _load().emu_render_split(*self._tree_args(), *args, _p(out), _p(aux), _p(cnt), None, None, *tail)
        if not with_cells:
            return out, aux, cnt, None
        offs = np.zeros(n + 1, np.int64)
        offs[1:] = np.cumsum(cnt)
        cells = np.zeros((max(int(offs[-1]), 1), 4), np.int32)
        _load().emu_render_split(*self._tree_args(), *args, None, None, None, _p(offs), _p(cells), *tail)
        return out, aux, cnt, (offs, cells[:int(offs[-1])])


class EmuStream:
    """The streamed render over a library stream plan's chunk arrays, on the
    CPU: each chunk's rays clipped to its cube and walked by the traversal
    core, partials merged in chunk order (as the streamed kernels do)."""

    def __init__(self, plan, tree):
        info = tree.info
        self.plan = plan
        self.base = min(int(info.levelmin), 10)
        self.lmax = int(info.lmax)
        self.nfields = int(info.nfields)
        self.chunks = [plan.chunk(i) for i in range(plan.nchunks)]

    def _chunk_call(self, c, cam, op, field, weight, los, ml, pix, acc, counts, entry, offsets=None, cells=None):
        k4, ofuv = _cam_args(cam)
        off = np.array(c["off_local"], np.int32)
        _load().emu_stream_chunk(
            _p(c["records"]), _p(c["values"]), _p(c["packed"]), ctypes.c_int64(c["ncells"]),
            ctypes.c_int32(self.nfields), ctypes.c_int32(self.base), ctypes.c_int32(self.lmax), _p(off),
            ctypes.c_int32(c["level"]), ctypes.c_int32(c["ix"]), ctypes.c_int32(c["iy"]), ctypes.c_int32(c["iz"]),
            _p(k4), _p(ofuv), ctypes.c_int32(op), ctypes.c_int32(field), ctypes.c_int32(weight),
            ctypes.c_int32(int(los)), ctypes.c_int32(ml), _p(pix), ctypes.c_int64(len(pix)), _p(acc), _p(counts),
            _p(entry), _p(offsets), _p(cells))

    def render(self, cam, op, field=0, weight=0, los=False, rays=None, check_rects=True):
        """(out, aux, counts); with check_rects, every ray that meets a
        chunk's cube must lie in the plan's pixel rectangle of that chunk."""
        n = cam.W * cam.H if rays is None else len(rays)
        pix = np.arange(n, dtype=np.int64) if rays is None else np.ascontiguousarray(rays, np.int64)
        acc = np.zeros((n, 4), np.float32)
        if op == 1:
            acc[:, 0] = -np.inf
        cnt = np.zeros(n, np.int32)
        for k, c in enumerate(self.chunks):
            entry = np.zeros(2 * n, np.int64)
            self._chunk_call(c, cam, op, field, weight, los, cam.max_level, pix, acc, cnt, entry)
            if check_rects:
                hit = entry[1::2] != 0
                i0, j0, i1, j1 = self.plan.rect(k, cam)
                pi, pj = pix % cam.W, pix // cam.W
                inside = (pi >= i0) & (pi <= i1) & (pj >= j0) & (pj <= j1)
                assert not (hit & ~inside).any(), f"chunk {k} rectangle misses rays"
        out = np.zeros(n, np.float32)
        aux = np.zeros(n, np.float32)
        _load().emu_stream_finish(ctypes.c_int32(op), _p(acc), ctypes.c_int64(n), _p(out), _p(aux))
        return out, aux, cnt

    def trace(self, cam, rays):
        """Cells of each ray: every chunk's piece, pieces ordered along the
        ray by their exact entry parameter."""
        from fractions import Fraction

        pix = np.ascontiguousarray(rays, np.int64)
        n = len(pix)
        pieces = [[] for _ in range(n)]
        for c in self.chunks:
            acc = np.zeros((n, 4), np.float32)
            cnt = np.zeros(n, np.int32)
            entry = np.zeros(2 * n, np.int64)
            self._chunk_call(c, cam, 1, 0, 0, False, cam.max_level, pix, acc, cnt, entry)
            offs = np.zeros(n + 1, np.int64)
            offs[1:] = np.cumsum(cnt)
            cells = np.zeros((max(int(offs[-1]), 1), 4), np.int32)
            cnt2 = np.zeros(n, np.int32)
            self._chunk_call(c, cam, 1, 0, 0, False, cam.max_level, pix, acc, cnt2, entry, offs, cells)
            for r in range(n):
                if entry[2 * r + 1]:
                    pieces[r].append((Fraction(int(entry[2 * r]), int(entry[2 * r + 1])), cells[offs[r]:offs[r + 1]]))
        out_offs = np.zeros(n + 1, np.int64)
        seqs = []
        for r in range(n):
            ps = sorted(pieces[r], key=lambda q: q[0])
            assert all(ps[k][0] < ps[k + 1][0] for k in range(len(ps) - 1)), "two pieces enter at one point"
            s = np.concatenate([q[1] for q in ps]) if ps else np.zeros((0, 4), np.int32)
            seqs.append(s)
            out_offs[r + 1] = out_offs[r] + len(s)
        cells = np.concatenate(seqs) if int(out_offs[-1]) else np.zeros((0, 4), np.int32)
        return out_offs, cells
