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
