"""MI355X octree AMR ray caster -- thin Python binding over libamr.so.

Every step of the path runs in the library's HIP kernels; this module only
marshals arguments through ctypes.  PyTorch supplies device memory and the
stream (``torch.cuda.current_stream().cuda_stream``).  The library must be
built (``python -m paper_1210_8014_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (AMR_DEVICE, AMR_HOST, AMR_MAX, AMR_SUM, AMR_WMEAN, BuildOpts, Camera, CameraDesc, LeavesC,
                   RenderOpts, TreeInfo)

SUM, MAX, WMEAN = AMR_SUM, AMR_MAX, AMR_WMEAN
HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamr.so")


class AmrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_abi.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libamr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1210_8014_amd.build`")
        _lib = _abi.declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _check(rc: int):
    if rc != 0:
        raise AmrError(rc, lib().amr_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    """Address of a torch tensor or numpy array (None -> NULL)."""
    if t is None:
        return ctypes.c_void_p(0)
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ tree

class Tree:
    """Library-owned linear octree (amr_build_linear_octree)."""

    def __init__(self, leaves, restrict=None, host_only: bool = False, stream=None):
        L = lib()
        lv = np.ascontiguousarray(leaves.level, np.int32)
        ix = np.ascontiguousarray(leaves.ix, np.int32)
        iy = np.ascontiguousarray(leaves.iy, np.int32)
        iz = np.ascontiguousarray(leaves.iz, np.int32)
        fl = np.ascontiguousarray(leaves.fields, np.float32)
        if fl.ndim == 1:
            fl = fl.reshape(1, -1)
        c = LeavesC()
        c.n = lv.shape[0]
        c.level, c.ix, c.iy, c.iz = (x.ctypes.data for x in (lv, ix, iy, iz))
        c.fields = fl.ctypes.data
        c.nfields = fl.shape[0]
        c.location = AMR_HOST
        c.field_stride = fl.shape[1]
        o = BuildOpts()
        if restrict is None:
            o.use_defaults = 1
        else:
            for k, w in enumerate(restrict):
                o.restrict_weight[k] = int(w)
        o.host_only = int(bool(host_only))
        h = ctypes.c_void_p()
        _check(L.amr_build_linear_octree(ctypes.byref(c), ctypes.byref(o),
                                         ctypes.c_void_p(0) if host_only else _stream(stream), ctypes.byref(h)))
        self._h = h
        self.info = TreeInfo()
        _check(L.amr_tree_info(h, ctypes.byref(self.info)))

    @property
    def handle(self):
        return self._h

    @property
    def lmax(self) -> int:
        return int(self.info.lmax)

    @property
    def ncells(self) -> int:
        return int(self.info.ncells)

    def arrays(self):
        """(child, values, maxdepth) addresses: host for host_only trees."""
        c, v, m = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().amr_tree_arrays(self._h, ctypes.byref(c), ctypes.byref(v), ctypes.byref(m)))
        return c.value, v.value, m.value

    def host_arrays(self):
        """numpy copies of the per-cell arrays of a host_only tree."""
        assert self.info.host_only
        c, v, m = self.arrays()
        n, nf = self.ncells, int(self.info.nfields)
        child = np.ctypeslib.as_array(ctypes.cast(c, ctypes.POINTER(ctypes.c_int32)), (n,)).copy()
        vals = np.ctypeslib.as_array(ctypes.cast(v, ctypes.POINTER(ctypes.c_float)), (nf * n,)).copy().reshape(nf, n)
        md = np.ctypeslib.as_array(ctypes.cast(m, ctypes.POINTER(ctypes.c_uint8)), (n,)).copy()
        return child, vals, md

    def close(self):
        if getattr(self, "_h", None):
            lib().amr_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- camera

_KIND = {"persp": 0, "ortho": 1}


def camera_desc(d: dict) -> CameraDesc:
    c = CameraDesc()
    c.kind = _KIND[d["kind"]] if isinstance(d["kind"], str) else int(d["kind"])
    c.W, c.H = int(d["W"]), int(d["H"])
    c.max_level = int(d.get("max_level", -1))
    c.level_bias = int(d.get("level_bias", 0))
    for k in range(3):
        c.eye[k], c.target[k], c.up[k] = d["eye"][k], d["target"][k], d["up"][k]
    c.fov_y = float(d.get("fov_y", 0.0))
    c.ortho_height = float(d.get("ortho_height", 0.0))
    return c


def set_camera(d: dict, tree: Optional[Tree] = None) -> Camera:
    out = Camera()
    _check(lib().amr_set_camera(ctypes.byref(camera_desc(d)), tree.handle if tree else None, ctypes.byref(out)))
    return out


# ---------------------------------------------------------------- render

def render(tree: Tree, cam: Camera, op: int, out, aux=None, field: int = 0, weight: int = 0, los: bool = False,
           variant: int = -1, stream=None):
    """Enqueue one image into ``out`` (device fp32 tensor of H*W)."""
    o = RenderOpts(field, weight, int(bool(los)), variant)
    _check(lib().amr_render(tree.handle, ctypes.byref(cam), op, ctypes.byref(o), _ptr(out), _ptr(aux),
                            _stream(stream)))
    return out


def count_segments(tree: Tree, cam: Camera, total, counts=None, stream=None):
    """Segments per pixel (``counts``, device int32, optional) and their
    total (``total``, device int64 of one element)."""
    _check(lib().amr_count_segments(tree.handle, ctypes.byref(cam), _ptr(counts), _ptr(total), _stream(stream)))


def mark_cells(tree: Tree, cam: Camera, bitmap, distinct, stream=None):
    """Sets bit c of ``bitmap`` (device int32/uint32, ceil(ncells/32) words)
    for every cell c the image's rays meet and adds the number of newly set
    bits to ``distinct`` (device int64 of one element)."""
    _check(lib().amr_mark_cells(tree.handle, ctypes.byref(cam), _ptr(bitmap), _ptr(distinct), _stream(stream)))


def resolution(tree: Tree, cam: Camera, res, stream=None):
    """Per-pixel local resolution (amr_render_resolution) into ``res``
    (device fp32 of H*W)."""
    _check(lib().amr_render_resolution(tree.handle, ctypes.byref(cam), _ptr(res), _stream(stream)))
    return res


def render_with_resolution(tree: Tree, cam: Camera, op: int, out, res, aux=None, field: int = 0, weight: int = 0,
                           los: bool = False, stream=None):
    """One walk for the image (``out``, as variant p8x8_w1_fast) and its
    resolution plane (``res``): amr_render_with_resolution."""
    o = RenderOpts(field, weight, int(bool(los)), -1)
    _check(lib().amr_render_with_resolution(tree.handle, ctypes.byref(cam), op, ctypes.byref(o), _ptr(out), _ptr(aux),
                                            _ptr(res), _stream(stream)))
    return out, res


def blur_workspace_bytes(W: int, H: int) -> int:
    return int(lib().amr_blur_workspace_bytes(W, H))


def blur_adaptive(img, res, W: int, H: int, kappa: float, out, workspace, stream=None):
    """Adaptive Gaussian blur (amr_blur_adaptive) of ``img`` with sigma =
    kappa * res; ``workspace`` a device tensor of blur_workspace_bytes(W, H)."""
    _check(lib().amr_blur_adaptive(_ptr(img), _ptr(res), W, H, float(kappa), _ptr(out), _ptr(workspace),
                                   int(workspace.numel() * workspace.element_size()), _stream(stream)))
    return out


def slice_map(tree: Tree, cam: Camera, out, field: int = 0, stream=None):
    """Slice map (amr_slice) of an orthographic record into ``out``."""
    _check(lib().amr_slice(tree.handle, ctypes.byref(cam), field, _ptr(out), _stream(stream)))
    return out


def count_rays(tree: Tree, cam: Camera, ray_ids, counts, stream=None):
    _check(lib().amr_count_rays(tree.handle, ctypes.byref(cam), _ptr(ray_ids), int(ray_ids.numel()), _ptr(counts),
                                _stream(stream)))


def trace_rays(tree: Tree, cam: Camera, ray_ids, offsets, cells, stream=None):
    _check(lib().amr_trace_rays(tree.handle, ctypes.byref(cam), _ptr(ray_ids), int(ray_ids.numel()), _ptr(offsets),
                                _ptr(cells), _stream(stream)))


def variants():
    L = lib()
    return [L.amr_variant_name(v).decode() for v in range(L.amr_variant_count())]


def default_variant() -> int:
    """Index of the variant amr_render uses when none is selected or tuned."""
    return int(lib().amr_variant_default())


# ----------------------------------------------------------------- batch

class Batch:
    """Persistent, graph-captured render of many (tree, camera) images
    (amr_batch_create / amr_render_batch).  outs[k] (and auxs[k]) are device
    tensors fixed at creation."""

    def __init__(self, trees, cams, pairs, op, outs, auxs=None, field=0, weight=0, los=False):
        L = lib()
        self._trees = list(trees)  # keep the Python handles alive
        nt, nc, n = len(trees), len(cams), len(pairs)
        th = (ctypes.c_void_p * nt)(*[t.handle.value for t in trees])
        ca = (Camera * nc)(*cams)
        pr = (ctypes.c_int32 * (2 * n))(*[int(v) for p in pairs for v in p])
        oa = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        xa = (ctypes.c_void_p * n)(*[x.data_ptr() for x in auxs]) if auxs is not None else None
        o = RenderOpts(field, weight, int(bool(los)), -1)
        h = ctypes.c_void_p()
        _check(L.amr_batch_create(th, nt, ca, nc, pr, n, op, ctypes.byref(o), oa, xa, ctypes.byref(h)))
        self._h = h
        self.outs, self.auxs = outs, auxs

    def run(self, stream=None):
        _check(lib().amr_render_batch(self._h, _stream(stream)))

    def tune(self, reps: int = 2):
        L = lib()
        n = L.amr_batch_config_count()
        times = (ctypes.c_float * n)()
        best = ctypes.c_int32()
        _check(L.amr_batch_tune(self._h, reps, ctypes.byref(best), times))
        return int(best.value), {L.amr_batch_config_name(c).decode(): float(times[c]) for c in range(n)}

    def set_config(self, c: int):
        _check(lib().amr_batch_set_config(self._h, c))

    @property
    def config(self) -> int:
        return int(lib().amr_batch_config(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().amr_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------- trees larger than the GPU

class StreamPlan:
    """A host_only tree cut into chunks for streamed renders
    (amr_stream_plan_create / amr_render_streamed).  ``tree`` must be built
    with ``host_only=True``; it may be closed once the plan exists."""

    def __init__(self, tree: Tree, max_chunk_cells: int, host_only: bool = False, nbuffers: int = 0):
        o = _abi.StreamOpts(int(max_chunk_cells), int(bool(host_only)), int(nbuffers))
        h = ctypes.c_void_p()
        _check(lib().amr_stream_plan_create(tree.handle, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.info = _abi.StreamPlanInfo()
        _check(lib().amr_stream_plan_info(h, ctypes.byref(self.info)))
        self.nfields = int(tree.info.nfields)

    @property
    def nchunks(self) -> int:
        return int(self.info.nchunks)

    def chunk(self, i: int) -> dict:
        """Chunk i: cube, level starts, local offsets and numpy views of its
        host arrays (records as (child int32, field-0 bits) pairs)."""
        c = _abi.StreamChunk()
        _check(lib().amr_stream_chunk(self._h, i, ctypes.byref(c)))
        n = int(c.ncells)
        rec = np.ctypeslib.as_array(ctypes.cast(c.records, ctypes.POINTER(ctypes.c_int32)), (n, 2))
        vals = np.ctypeslib.as_array(ctypes.cast(c.values, ctypes.POINTER(ctypes.c_float)), (self.nfields, n))
        pk = (np.ctypeslib.as_array(ctypes.cast(c.packed, ctypes.POINTER(ctypes.c_float)), (n, 4))
              if c.packed else None)
        return dict(level=c.level, ix=c.ix, iy=c.iy, iz=c.iz, ncells=n, first=int(c.first),
                    level_start=list(c.level_start), off_local=list(c.off_local), records=rec, values=vals, packed=pk)

    def rect(self, i: int, cam: Camera):
        """(i0, j0, i1, j1) of chunk i for cam (i1 < i0: no pixel)."""
        r = (ctypes.c_int32 * 4)()
        _check(lib().amr_stream_chunk_rect(self._h, i, ctypes.byref(cam), r))
        return tuple(int(v) for v in r)

    @staticmethod
    def workspace_bytes(W: int, H: int) -> int:
        return int(lib().amr_stream_workspace_bytes(W, H))

    def render(self, cam: Camera, op: int, out, workspace, aux=None, field: int = 0, weight: int = 0,
               los: bool = False, stream=None):
        """Streamed render into ``out``; returns (chunks walked, bytes copied
        to the device, pixels covered)."""
        o = RenderOpts(field, weight, int(bool(los)), -1)
        st = (ctypes.c_int64 * 3)()
        _check(lib().amr_render_streamed(self._h, ctypes.byref(cam), op, ctypes.byref(o), _ptr(out), _ptr(aux),
                                         _ptr(workspace), int(workspace.numel() * workspace.element_size()), st,
                                         _stream(stream)))
        return int(st[0]), int(st[1]), int(st[2])

    def close(self):
        if getattr(self, "_h", None):
            lib().amr_stream_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_configs():
    L = lib()
    return [L.amr_batch_config_name(c).decode() for c in range(L.amr_batch_config_count())]


# ----------------------------------------------------------------- tuning

def tune(tree: Tree, cam: Camera, op: int, out, aux=None, field: int = 0, weight: int = 0, los: bool = False,
         reps: int = 2, stream=None, cache: Optional[str] = None):
    """Time every kernel variant on this image, make the fastest the tree's
    default for ``op`` and return (best, {variant: ms}).  With ``cache`` (a
    JSON path, default $AMR_TUNE_CACHE) the choice is stored under a key of
    the tree shape, image size and op, and reused by :func:`apply_tuning`."""
    L = lib()
    n = L.amr_variant_count()
    times = (ctypes.c_float * n)()
    best = ctypes.c_int32()
    o = RenderOpts(field, weight, int(bool(los)), -1)
    _check(L.amr_tune(tree.handle, ctypes.byref(cam), op, ctypes.byref(o), _ptr(out), _ptr(aux), _stream(stream),
                      reps, ctypes.byref(best), times))
    res = {L.amr_variant_name(v).decode(): float(times[v]) for v in range(n)}
    path = cache or os.environ.get("AMR_TUNE_CACHE")
    if path:
        import json

        data = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
        data[_tune_key(tree, cam, op)] = L.amr_variant_name(best.value).decode()
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return int(best.value), res


def _tune_key(tree: Tree, cam: Camera, op: int) -> str:
    i = tree.info
    return f"gfx950/cells{i.ncells}/l{i.levelmin}-{i.lmax}/cam{cam.kind}/{cam.W}x{cam.H}/L{cam.max_level}/op{op}"


def apply_tuning(tree: Tree, cam: Camera, op: int, cache: Optional[str] = None) -> int:
    """Set the tree's default variant for ``op`` from the tuning cache;
    returns the variant (or -1 if the cache has no entry)."""
    import json

    path = cache or os.environ.get("AMR_TUNE_CACHE")
    if not path or not os.path.exists(path):
        return -1
    with open(path) as f:
        name = json.load(f).get(_tune_key(tree, cam, op))
    if name is None or name not in variants():
        return -1
    v = variants().index(name)
    _check(lib().amr_set_default_variant(tree.handle, op, v))
    return v
