"""CPU oracle for octree ray casting (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it
and shares no code with it.  The ray casting lives in ``oracle.c`` (fp64 plus
exact 128-bit integer predicates), which consumes the integer camera record;
the record itself comes from ``camera.py`` (exact rational and 90-digit
decimal arithmetic).  This module builds the C part with gcc and marshals
numpy arrays through ctypes.

Function -> what pins it (tests/test_oracle_pins.py, tests/golden/):
  camera quantisation   hand-derived orthographic and perspective records,
                        the field-of-view edge ray, integer round trip,
                        bounds, mirror symmetry
  tree build/restrict   mass conservation at every truncation level,
                        momentum conservation, rejection of gaps/overlaps
  segments and order    exact Fraction brute force over every leaf,
                        textbook grid DDA on uniform trees, closed-form counts
  chord lengths         constant field -> value x box chord; sum of chords
  sum / max / wmean     brute force, dense-grid sums, bounds, constant-field
                        and unit-weight identities; a hand-worked three-cell
                        weighted mean with its error scales; a cancelling
                        sum that plain fp64 accumulation gets wrong
                        (compensation)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

from . import camera as _camera

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SUM, MAX, WMEAN = 0, 1, 2
OK, EINVAL, ETREE, ENOMEM, ECAPACITY = 0, 1, 2, 3, 4


class Camera(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("max_level", ctypes.c_int32),
        ("O", ctypes.c_int64 * 3), ("F", ctypes.c_int64 * 3), ("U", ctypes.c_int64 * 3), ("V", ctypes.c_int64 * 3),
    ]

    def as_dict(self) -> dict:
        return dict(kind=self.kind, W=self.W, H=self.H, max_level=self.max_level, O=list(self.O), F=list(self.F),
                    U=list(self.U), V=list(self.V))


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", _SRC,
               "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
_P = ctypes.POINTER


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oc_tree_build.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5 + [ctypes.c_int32, ctypes.c_int64,
                                                                                 ctypes.c_void_p,
                                                                                 _P(ctypes.c_void_p)]
        lib.oc_tree_free.argtypes = [ctypes.c_void_p]
        lib.oc_tree_nodes.argtypes = [ctypes.c_void_p]
        lib.oc_tree_nodes.restype = ctypes.c_int64
        lib.oc_tree_lmax.argtypes = [ctypes.c_void_p]
        lib.oc_lookup.argtypes = [ctypes.c_void_p] + [ctypes.c_int32] * 4 + [ctypes.c_void_p, ctypes.c_void_p]
        lib.oc_render.argtypes = [ctypes.c_void_p, _P(Camera), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 6 + [
                                      ctypes.c_int32]
        lib.oc_trace.argtypes = [ctypes.c_void_p, _P(Camera), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32]
        lib.oc_pixel_ray.argtypes = [_P(Camera), ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        lib.oc_slice.argtypes = [ctypes.c_void_p, _P(Camera), ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p]
        lib.oc_resolution.argtypes = [ctypes.c_void_p, _P(Camera), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_int32]
        lib.oc_probe_stats.argtypes = [ctypes.c_void_p, _P(Camera), ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int32]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def set_camera(d: dict, tree_lmax: int = -1) -> Camera:
    """Quantise a camera description (camera.quantise); raises ValueError
    (camera.CameraError) when rejected."""
    r = _camera.quantise(d, tree_lmax if tree_lmax >= 0 else None)
    return record(r.as_dict())


def record(rec: dict) -> Camera:
    """The C struct of an integer camera record given as a dict."""
    out = Camera()
    out.kind, out.W, out.H, out.max_level = int(rec["kind"]), int(rec["W"]), int(rec["H"]), int(rec["max_level"])
    for k in range(3):
        out.O[k], out.F[k], out.U[k], out.V[k] = (int(rec["O"][k]), int(rec["F"][k]), int(rec["U"][k]),
                                                  int(rec["V"][k]))
    return out


def pixel_ray(cam: Camera, i: int, j: int):
    o = np.zeros(3, np.int64)
    d = np.zeros(3, np.int64)
    _load().oc_pixel_ray(ctypes.byref(cam), i, j, _ptr(o), _ptr(d))
    return o, d


def default_restrict(nfields: int) -> np.ndarray:
    """Field 0 (density) restricts as a volume mean; the others as means
    weighted by field 0 (mass-weighted)."""
    r = np.full(nfields, 0, np.int32)
    r[0] = -1
    return r


class Tree:
    """The oracle's own octree, built by inserting each leaf from the root."""

    def __init__(self, leaves, restrict: Optional[Sequence[int]] = None):
        lib = _load()
        self.level = np.ascontiguousarray(leaves.level, np.int32)
        ix = np.ascontiguousarray(leaves.ix, np.int32)
        iy = np.ascontiguousarray(leaves.iy, np.int32)
        iz = np.ascontiguousarray(leaves.iz, np.int32)
        fl = np.ascontiguousarray(leaves.fields, np.float32)
        if fl.ndim == 1:
            fl = fl.reshape(1, -1)
        self.nfields = fl.shape[0]
        rs = default_restrict(self.nfields) if restrict is None else np.asarray(restrict, np.int32)
        h = ctypes.c_void_p()
        rc = lib.oc_tree_build(int(self.level.shape[0]), _ptr(self.level), _ptr(ix), _ptr(iy), _ptr(iz), _ptr(fl),
                               self.nfields, fl.shape[1], _ptr(rs), ctypes.byref(h))
        if rc != OK:
            raise ValueError(f"oracle tree build failed ({rc})")
        self._h = h
        self.lmax = int(lib.oc_tree_lmax(h))
        self.nodes = int(lib.oc_tree_nodes(h))

    def close(self):
        if getattr(self, "_h", None):
            _load().oc_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lookup(self, level, ix, iy, iz):
        v32 = np.zeros(self.nfields, np.float32)
        v64 = np.zeros(self.nfields, np.float64)
        rc = _load().oc_lookup(self._h, level, ix, iy, iz, _ptr(v32), _ptr(v64))
        if rc != OK:
            raise KeyError((level, ix, iy, iz))
        return v32, v64

    def camera(self, d: dict) -> Camera:
        return set_camera(d, self.lmax)

    def render(self, cam: Camera, op: int, field: int = 0, weight: int = 0, los: bool = False,
               rays: Optional[np.ndarray] = None, nthreads: int = 0):
        """Returns dict with 'val' (fp64; sum or wmean), 'max' (fp32),
        'aux' (wmean weight), 'absf' (wmean: weighted mean of |f|, with los of
        the summed magnitudes of the three velocity terms: the error-bar
        scale), 'absdot' (wmean: weighted mean of |f| itself), 'count'.  Arrays are
        flat over the requested rays (pixel index j*W+i), or over all pixels."""
        n = cam.W * cam.H if rays is None else int(len(rays))
        r = None if rays is None else np.ascontiguousarray(rays, np.int64)
        val = np.zeros(n, np.float64) if op != MAX else None
        mx = np.zeros(n, np.float32) if op == MAX else None
        aux = np.zeros(n, np.float64) if op == WMEAN else None
        absf = np.zeros(n, np.float64) if op == WMEAN else None
        absdot = np.zeros(n, np.float64) if op == WMEAN else None
        cnt = np.zeros(n, np.int32)
        rc = _load().oc_render(self._h, ctypes.byref(cam), op, field, weight, int(bool(los)), _ptr(r), n, _ptr(val),
                               _ptr(mx), _ptr(aux), _ptr(absf), _ptr(absdot), _ptr(cnt),
                               int(nthreads))
        if rc != OK:
            raise RuntimeError(f"oracle render failed ({rc})")
        return dict(val=val, max=mx, aux=aux, absf=absf, absdot=absdot, count=cnt)

    def slice(self, cam: Camera, field: int = 0, rays: Optional[np.ndarray] = None) -> np.ndarray:
        """Slice map of an orthographic record (oc_slice): fp32 value of the
        truncated cell holding each pixel's point, NaN outside the box."""
        n = cam.W * cam.H if rays is None else int(len(rays))
        r = None if rays is None else np.ascontiguousarray(rays, np.int64)
        out = np.zeros(n, np.float32)
        rc = _load().oc_slice(self._h, ctypes.byref(cam), field, _ptr(r), n, _ptr(out))
        if rc != OK:
            raise ValueError(f"oracle slice failed ({rc})")
        return out

    def resolution(self, cam: Camera, rays: Optional[np.ndarray] = None, nthreads: int = 0) -> np.ndarray:
        """Per-pixel local resolution (oc_resolution): chord-weighted mean
        cell side in pixels at the cell's depth, fp64."""
        n = cam.W * cam.H if rays is None else int(len(rays))
        r = None if rays is None else np.ascontiguousarray(rays, np.int64)
        out = np.zeros(n, np.float64)
        rc = _load().oc_resolution(self._h, ctypes.byref(cam), _ptr(r), n, _ptr(out), int(nthreads))
        if rc != OK:
            raise RuntimeError(f"oracle resolution failed ({rc})")
        return out

    def probe_stats(self, cam: Camera, rays: np.ndarray, field: int = 0, nthreads: int = 0) -> np.ndarray:
        """[n, 16] per-ray statistics for the learned level of detail (see
        oc_probe_stats in oracle.c)."""
        r = np.ascontiguousarray(rays, np.int64)
        out = np.zeros((len(r), 16), np.float64)
        rc = _load().oc_probe_stats(self._h, ctypes.byref(cam), field, _ptr(r), len(r), _ptr(out), int(nthreads))
        if rc != OK:
            raise RuntimeError(f"oracle probe stats failed ({rc})")
        return out

    def trace(self, cam: Camera, rays: np.ndarray, with_t: bool = False, nthreads: int = 0):
        """Cell sequences: (offsets[n+1], cells[S,4] = level, ix, iy, iz,
        tq[S,4] exact entry/exit parameters as num/den pairs or None)."""
        lib = _load()
        r = np.ascontiguousarray(rays, np.int64)
        n = int(r.shape[0])
        offs = np.zeros(n + 1, np.int64)
        rc = lib.oc_trace(self._h, ctypes.byref(cam), _ptr(r), n, None, None, 0, _ptr(offs), int(nthreads))
        if rc != OK:
            raise RuntimeError(f"oracle trace failed ({rc})")
        S = int(offs[-1])
        cells = np.zeros((max(S, 1), 4), np.int32)
        tq = np.zeros((max(S, 1), 4), np.int64) if with_t else None
        rc = lib.oc_trace(self._h, ctypes.byref(cam), _ptr(r), n, _ptr(cells), _ptr(tq), S, _ptr(offs),
                          int(nthreads))
        if rc != OK:
            raise RuntimeError(f"oracle trace failed ({rc})")
        return offs, cells[:S], (tq[:S] if with_t else None)
