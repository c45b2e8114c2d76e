"""Seeded synthetic AMR octree scenes and camera descriptions (inputs only).

The module builds ``libamrgen.so`` from ``amrgen.cpp`` (g++, no GPU) and
exposes the scenes as numpy arrays.  It holds none of the renderer's
arithmetic: it decides which cells are leaves, what fp32 fields they carry
and where the cameras are.  Both the CPU oracle and the GPU library take its
output as plain data.

Workloads (a level-l cell has side 2^-l of the unit box):

* ``tiny``      levels 3..6, ~40k leaves, 8 Gaussian blobs x lognormal(0.5)
                noise, one density field; 256x256 orthographic camera along +z.
* ``disk``      galaxy disk in a 50 kpc box, levels 7..16, ~20M leaves,
                density + 3 velocity components; 2048^2 perspective cameras at
                inclinations 0, 45 and 90 degrees.
* ``deepzoom``  the same disk model to level 22, ~200M leaves, density only;
                a 4096^2 camera inside the disk aimed at core 0, whose maximum
                level follows from the pixel footprint.
* ``batch``     8 disk snapshots (seeds 0..7, 5..25M leaves) x 64 orbit
                cameras with image sides log-uniform in [512, 2048].
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amrgen.cpp")
_LIB = os.path.join(_HERE, "libamrgen.so")
_CONFIGS = os.path.join(_HERE, "configs.json")

BLOBS, DISK = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("levelmin", ctypes.c_int32),
        ("lmax", ctypes.c_int32),
        ("with_cores", ctypes.c_int32),
        ("with_velocity", ctypes.c_int32),
        ("ncores", ctypes.c_int32),
        ("nmodes", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("threshold", ctypes.c_double),
        ("kappa", ctypes.c_double),
    ]


class _Leaves(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nfields", ctypes.c_int32),
        ("lmax_reached", ctypes.c_int32),
        ("level", ctypes.POINTER(ctypes.c_int32)),
        ("ix", ctypes.POINTER(ctypes.c_int32)),
        ("iy", ctypes.POINTER(ctypes.c_int32)),
        ("iz", ctypes.POINTER(ctypes.c_int32)),
        ("fields", ctypes.POINTER(ctypes.c_float)),
    ]


def build(force: bool = False) -> str:
    """Compile libamrgen.so (host C++, multithreaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", _SRC, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.amrgen_generate.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Leaves), ctypes.c_int, ctypes.c_int]
        lib.amrgen_generate.restype = ctypes.c_int
        lib.amrgen_free.argtypes = [ctypes.POINTER(_Leaves)]
        lib.amrgen_core_position.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        lib.amrgen_core_position.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Leaves:
    """Octree leaves: level and integer coordinates (0 <= i < 2^level) plus
    fp32 fields laid out [nfields][n] (field 0 = density; fields 1..3 =
    velocity when present)."""

    level: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    iz: np.ndarray
    fields: np.ndarray
    lmax: int = 0
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.level.shape[0])

    @property
    def nfields(self) -> int:
        return int(self.fields.shape[0])

    def permuted(self, seed: int) -> "Leaves":
        """The same leaves in a seeded random order (for builder tests)."""
        p = np.random.default_rng(seed).permutation(self.n)
        return Leaves(self.level[p].copy(), self.ix[p].copy(), self.iy[p].copy(), self.iz[p].copy(),
                      np.ascontiguousarray(self.fields[:, p]), self.lmax, dict(self.params))


def _params(kind, seed, levelmin, lmax, threshold, with_cores=1, with_velocity=1, ncores=16, nmodes=64,
            kappa=4.0) -> _Params:
    return _Params(kind, levelmin, lmax, with_cores, with_velocity, ncores, nmodes, 0, seed, threshold, kappa)


def generate(kind: int, seed: int, levelmin: int, lmax: int, threshold: float, with_cores: bool = True,
             with_velocity: bool = True, nthreads: int = 0, count_only: bool = False):
    lib = _load()
    prm = _params(kind, seed, levelmin, lmax, threshold, int(with_cores), int(with_velocity))
    out = _Leaves()
    rc = lib.amrgen_generate(ctypes.byref(prm), ctypes.byref(out), int(count_only), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"amrgen_generate failed ({rc})")
    if count_only:
        return int(out.n), int(out.lmax_reached)
    try:
        n, nf = int(out.n), int(out.nfields)

        def grab(ptr, count, dtype):
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)

        lv = grab(out.level, n, np.int32)
        ix = grab(out.ix, n, np.int32)
        iy = grab(out.iy, n, np.int32)
        iz = grab(out.iz, n, np.int32)
        fl = grab(out.fields, n * nf, np.float32).reshape(nf, n)
        return Leaves(lv, ix, iy, iz, fl, int(out.lmax_reached),
                      dict(kind=kind, seed=seed, levelmin=levelmin, lmax=lmax, threshold=threshold,
                           with_cores=with_cores, with_velocity=with_velocity))
    finally:
        lib.amrgen_free(ctypes.byref(out))


def blobs(seed: int = 0, levelmin: int = 3, lmax: int = 6, tau: Optional[float] = None, nthreads: int = 0) -> Leaves:
    if tau is None:
        tau = configs()["tiny"]["tau"]
    return generate(BLOBS, seed, levelmin, lmax, tau, False, False, nthreads)


def disk(seed: int = 0, levelmin: int = 7, lmax: int = 16, m_thr: Optional[float] = None, cores: bool = True,
         velocity: bool = True, nthreads: int = 0) -> Leaves:
    if m_thr is None:
        m_thr = configs()["disk"]["m_thr"]
    return generate(DISK, seed, levelmin, lmax, m_thr, cores, velocity, nthreads)


def core_position(seed: int, lmax: int, m_thr: float, k: int = 0) -> np.ndarray:
    lib = _load()
    prm = _params(DISK, seed, 7, lmax, m_thr)
    xyz = (ctypes.c_double * 3)()
    if lib.amrgen_core_position(ctypes.byref(prm), k, xyz) != 0:
        raise ValueError("bad core index")
    return np.array(list(xyz))


def uniform(level: int, values: Optional[np.ndarray] = None, nfields: int = 1, seed: int = 0) -> Leaves:
    """Uniform tree: every leaf at ``level``; seeded positive random values
    unless ``values`` ([nfields, 8^level] or [8^level]) is given."""
    n = 1 << (3 * level)
    g = np.arange(1 << level, dtype=np.int32)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    lv = np.full(n, level, np.int32)
    if values is None:
        fl = np.random.default_rng(seed).uniform(0.5, 2.0, size=(nfields, n)).astype(np.float32)
    else:
        fl = np.asarray(values, np.float32).reshape(-1, n)
    return Leaves(lv, ix.ravel().astype(np.int32), iy.ravel().astype(np.int32), iz.ravel().astype(np.int32), fl, level)


def random_tree(seed: int, lmax: int, p_refine: float = 0.45, levelmin: int = 1, nfields: int = 1,
                value_range=(0.1, 10.0)) -> Leaves:
    """Small seeded random complete octree (for exhaustive checks)."""
    rng = np.random.default_rng(seed)
    out = []

    def rec(l, x, y, z):
        if l < levelmin or (l < lmax and rng.random() < p_refine):
            for c in range(8):
                rec(l + 1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1))
        else:
            out.append((l, x, y, z))

    rec(0, 0, 0, 0)
    a = np.array(out, dtype=np.int32).reshape(-1, 4)
    fl = rng.uniform(value_range[0], value_range[1], size=(nfields, a.shape[0])).astype(np.float32)
    return Leaves(a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), a[:, 3].copy(), fl, int(a[:, 0].max()))


# ---------------------------------------------------------------- configs

def configs() -> Dict:
    with open(_CONFIGS) as f:
        return json.load(f)


def scene(name: str, seed: Optional[int] = None, nthreads: int = 0) -> Leaves:
    c = configs()[name]
    if seed is None:
        seed = c.get("seed", 0)
    if c["kind"] == "blobs":
        return generate(BLOBS, seed, c["levelmin"], c["lmax"], c["tau"], False, False, nthreads)
    thr = c["m_thr"]
    if "m_thr_by_seed" in c and str(seed) in c["m_thr_by_seed"]:
        thr = c["m_thr_by_seed"][str(seed)]
    return generate(DISK, seed, c["levelmin"], c["lmax"], thr, True, bool(c.get("velocity", True)), nthreads)


# ---------------------------------------------------------------- cameras
# A camera description is a plain dict consumed by both sides:
#   kind 'persp' | 'ortho', eye/target/up (box units), fov_y (radians) or
#   ortho_height (box units), W, H, max_level (-1 = from the pixel footprint),
#   level_bias.

def camera(kind, eye, target, up, W, H, fov_y=0.0, ortho_height=0.0, max_level=-1, level_bias=0) -> dict:
    return dict(kind=kind, eye=[float(v) for v in eye], target=[float(v) for v in target],
                up=[float(v) for v in up], fov_y=float(fov_y), ortho_height=float(ortho_height),
                W=int(W), H=int(H), max_level=int(max_level), level_bias=int(level_bias))


def tiny_camera(W: int = 256, H: int = 256, max_level: int = 6) -> dict:
    """Orthographic view along +z covering [0,1)^2 exactly; origin plane z = -0.5."""
    return camera("ortho", (0.5, 0.5, -0.5), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), W, H, ortho_height=1.0,
                  max_level=max_level)


def disk_camera(incl_deg: float, W: int = 2048, H: int = 2048, max_level: int = 16, azim_deg: float = 0.0,
                dist_kpc: float = 100.0) -> dict:
    """Perspective camera at ``dist_kpc`` from the box centre, inclination
    ``incl_deg`` from face-on, fov_y = 2 atan(25 kpc / dist)."""
    i = math.radians(incl_deg)
    a = math.radians(azim_deg)
    d = dist_kpc / 50.0
    # inclination tilts the view from +z towards -y; azimuth rotates about z
    ox, oy, oz = 0.0, -math.sin(i) * d, math.cos(i) * d
    ux, uy, uz = 0.0, math.cos(i), math.sin(i)
    ca, sa = math.cos(a), math.sin(a)
    eye = (0.5 + ca * ox - sa * oy, 0.5 + sa * ox + ca * oy, 0.5 + oz)
    up = (ca * ux - sa * uy, sa * ux + ca * uy, uz)
    fov = 2.0 * math.atan(25.0 / dist_kpc)
    return camera("persp", eye, (0.5, 0.5, 0.5), up, W, H, fov_y=fov, max_level=max_level)


def disk_cameras(W: int = 2048, H: int = 2048, max_level: int = 16) -> List[dict]:
    return [disk_camera(i, W, H, max_level) for i in (0.0, 45.0, 90.0)]


def deepzoom_camera(W: int = 4096, H: int = 4096, seed: int = 0, max_level: int = -1) -> dict:
    """Eye 2^-9 box from core 0, inside the disk, fov_y = 2 atan(0.625): the
    pixel footprint at the target is 1.25 x 2^-21 box at 4096^2, so the
    automatic maximum level is 21 (not on a rounding boundary of the level
    rule)."""
    c = configs()["deepzoom"]
    tgt = core_position(seed, c["lmax"], c["m_thr"], 0)
    s = 2.0 ** -9
    th = math.radians(60.0)
    eye = (tgt[0], tgt[1] - s * math.sin(th), tgt[2] + s * math.cos(th))
    up = (0.0, math.cos(th), math.sin(th))
    return camera("persp", eye, tgt, up, W, H, fov_y=2.0 * math.atan(0.625), max_level=max_level)


def orbit_cameras(n: int = 64, seed: int = 0, side_lo: int = 512, side_hi: int = 2048, multiple: int = 16,
                  max_level: int = 16) -> List[dict]:
    """Orbit cameras for the batched workload: distance 100 kpc, inclination
    cycling 0/30/60/90 degrees, 16 azimuths; image sides seeded log-uniform in
    [side_lo, side_hi], rounded to ``multiple`` (1 keeps odd sides)."""
    rng = np.random.default_rng(1000 + seed)
    cams = []
    for k in range(n):
        incl = (0.0, 30.0, 60.0, 90.0)[k % 4]
        az = 360.0 * (k // 4) / max(1, n // 4)
        sides = np.exp(rng.uniform(math.log(side_lo), math.log(side_hi), size=2))
        W, H = (int(max(multiple, round(s / multiple) * multiple)) for s in sides)
        W, H = min(W, side_hi), min(H, side_hi)
        cams.append(disk_camera(incl, W, H, max_level, azim_deg=az))
    return cams
