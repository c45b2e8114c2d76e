"""Learned level of detail: binding over the amr_lod_* entry points plus the
dataset, training and evaluation drivers.  Every step runs in libamr.so;
this module marshals device tensors (torch) and loops."""
from __future__ import annotations

import ctypes
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import SUM, Camera, RenderOpts, Tree, _check, _ptr, _stream, lib, render, set_camera

_vp = ctypes.c_void_p
_i32, _i64, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
NCLS, LV0, TILE, NIN, NHID, NOUT = 16, 1, 16, 32, 64, 16
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lod_model.bin")


class LodConfig(ctypes.Structure):
    _fields_ = [("coarse_level", _i32), ("quantile", _f32), ("conf_thresh", _f32), ("rel_tol", _f32),
                ("audit_frac", _f32), ("audit_seed", _i32)]


_SIGS = {
    "amr_lod_param_count": (_i32, []),
    "amr_lod_create": (_i32, [ctypes.POINTER(LodConfig), ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "amr_lod_free": (None, [_vp]),
    "amr_lod_save": (_i32, [_vp, ctypes.c_char_p]),
    "amr_lod_load": (_i32, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "amr_lod_get_config": (_i32, [_vp, ctypes.POINTER(LodConfig)]),
    "amr_lod_set_config": (_i32, [_vp, ctypes.POINTER(LodConfig)]),
    "amr_lod_get_params": (_i32, [_vp, _vp]),
    "amr_lod_set_params": (_i32, [_vp, _vp]),
    "amr_lod_get_grads": (_i32, [_vp, _vp]),
    "amr_lod_tiles": (_i64, [_i32, _i32]),
    "amr_lod_features": (_i32, [_vp, ctypes.POINTER(Camera), _i32, _vp, _vp]),
    "amr_lod_forward": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "amr_lod_loss": (_i32, [_vp, _vp, _i64, _f32, _f32, _vp, _vp, _vp]),
    "amr_lod_backward": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp]),
    "amr_lod_zero_grads": (_i32, [_vp, _vp]),
    "amr_lod_adam_step": (_i32, [_vp, _f32, _vp]),
    "amr_lod_labels": (_i32, [ctypes.POINTER(_vp), _i32, _i32, _f32, _vp, _vp]),
    "amr_lod_workspace_bytes": (_i64, [_i32, _i32]),
    "amr_render_lod": (_i32, [_vp, ctypes.POINTER(Camera), _i32, _vp, ctypes.POINTER(RenderOpts), _vp, _vp, _vp,
                              _vp, _vp, _i64, _vp, _vp]),
    "amr_lod_noalloc_max_bytes": (_i64, []),
    "amr_render_lod_noalloc": (_i32, [_vp, ctypes.POINTER(Camera), _i32, _vp, ctypes.POINTER(RenderOpts), _vp, _vp,
                                      _vp, _vp, _vp, _vp]),
}
_declared = False


def _lib():
    global _declared
    L = lib()
    if not _declared:
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _declared = True
    return L


def default_config() -> dict:
    return dict(coarse_level=4, quantile=0.99, conf_thresh=0.5, rel_tol=1e-3, audit_frac=0.02, audit_seed=0)


def tiles(W: int, H: int) -> int:
    return int(_lib().amr_lod_tiles(W, H))


def workspace_bytes(W: int, H: int) -> int:
    return int(_lib().amr_lod_workspace_bytes(W, H))


class LodModel:
    """Library-owned network (amr_lod_create / amr_lod_load)."""

    def __init__(self, cfg: Optional[dict] = None, seed: int = 0, path: Optional[str] = None):
        L = _lib()
        h = _vp()
        if path is not None:
            _check(L.amr_lod_load(path.encode(), ctypes.byref(h)))
        else:
            c = LodConfig(**(cfg or default_config()))
            _check(L.amr_lod_create(ctypes.byref(c), seed, ctypes.byref(h)))
        self._h = h
        self.nparams = int(L.amr_lod_param_count())

    @property
    def handle(self):
        return self._h

    @property
    def config(self) -> dict:
        c = LodConfig()
        _check(_lib().amr_lod_get_config(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in LodConfig._fields_}

    @config.setter
    def config(self, d: dict):
        cur = self.config
        cur.update(d)
        c = LodConfig(**cur)
        _check(_lib().amr_lod_set_config(self._h, ctypes.byref(c)))

    def params(self) -> np.ndarray:
        p = np.zeros(self.nparams, np.float32)
        _check(_lib().amr_lod_get_params(self._h, p.ctypes.data))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.nparams
        _check(_lib().amr_lod_set_params(self._h, p.ctypes.data))

    def grads(self) -> np.ndarray:
        g = np.zeros(self.nparams, np.float32)
        _check(_lib().amr_lod_get_grads(self._h, g.ctypes.data))
        return g

    def save(self, path: str):
        _check(_lib().amr_lod_save(self._h, path.encode()))

    def forward(self, feat, n, logits, acts=None, stream=None):
        _check(_lib().amr_lod_forward(self._h, _ptr(feat), int(n), _ptr(logits), _ptr(acts), _stream(stream)))

    def backward(self, feat, acts, dlogits, n, dz, stream=None):
        _check(_lib().amr_lod_backward(self._h, _ptr(feat), _ptr(acts), _ptr(dlogits), int(n), _ptr(dz),
                                       _stream(stream)))

    def zero_grads(self, stream=None):
        _check(_lib().amr_lod_zero_grads(self._h, _stream(stream)))

    def adam_step(self, lr: float, stream=None):
        _check(_lib().amr_lod_adam_step(self._h, lr, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib().amr_lod_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(tree: Tree, cam: Camera, feat, coarse_level: int = 9, stream=None):
    """feat: device int16 tensor [tiles, 32] (bf16 bit patterns)."""
    _check(_lib().amr_lod_features(tree.handle, ctypes.byref(cam), coarse_level, _ptr(feat), _stream(stream)))


def loss(logits, labels, n, lam, scale, dlogits, loss_sum=None, stream=None):
    _check(_lib().amr_lod_loss(_ptr(logits), _ptr(labels), int(n), lam, scale, _ptr(dlogits), _ptr(loss_sum),
                               _stream(stream)))


def labels(imgs: Sequence, W: int, H: int, tol: float, out, stream=None):
    arr = (_vp * NCLS)(*[x.data_ptr() for x in imgs])
    _check(_lib().amr_lod_labels(arr, W, H, tol, _ptr(out), _stream(stream)))


def render_lod(tree: Tree, cam: Camera, op: int, model: LodModel, out, workspace, stats, aux=None, field: int = 0,
               weight: int = 0, los: bool = False, tile_levels=None, forced=None, stream=None):
    o = RenderOpts(field, weight, int(bool(los)), -1)
    _check(_lib().amr_render_lod(tree.handle, ctypes.byref(cam), op, model.handle, ctypes.byref(o), _ptr(out),
                                 _ptr(aux), _ptr(tile_levels), _ptr(forced), _ptr(workspace), workspace.numel(),
                                 _ptr(stats), _stream(stream)))


def noalloc_max_bytes() -> int:
    return int(_lib().amr_lod_noalloc_max_bytes())


def render_lod_noalloc(tree: Tree, cam: Camera, op: int, model: LodModel, out, stats, aux=None, field: int = 0,
                       weight: int = 0, los: bool = False, tile_levels=None, forced=None, stream=None):
    """amr_render_lod_noalloc: the LOD render on the library's fixed device
    scratch (no workspace argument, no allocation)."""
    o = RenderOpts(field, weight, int(bool(los)), -1)
    _check(_lib().amr_render_lod_noalloc(tree.handle, ctypes.byref(cam), op, model.handle, ctypes.byref(o), _ptr(out),
                                         _ptr(aux), _ptr(tile_levels), _ptr(forced), _ptr(stats), _stream(stream)))


# ------------------------------------------------------------- drivers

def render_levels(tree: Tree, desc: dict, levels=range(LV0, LV0 + NCLS), op: int = SUM):
    """Plain renders of one camera at each level (device tensors), with the
    library's default walk (the one the tile render also runs)."""
    import torch

    out = []
    for L in levels:
        cam = set_camera(dict(desc, max_level=L), tree)
        img = torch.empty(cam.W * cam.H, dtype=torch.float32, device="cuda")
        render(tree, cam, op, img)
        out.append(img)
    return out


def make_samples(tree: Tree, desc: dict, tol: float = 1e-3, coarse_level: int = 7):
    """(features [tiles, 32] int16, labels [tiles] int8) for one camera."""
    import torch

    imgs = render_levels(tree, desc)
    W, H = desc["W"], desc["H"]
    nt = tiles(W, H)
    lab = torch.empty(nt, dtype=torch.int8, device="cuda")
    labels(imgs, W, H, tol, lab)
    feat = torch.empty((nt, NIN), dtype=torch.int16, device="cuda")
    cam = set_camera(dict(desc, max_level=LV0 + NCLS - 1), tree)
    features(tree, cam, feat, coarse_level)
    return feat, lab


def train(model: LodModel, feat, lab, steps: int = 2000, batch: int = 8192, lr: float = 2e-3, lam: float = 4.0,
          seed: int = 0, log=None):
    """Minibatch Adam on device-resident samples; returns the loss curve."""
    import torch

    n = int(feat.shape[0])
    g = torch.Generator(device="cpu").manual_seed(seed)
    logits = torch.empty((batch, NOUT), dtype=torch.float32, device="cuda")
    dlog = torch.empty_like(logits)
    acts = torch.empty((3, batch, NHID), dtype=torch.int16, device="cuda")
    dz = torch.empty((3 * batch * NHID + batch * NOUT,), dtype=torch.int16, device="cuda")
    lsum = torch.zeros(1, dtype=torch.float32, device="cuda")
    curve = []
    perm = torch.randperm(n, generator=g).cuda()
    pos = 0
    for it in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, generator=g).cuda()
            pos = 0
        idx = perm[pos:pos + min(batch, n)]
        pos += batch
        m = int(idx.numel())
        xb = feat[idx].contiguous()
        yb = lab[idx].contiguous()
        lsum.zero_()
        model.forward(xb, m, logits, acts)
        loss(logits, yb, m, lam, 1.0 / m, dlog, lsum)
        model.backward(xb, acts, dlog, m, dz)
        model.adam_step(lr)
        if it % 50 == 0 or it == steps - 1:
            curve.append((it, float(lsum.item()) / m))
            if log:
                log(f"step {it}: loss {curve[-1][1]:.4f}")
    return curve


def evaluate(tree: Tree, desc: dict, model: Optional[LodModel], reps: int = 5, op: int = SUM) -> Dict:
    """Per-pixel error of the LOD render against full depth and the time of
    both: after one warm-up call of each, the mean over `reps` calls issued
    back to back (HIP events around the run, as in a render loop, so host
    launch gaps are hidden alike); the LOD time includes features, network,
    plan, render and audit."""
    import torch

    cam = set_camera(desc, tree)
    n = cam.W * cam.H
    full = torch.empty(n, dtype=torch.float32, device="cuda")
    out = torch.empty_like(full)
    ws = torch.empty(workspace_bytes(cam.W, cam.H), dtype=torch.uint8, device="cuda")
    st = torch.zeros(8, dtype=torch.int64, device="cuda")
    lev = torch.empty(tiles(cam.W, cam.H), dtype=torch.int8, device="cuda")

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    plain = lambda: render(tree, cam, op, full)
    lod_fn = lambda: render_lod(tree, cam, op, model, out, ws, st, tile_levels=lev)
    plain()
    if model is not None:
        lod_fn()
    torch.cuda.synchronize()
    t_plain = timed(plain)
    res = dict(t_plain_ms=t_plain)
    if model is not None:
        t_lod = timed(lod_fn)
        f = full.double()
        d = (out.double() - f).abs()
        rel = torch.where(f != 0, d / f.abs().clamp_min(1e-300), torch.where(d == 0, 0.0, float("inf")))
        s = st.cpu().numpy()
        res.update(t_lod_ms=t_lod, speedup=t_plain / t_lod, max_rel=float(rel.max()),
                   p999_rel=float(torch.quantile(rel[::7].float(), 0.999)), frac_bad=float((rel > 1e-3).double().mean()),
                   fallback_frac=float(s[1]) / max(1, s[0]), audited=int(s[2]), overwritten=int(s[3]),
                   mean_level=float(s[4]) / max(1, s[0]), rewalked_packets=int(s[5]))
    return res
