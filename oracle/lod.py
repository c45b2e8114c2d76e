"""Oracle for the learned level of detail (TEST INFRASTRUCTURE ONLY).

Plain NumPy, fp64 unless stated:
  * bf16 round-to-nearest-even emulation;
  * tile features from the C oracle's per-ray probe statistics;
  * the 32 -> 64 -> 64 -> 64 -> 16 ReLU network forward and backward with
    the same bf16 roundings the GPU applies (weights, inputs, hidden
    activations, back-propagated pre-activation gradients);
  * the loss over the 16 level classes 1..16 (cross-entropy + lambda *
    probability of too-shallow levels)
    and its analytic gradient, pinned by central finite differences;
  * per-tile labels from renders at every level, and the plan (quantile
    level, confidence fallback);
  * the Adam update (Kingma and Ba: moment estimates with bias correction),
    pinned by its closed forms for constant and alternating gradients.
Parameter layout: W1[32][64], b1[64], W2[64][64], b2, W3[64][64], b3,
W4[64][16], b4[16].
"""
from __future__ import annotations

import math

import numpy as np

IN, HID, OUT, CLS, LV0, TILE = 32, 64, 16, 16, 1, 16
BINS, BIN0 = 10, 7  # subtree-depth histogram of the probe features: levels 7..16
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, HID)),
          ("b3", (HID,)), ("W4", (HID, OUT)), ("b4", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[k:k + n], np.float64).reshape(shp)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest even); returns float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(x):
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def from_bits(b):
    return (np.asarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(params, X, emulate=True):
    """X: [n, 32] (already bf16 values).  Returns logits [n, 16] and the
    hidden activations [A1, A2, A3]."""
    p = unpack(params)
    r = bf16 if emulate else (lambda v: np.asarray(v, np.float64))
    h = np.asarray(X, np.float64)
    acts = []
    for L in (1, 2, 3):
        z = h @ r(p[f"W{L}"]) + p[f"b{L}"]
        h = r(np.maximum(z, 0.0))
        acts.append(h)
    logits = h @ r(p["W4"]) + p["b4"]
    return logits, acts


def softmax10(logits):
    z = np.asarray(logits, np.float64)[:, :CLS]
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(logits, labels, lam):
    """Per-sample loss -log p_y + lam * sum_{c<y} p_c and d loss / d logits."""
    p = softmax10(logits)
    n = p.shape[0]
    y = np.asarray(labels, np.int64)
    idx = np.arange(n)
    below = np.arange(CLS)[None, :] < y[:, None]
    S = (p * below).sum(axis=1)
    loss = -np.log(np.maximum(p[idx, y], 1e-300)) + lam * S
    g = p.copy()
    g[idx, y] -= 1.0
    g += lam * p * (below.astype(np.float64) - S[:, None])
    d = np.zeros((n, OUT))
    d[:, :CLS] = g
    return loss, d


def backward(params, X, acts, dlogits, emulate=True):
    """Parameter gradients of sum over samples; with emulate the
    back-propagated pre-activation gradients are rounded to bf16 as on the
    GPU."""
    p = unpack(params)
    r = bf16 if emulate else (lambda v: np.asarray(v, np.float64))
    dz = r(dlogits)
    g = {"W4": acts[2].T @ dz, "b4": dz.sum(axis=0)}
    for L in (3, 2, 1):
        da = dz @ r(p[f"W{L + 1}"]).T
        dz = r(da * (acts[L - 1] > 0))
        xin = X if L == 1 else acts[L - 2]
        g[f"W{L}"] = np.asarray(xin, np.float64).T @ dz
        g[f"b{L}"] = dz.sum(axis=0)
    return pack(g)


def total_loss(params, X, labels, lam, emulate=False):
    logits, _ = forward(params, X, emulate)
    return loss_and_grad(logits, labels, lam)[0].sum()


def tile_features(stats, probe_col_max, foot_log2, tiles):
    """Features per tile from the C oracle's probe statistics.
    stats: [tiles * 16, 16] (16 probes per tile, tile-major)."""
    f = np.zeros((tiles, IN))
    s = stats.reshape(tiles, 16, 16)
    col = s[:, :, 0]
    mean_col = col.sum(axis=1) / 16.0
    L = s[:, :, 1].sum(axis=1)
    slg = s[:, :, 2].sum(axis=1)
    slg2 = s[:, :, 3].sum(axis=1)
    hit = s[:, :, 4].sum(axis=1)
    hist = s[:, :, 5:15].sum(axis=1)
    segs = s[:, :, 15].sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        mlg = np.where(L > 0, slg / np.where(L > 0, L, 1), 0.0)
        vlg = np.where(L > 0, np.maximum(slg2 / np.where(L > 0, L, 1) - mlg * mlg, 0.0), 0.0)
        f[:, 0] = np.log10(1e-12 + mean_col)
        f[:, 1] = np.log10(1e-12 + col.max(axis=1)) - np.log10(1e-12 + mean_col)
        f[:, 2:12] = np.where(L[:, None] > 0, hist / np.where(L > 0, L, 1)[:, None], 0.0)
    f[:, 12] = mlg
    f[:, 13] = vlg
    f[:, 14] = foot_log2
    f[:, 15] = hit / 16.0
    f[:, 16] = segs / (16.0 * 64.0)
    return f


def probe_pixels(W, H):
    """Pixel ids of the 16 probe rays of every tile (tile-major)."""
    tx, ty = -(-W // TILE), -(-H // TILE)
    ids = []
    for t in range(tx * ty):
        y0, x0 = divmod(t, tx)
        for p in range(16):
            i = min(x0 * TILE + (p & 3) * 4 + 2, W - 1)
            j = min(y0 * TILE + (p >> 2) * 4 + 2, H - 1)
            ids.append(j * W + i)
    return np.array(ids, np.int64), tx * ty


def footprint_log2(cam, coarse_level):
    """log2(pixel footprint / coarse cell side) from the integer camera."""
    V = np.array(list(cam.V), np.float64)
    F = np.array(list(cam.F), np.float64)
    foot = 2.0 * math.sqrt((V * V).sum() / (F * F).sum()) if cam.kind == 0 else 2.0 * math.sqrt((V * V).sum()) * 2.0 ** -28
    return math.log2(foot * 2.0 ** coarse_level + 1e-30)


def labels_from_renders(imgs, W, H, tol):
    """imgs: 16 images (levels 1..16) as [H*W] arrays; first level whose
    image is within tol of the last at every pixel of the tile."""
    tx, ty = -(-W // TILE), -(-H // TILE)
    ref = np.asarray(imgs[-1], np.float64).reshape(H, W)
    lab = np.full(tx * ty, CLS - 1, np.int64)
    for t in range(tx * ty):
        y0, x0 = divmod(t, tx)
        sl = (slice(y0 * TILE, min(H, y0 * TILE + TILE)), slice(x0 * TILE, min(W, x0 * TILE + TILE)))
        r = ref[sl]
        for c in range(CLS - 1):
            x = np.asarray(imgs[c], np.float64).reshape(H, W)[sl]
            d = np.abs(x - r)
            e = np.where(r != 0, d / np.where(r != 0, np.abs(r), 1), np.where(d == 0, 0.0, np.inf))
            if e.max() <= tol:
                lab[t] = c
                break
    return lab


def plan(logits, q, conf_thresh, full_level):
    p = softmax10(logits)
    cdf = np.cumsum(p, axis=1)
    cls = np.argmax(cdf >= q, axis=1)
    cls = np.where((cdf >= q).any(axis=1), cls, CLS - 1)
    lev = LV0 + cls
    fb = (p.max(axis=1) < conf_thresh) | (conf_thresh >= 1.0)
    lev = np.where(fb, full_level, lev)
    return np.minimum(lev, full_level), fb


def adam(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step, step number t >= 1: returns (params, m, v) after it.
    m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2;
    params <- params - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)."""
    g = np.asarray(grads, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
