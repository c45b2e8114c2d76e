"""Oracle for the adaptive Gaussian post-filter (TEST INFRASTRUCTURE ONLY).

The paper smooths the ray-cast image with a Gaussian whose size follows the
local resolution of the image, so that regions drawn from coarse cells lose
their blocky look (Sec. 2.2).  It gives no formula; the reading implemented
here (and in the library) is:

  sigma(p) = kappa * r(p) pixels, r(p) the local resolution of pixel p (the
  chord-weighted mean cell side in pixels, oracle.Tree.resolution);

  a ladder of Gaussians sigma_k = SIGMA0 * 2^(k/2), k = 0..NLEVELS-1, each the
  2-D Gaussian of standard deviation sigma_k truncated to the square window
  |dx|, |dy| <= R_k = ceil(3 sigma_k) and normalised over the window's pixels
  inside the image:
      B_k(p) = sum_q g_k(q - p) I(q) / sum_q g_k(q - p),
      g_k(dx, dy) = exp(-(dx^2 + dy^2) / (2 sigma_k^2));

  the output interpolates between the two ladder levels around sigma(p),
  linearly in log2 sigma (in sigma below the first level, from the image
  itself at sigma = 0):
      sigma <= 0              -> I(p)
      0 < sigma < SIGMA0      -> (1 - a) I(p) + a B_0(p),  a = sigma / SIGMA0
      u = 2 log2(sigma / SIGMA0), k = floor(u), a = u - k:
      k < NLEVELS - 1         -> (1 - a) B_k(p) + a B_(k+1)(p)
      otherwise               -> B_(NLEVELS-1)(p).

Everything here is fp64 and evaluated by direct 2-D sums, pixel by pixel.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

SIGMA0 = 0.5
NLEVELS = 11  # sigma up to 16 pixels


def sigma_level(k: int) -> float:
    return SIGMA0 * 2.0 ** (k / 2.0)


def radius(k: int) -> int:
    return int(math.ceil(3.0 * sigma_level(k)))


def level_blur_at(img: np.ndarray, x: int, y: int, k: int) -> float:
    """B_k at pixel (x, y) of img [H, W]: direct 2-D sum over the window."""
    H, W = img.shape
    R = radius(k)
    s = sigma_level(k)
    x0, x1, y0, y1 = max(0, x - R), min(W - 1, x + R), max(0, y - R), min(H - 1, y + R)
    dx = np.arange(x0, x1 + 1) - x
    dy = np.arange(y0, y1 + 1) - y
    g = np.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2.0 * s * s))
    win = np.asarray(img[y0:y1 + 1, x0:x1 + 1], np.float64)
    return float((g * win).sum() / g.sum())


def blend(sigma: float):
    """(k_lo, k_hi, a): the output is (1 - a) B_lo + a B_hi, where level -1
    is the image itself."""
    if not sigma > 0.0:
        return -1, -1, 0.0
    if sigma < SIGMA0:
        return -1, 0, sigma / SIGMA0
    u = 2.0 * math.log2(sigma / SIGMA0)
    k = int(math.floor(u))
    if k >= NLEVELS - 1:
        return NLEVELS - 1, NLEVELS - 1, 0.0
    return k, k + 1, u - k


def adaptive_blur(img: np.ndarray, res: np.ndarray, kappa: float, pixels: Optional[np.ndarray] = None):
    """Filtered values at the given flat pixel indices (all by default) of
    img [H, W] with the resolution plane res [H, W]."""
    H, W = img.shape
    img = np.asarray(img, np.float64)
    res = np.asarray(res, np.float64)
    pix = np.arange(H * W) if pixels is None else np.asarray(pixels, np.int64)
    out = np.zeros(pix.size)
    for n, p in enumerate(pix):
        y, x = divmod(int(p), W)
        lo, hi, a = blend(kappa * res[y, x])
        b_lo = img[y, x] if lo < 0 else level_blur_at(img, x, y, lo)
        b_hi = img[y, x] if hi < 0 else (b_lo if hi == lo else level_blur_at(img, x, y, hi))
        out[n] = (1.0 - a) * b_lo + a * b_hi
    return out


def adaptive_blur_terms(img: np.ndarray, res: np.ndarray, kappa: float, pixels: np.ndarray):
    """(values, spread) at the given pixels: the filtered value and the
    spread (max - min) of the image value and the ladder levels from one
    below to one above the blended pair (the scale on which an error in
    sigma, or the choice of pair at a level boundary, moves the result)."""
    H, W = img.shape
    img = np.asarray(img, np.float64)
    vals = adaptive_blur(img, res, kappa, pixels)
    spread = np.zeros(len(pixels))
    for n, p in enumerate(np.asarray(pixels, np.int64)):
        y, x = divmod(int(p), W)
        lo, hi, _ = blend(kappa * float(res[y, x]))
        ks = range(max(0, lo - 1), min(NLEVELS - 1, max(hi, 0) + 1) + 1)
        b = [img[y, x]] + [level_blur_at(img, x, y, k) for k in ks]
        spread[n] = max(b) - min(b)
    return vals, spread
