"""Exact reference computations used to pin the oracle (tests only).

* ``brute_segments``: the plain definition of the cells on a ray -- every
  cell of the truncated tree is slab-tested against the ray with exact
  ``Fraction`` arithmetic; cells met over a positive parameter length are
  kept and sorted by entry parameter.
* ``grid_dda``: the textbook grid traversal of Amanatides and Woo (1987) on a
  uniform 2^l grid, in exact arithmetic, stepping every tied axis at once so
  zero-length cells are skipped.

Positions are integers in units of 2^-28 of the unit box; cells are
half-open boxes [a, b).
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Iterable, List, Tuple

FIX = 28


def truncated_cells(level, ix, iy, iz, L: int):
    """Leaves of the tree truncated at level L (deduplicated ancestors)."""
    out = set()
    for l, x, y, z in zip(level, ix, iy, iz):
        l, x, y, z = int(l), int(x), int(y), int(z)
        if l > L:
            s = l - L
            out.add((L, x >> s, y >> s, z >> s))
        else:
            out.add((l, x, y, z))
    return sorted(out)


def slab(cell, o, d):
    """Exact parameter interval [t0, t1) of the ray inside the cell, t >= 0,
    or None when the ray spends no positive length inside it."""
    l, x, y, z = cell
    sh = FIX - l
    t0, t1 = Fraction(0), None
    for k, c in enumerate((x, y, z)):
        lo, hi = c << sh, (c + 1) << sh
        if d[k] == 0:
            if not (lo <= o[k] < hi):
                return None
            continue
        a, b = Fraction(lo - o[k], d[k]), Fraction(hi - o[k], d[k])
        if d[k] < 0:
            a, b = b, a
        t0 = max(t0, a)
        t1 = b if t1 is None else min(t1, b)
    if t1 is None or not t0 < t1:
        return None
    return t0, t1


def brute_segments(cells: Iterable[Tuple[int, int, int, int]], o, d) -> List[Tuple[tuple, Fraction, Fraction]]:
    segs = []
    for c in cells:
        iv = slab(c, o, d)
        if iv is not None:
            segs.append((c, iv[0], iv[1]))
    segs.sort(key=lambda s: s[1])
    return segs


def ray_length_unit(d) -> float:
    """|d| * 2^-28 in box units per unit of ray parameter."""
    return math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * 2.0 ** -FIX


def box_chord(o, d) -> float:
    """Length (box units) of the ray inside the unit box, by one slab test."""
    iv = slab((0, 0, 0, 0), o, d)
    if iv is None:
        return 0.0
    return float(iv[1] - iv[0]) * ray_length_unit(d)


def grid_dda(level: int, o, d):
    """Amanatides-Woo traversal of the uniform 2^level grid, exact.

    Returns [(cell, t0, t1)] with cell = (level, i, j, k)."""
    box = slab((0, 0, 0, 0), o, d)
    if box is None:
        return []
    t, tend = box
    h = 1 << (FIX - level)
    n = 1 << level
    idx, step, tnext, tdelta = [], [], [], []
    for k in range(3):
        p = o[k] + t * d[k]  # exact entry position (Fraction)
        if d[k] > 0:
            c = math.floor(p / h)
            step.append(1)
            tnext.append(Fraction((c + 1) * h - o[k], d[k]))
            tdelta.append(Fraction(h, d[k]))
        elif d[k] < 0:
            c = math.ceil(p / h) - 1  # moving down: the cell just below p
            step.append(-1)
            tnext.append(Fraction(c * h - o[k], d[k]))
            tdelta.append(Fraction(h, -d[k]))
        else:
            c = math.floor(p / h)
            step.append(0)
            tnext.append(None)
            tdelta.append(None)
        idx.append(c)
    out = []
    while True:
        cand = [tnext[k] for k in range(3) if tnext[k] is not None]
        tm = min(cand + [tend])
        if tm > t:
            out.append(((level, idx[0], idx[1], idx[2]), t, tm))
        if tm >= tend:
            break
        for k in range(3):
            if tnext[k] is not None and tnext[k] == tm:
                idx[k] += step[k]
                tnext[k] += tdelta[k]
        if not all(0 <= v < n for v in idx):
            break
        t = tm
    return out
