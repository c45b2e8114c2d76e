"""Calibrate the refinement thresholds of the synthetic scenes and freeze them
in ``configs.json``.

Leaf count is monotone (decreasing) in the threshold, close to a power law,
so a secant step in log-log space converges in a handful of generator runs;
a bracketing bisection guards it.  Disk thresholds are calibrated on the disk
alone (no cores); the cores are then added by the generator, which adds well
under 1% of the leaves.

Usage:  python -m amrgen.calibrate [--only tiny,disk,deepzoom,batch]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

from . import BLOBS, DISK, _CONFIGS, build, generate


def _solve(count_fn, target, x0, rel_tol=0.02, max_iter=30):
    """Find threshold x with count_fn(x) within rel_tol of target."""
    lo = hi = None  # lo: count > target, hi: count < target (in x)
    x = x0
    best = None
    lx_prev = lc_prev = None
    for _ in range(max_iter):
        c = count_fn(x)
        if best is None or abs(c - target) < abs(best[1] - target):
            best = (x, c)
        if abs(c - target) <= rel_tol * target:
            return x, c
        if c > target:
            lo = x if lo is None or x > lo else lo
        else:
            hi = x if hi is None or x < hi else hi
        lx, lc = math.log(x), math.log(max(c, 1))
        if lx_prev is not None and lc != lc_prev:
            slope = (lc - lc_prev) / (lx - lx_prev)
            nx = lx + (math.log(target) - lc) / slope if slope < 0 else None
        else:
            nx = lx + (0.7 if c > target else -0.7)
        if nx is not None and lo is not None and hi is not None:
            if not (math.log(lo) < nx < math.log(hi)):
                nx = 0.5 * (math.log(lo) + math.log(hi))
        elif nx is None:
            nx = lx + (0.7 if c > target else -0.7)
        lx_prev, lc_prev = lx, lc
        x = math.exp(nx)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="tiny,disk,deepzoom,batch")
    args = ap.parse_args()
    build()
    cfg = {}
    if os.path.exists(_CONFIGS):
        with open(_CONFIGS) as f:
            cfg = json.load(f)
    only = set(args.only.split(","))

    def log(*a):
        print(*a, flush=True)

    if "tiny" in only:
        x, c = _solve(lambda t: generate(BLOBS, 0, 3, 6, t, False, False, count_only=True)[0], 40_000, 0.005)
        cfg["tiny"] = dict(kind="blobs", seed=0, levelmin=3, lmax=6, tau=x, leaves_seed0=c)
        log("tiny", x, c)
    if "disk" in only:
        fn = lambda m: generate(DISK, 0, 7, 16, m, False, False, count_only=True)[0]
        x, c = _solve(fn, 20_000_000, 6.3e-6)
        n, lm = generate(DISK, 0, 7, 16, x, True, False, count_only=True)
        cfg["disk"] = dict(kind="disk", seed=0, levelmin=7, lmax=16, m_thr=x, velocity=True,
                           leaves_seed0_no_cores=c, leaves_seed0=n, lmax_seed0=lm)
        log("disk", x, c, n, lm)
    if "deepzoom" in only:
        t0 = time.time()
        fn = lambda m: generate(DISK, 0, 7, 22, m, False, False, count_only=True)[0]
        x, c = _solve(fn, 200_000_000, 5.8e-7)
        n, lm = generate(DISK, 0, 7, 22, x, True, False, count_only=True)
        cfg["deepzoom"] = dict(kind="disk", seed=0, levelmin=7, lmax=22, m_thr=x, velocity=False,
                               leaves_seed0_no_cores=c, leaves_seed0=n, lmax_seed0=lm)
        log("deepzoom", x, c, n, lm, time.time() - t0)
    if "batch" in only:
        by_seed = {}
        counts = {}
        base = cfg.get("disk", {}).get("m_thr", 6.3e-6)
        for s in range(8):
            target = 5_000_000 + s * 20_000_000 / 7.0
            fn = lambda m, s=s: generate(DISK, s, 7, 16, m, False, False, count_only=True)[0]
            x, c = _solve(fn, target, base * (20e6 / target) ** 1.2)
            by_seed[str(s)] = x
            counts[str(s)] = generate(DISK, s, 7, 16, x, True, False, count_only=True)[0]
            log("batch", s, x, c, counts[str(s)])
        cfg["batch"] = dict(kind="disk", levelmin=7, lmax=16, m_thr=by_seed["0"], m_thr_by_seed=by_seed,
                            leaves_by_seed=counts, velocity=False, seeds=list(range(8)))
    with open(_CONFIGS, "w") as f:
        json.dump(cfg, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
