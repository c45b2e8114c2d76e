"""Train and evaluate the learned level of detail on galaxy-disk renders.

Training data: for every training seed, a ~20M-leaf disk (levels 7..16) and
`--cams` cameras at 100 kpc with inclination U[0, 90] deg and azimuth
U[0, 360) deg; each camera is rendered at every level 1..16, giving one
(features, label) sample per 16 x 16 tile.  The samples stay on the device.
Evaluation: held-out seeds, the inclinations 0/45/90 deg, LOD render vs the
plain full-depth render (time and per-pixel error), for the trained and the
untrained network.

python -m paper_1210_8014_amd.lod_train --train-seeds 0-99 --test-seeds 100-119 \
    --out paper_1210_8014_amd/lod_model.bin --report lod_report.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def _range(s: str):
    a, b = s.split("-") if "-" in s else (s, s)
    return list(range(int(a), int(b) + 1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_dataset(seeds, ncams, size, coarse_level, rng_seed=1234):
    import torch

    import amrgen
    import paper_1210_8014_amd as amr
    from . import lod

    rng = np.random.default_rng(rng_seed)
    feats, labs = [], []
    t0 = time.time()
    for s in seeds:
        T = amr.Tree(amrgen.disk(seed=s))
        for _ in range(ncams):
            desc = amrgen.disk_camera(float(rng.uniform(0, 90)), size, size, max_level=16,
                                      azim_deg=float(rng.uniform(0, 360)))
            f, l = lod.make_samples(T, desc, coarse_level=coarse_level)
            feats.append(f)
            labs.append(l)
        T.close()
        torch.cuda.synchronize()
        log(f"train seed {s}: {sum(int(x.shape[0]) for x in feats)} samples ({time.time() - t0:.0f} s)")
    return torch.cat(feats), torch.cat(labs)


def evaluate_seeds(model, seeds, size, reps=5):
    import amrgen
    import paper_1210_8014_amd as amr
    from . import lod

    rows = []
    for s in seeds:
        T = amr.Tree(amrgen.disk(seed=s))
        for inc in (0.0, 45.0, 90.0):
            r = lod.evaluate(T, amrgen.disk_camera(inc, size, size, max_level=16), model, reps=reps)
            r.update(seed=s, incl=inc)
            rows.append(r)
            log(f"test seed {s} incl {inc}: " + ", ".join(f"{k} {v:.4g}" for k, v in r.items()
                                                           if isinstance(v, float)))
        T.close()
    return rows


def summarize(rows):
    sp = np.array([r["speedup"] for r in rows])
    return dict(images=len(rows), geomean_speedup=float(np.exp(np.log(sp).mean())), min_speedup=float(sp.min()),
                max_rel_err=float(max(r["max_rel"] for r in rows)),
                mean_frac_pixels_over_1e3=float(np.mean([r["frac_bad"] for r in rows])),
                worst_frac_pixels_over_1e3=float(max(r["frac_bad"] for r in rows)),
                mean_fallback=float(np.mean([r["fallback_frac"] for r in rows])),
                mean_level=float(np.mean([r["mean_level"] for r in rows])),
                overwritten_pixels=int(sum(r["overwritten"] for r in rows)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", default="0-99")
    ap.add_argument("--test-seeds", default="100-119")
    ap.add_argument("--cams", type=int, default=8)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lam", type=float, default=4.0)
    ap.add_argument("--quantile", type=float, default=0.99)
    ap.add_argument("--conf", type=float, default=0.5)
    ap.add_argument("--audit", type=float, default=0.02)
    ap.add_argument("--coarse-level", type=int, default=None, help="probe level of the features (default: the config's)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--model", default=None, help="evaluate this saved model instead of training one")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    import torch

    from . import lod

    torch.cuda.set_device(0)
    cfg = dict(lod.default_config(), quantile=args.quantile, conf_thresh=args.conf, audit_frac=args.audit)
    if args.coarse_level is not None:
        cfg["coarse_level"] = args.coarse_level
    untrained = lod.LodModel(cfg, seed=11)
    if args.model:
        model = lod.LodModel(path=args.model)
        if args.coarse_level is None:  # the probe level the model was trained with
            cfg["coarse_level"] = model.config["coarse_level"]
        model.config = cfg
        hist, curve, t_train = np.zeros(16, np.int64), [], 0.0
    else:
        t0 = time.time()
        feat, lab = build_dataset(_range(args.train_seeds), args.cams, args.size, cfg["coarse_level"])
        hist = np.bincount(lab.cpu().numpy().astype(np.int64), minlength=16)
        log(f"dataset: {feat.shape[0]} tiles, label histogram (levels 1..16) {hist.tolist()} ({time.time() - t0:.0f} s)")
        model = lod.LodModel(cfg, seed=11)
        t1 = time.time()
        curve = lod.train(model, feat, lab, steps=args.steps, batch=args.batch, lr=args.lr, lam=args.lam, log=log)
        torch.cuda.synchronize()
        t_train = time.time() - t1
        log(f"trained {args.steps} steps in {t_train:.1f} s")
        del feat, lab
        if args.out:
            model.save(args.out)
    rows = evaluate_seeds(model, _range(args.test_seeds), args.size)
    rows_u = evaluate_seeds(untrained, _range(args.test_seeds)[:2], args.size)
    rep = dict(config=cfg, train_seeds=args.train_seeds, test_seeds=args.test_seeds, cams_per_seed=args.cams,
               image_size=args.size, samples=int(hist.sum()), label_histogram=hist.tolist(), steps=args.steps,
               batch=args.batch, lr=args.lr, lam=args.lam, train_seconds=t_train, loss_curve=curve,
               trained=summarize(rows), untrained=summarize(rows_u), per_image=rows)
    log(json.dumps({k: rep[k] for k in ("trained", "untrained")}, indent=1))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep["trained"]), flush=True)


if __name__ == "__main__":
    main()
