"""Benchmark: ray-casting throughput on the galaxy-disk workload.

One step = the whole render path over one batch: the three 2048^2
perspective cameras (inclinations 0, 45, 90 degrees) of the ~20.5M-leaf disk
(levels 7..16), each rendered twice -- the line-of-sight column integral of
density (sum) and the density-weighted mean line-of-sight velocity (wmean).
Inputs are resident in HBM before timing; tree build, camera set-up and the
segment counts used for byte accounting are outside the timed region.

Prints ONE JSON line on stdout.  Timings are taken with HIP events on the
stream the library launches on (torch's current stream).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
B_SEG = {"sum": 8, "wmean": 20}   # value(s) + own first-child word per ray-cell segment
B_PIX = {"sum": 4, "wmean": 8}    # output plane(s) per ray
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_disk.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1210_8014_amd", "csrc", f) for f in ("render.hip", "batch.hip", "traverse.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_name(variant: int, op: str) -> str:
    """Name of the render kernel a variant launches for op (as rocprofv3 shows it)."""
    import paper_1210_8014_amd as amr

    name = amr.variants()[variant if variant >= 0 else amr.default_variant()]
    code = {"sum": 0, "max": 1, "wmean": 2}[op]
    if "split" in name:
        remap = 2 if name.endswith("center") else (1 if name.endswith("xcdband") else 0)
        # both ops of this workload have the common field layout: the specialised walk
        return "k_render_split<%d, %s, %d, true>" % (code, name.split("split")[1].split("_")[0], remap)
    return "k_render<%d, ...> (%s)" % (code, name)


def lod_leg(seed: int = 100):
    """Learned-LOD speed-up over the default plain render with the committed
    model on a held-out disk (seed 100, not among the training seeds 0-99), the
    three bench cameras, op sum: times include features, network, plan, tile
    render and the 2% audit."""
    import numpy as np

    import amrgen
    import paper_1210_8014_amd as amr
    from paper_1210_8014_amd import lod

    if not os.path.exists(lod.MODEL_PATH):
        return None
    t0 = time.time()
    tree = amr.Tree(amrgen.disk(seed=seed))
    model = lod.LodModel(path=lod.MODEL_PATH)
    rows = [lod.evaluate(tree, d, model, reps=10) for d in amrgen.disk_cameras(2048, 2048, max_level=16)]
    tree.close()
    sp = np.array([r["speedup"] for r in rows])
    res = {"speedup_geomean": float(np.exp(np.log(sp).mean())), "speedup_per_camera": [round(float(x), 4) for x in sp],
           "max_frac_pixels_over_1e-3": float(max(r["frac_bad"] for r in rows)),
           "max_rel_err": float(max(r["max_rel"] for r in rows)),
           "mean_level": float(np.mean([r["mean_level"] for r in rows])),
           "scene": "disk seed %d (held out), 2048x2048, inclinations 0/45/90 deg, sum" % seed}
    log(f"lod: speed-up {res['speedup_geomean']:.3f} ({time.time() - t0:.1f} s)")
    return res


def batch_kernel_name(config: str, op: str) -> str:
    """Name of the kernel a batch launch shape runs for op on this workload
    (as rocprofv3 shows it).  Both ops here have the common field layout
    (sum of density; line-of-sight velocity weighted by density on the
    interleaved records), so the grid shapes run their specialised walk."""
    code = {"sum": 0, "max": 1, "wmean": 2}[op]
    if "grid" in config:
        return "k_batch_grid<%d, %d, true>" % (code, 2 if "split2" in config else 1)
    return "k_batch<%d, ...> (%s)" % (code, config)


def cpu_baseline(leaves, cams_desc, seconds_target: float = 15.0):
    """The oracle, as is, on a seeded sample of the same rays."""
    import numpy as np

    import oracle

    ot = oracle.Tree(leaves)
    nthreads = os.cpu_count() or 1
    rng = np.random.default_rng(7)
    n = cams_desc[0]["W"] * cams_desc[0]["H"]
    per_cam = n // 2
    rays_done = 0
    t_total = 0.0
    for d in cams_desc:
        cam = ot.camera(d)
        rays = np.sort(rng.choice(n, per_cam, replace=False))
        t0 = time.perf_counter()
        ot.render(cam, oracle.SUM, rays=rays, nthreads=nthreads)
        ot.render(cam, oracle.WMEAN, field=1, weight=0, los=True, rays=rays, nthreads=nthreads)
        t_total += time.perf_counter() - t0
        rays_done += 2 * per_cam
        if t_total > seconds_target:
            break
    ot.close()
    return dict(value=rays_done / t_total / 1e6, unit="Mrays/s", cores=nthreads, kind="oracle",
                sample=f"half the pixels of each 2048^2 camera (seeded), sum and wmean each, cameras in turn "
                       f"until >= {seconds_target:.0f} s; "
                       f"{rays_done} ray renders in {t_total:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["disk", "batch"], default="disk",
                    help="disk: the 3-camera galaxy disk (default); batch: 8 snapshots x 64 orbit cameras "
                         "in one persistent launch, compared with per-image launches")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, run one 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--no-lod", action="store_true", help="skip the learned-LOD leg")
    ap.add_argument("--per-image", action="store_true",
                    help="render the step with six single-image launches instead of two batch launches")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build renders on one GPU only; multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import amrgen
    import paper_1210_8014_amd as amr

    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args)
    t0 = time.time()
    leaves = amrgen.scene("disk")
    log(f"scene: {leaves.n} leaves, lmax {leaves.lmax} ({time.time() - t0:.1f} s)")
    tree = amr.Tree(leaves)
    log(f"tree: {tree.ncells} cells ({time.time() - t0:.1f} s)")
    descs = amrgen.disk_cameras(2048, 2048, max_level=16)
    cams = [amr.set_camera(d, tree) for d in descs]
    W, H = 2048, 2048
    npix = W * H
    outs = [torch.empty(npix, dtype=torch.float32, device="cuda") for _ in range(len(cams) * 2)]
    auxs = [torch.empty(npix, dtype=torch.float32, device="cuda") for _ in cams]

    # exact segment counts (untimed) for the algorithmic byte count
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    segs = []
    for c in cams:
        amr.count_segments(tree, c, tot)
        torch.cuda.synchronize()
        segs.append(int(tot.item()))
    log(f"segments per camera: {segs}")

    stream = torch.cuda.current_stream()
    ev = {"sum": [], "wmean": []}
    batched = not args.per_image
    plans = {}
    if batched:
        # one plan per op over the three cameras, launch shape chosen by the tuner (untimed)
        pairs = [(0, k) for k in range(len(cams))]
        plans["sum"] = amr.Batch([tree], cams, pairs, amr.SUM, [outs[2 * k] for k in range(len(cams))], field=0)
        plans["wmean"] = amr.Batch([tree], cams, pairs, amr.WMEAN, [outs[2 * k + 1] for k in range(len(cams))],
                                   auxs, field=1, weight=0, los=True)
        for op, B in plans.items():
            best, times = B.tune(reps=2)
            log(f"{op} batch configurations (ms): " + ", ".join(f"{k} {v:.2f}" for k, v in times.items()) +
                f"; chosen {amr.batch_configs()[best]}")

    def batched_step(record: bool):
        for op in ("sum", "wmean"):
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            plans[op].run()
            if record:
                e1.record(stream)
                ev[op].append((-1, e0, e1))

    def step(record: bool):
        if batched:
            return batched_step(record)
        for k, c in enumerate(cams):
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            amr.render(tree, c, amr.SUM, outs[2 * k], field=0, variant=args.variant)
            if record:
                e1.record(stream)
                ev["sum"].append((k, e0, e1))
                e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e2.record(stream)
            amr.render(tree, c, amr.WMEAN, outs[2 * k + 1], auxs[k], field=1, weight=0, los=True,
                       variant=args.variant)
            if record:
                e3.record(stream)
                ev["wmean"].append((k, e2, e3))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start

    ms_per_step = 1e3 * t_wall / args.steps
    rays_per_step = 2 * len(cams) * npix
    value = rays_per_step / (t_wall / args.steps) / 1e6

    per_image_ms = None
    if batched:
        # reference: the same step as six single-image launches of the default variant
        def singles():
            for k, c in enumerate(cams):
                amr.render(tree, c, amr.SUM, outs[2 * k], field=0)
                amr.render(tree, c, amr.WMEAN, outs[2 * k + 1], auxs[k], field=1, weight=0, los=True)
        singles()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            singles()
        torch.cuda.synchronize()
        per_image_ms = 1e3 * (time.perf_counter() - t1) / 5

    def launch_bytes(op, k):
        if k < 0:  # one batch launch covers all cameras
            return sum(segs[q] * B_SEG[op] + npix * B_PIX[op] for q in range(len(cams)))
        return segs[k] * B_SEG[op] + npix * B_PIX[op]

    kern = {}
    for op in ("sum", "wmean"):
        durs = [e0.elapsed_time(e1) * 1e-3 for _, e0, e1 in ev[op]]
        byts = [launch_bytes(op, k) for k, _, _ in ev[op]]
        avg_t = sum(durs) / len(durs)
        avg_b = sum(byts) / len(byts)
        ipl = len(cams) if batched else 1  # images per launch
        kern[op] = dict(avg_ms=avg_t * 1e3, alg_bytes=avg_b, gbs=avg_b / avg_t / 1e9, total_s=sum(durs),
                        mrays=ipl * npix / avg_t / 1e6, seg_per_s=ipl * (sum(segs) / len(segs)) / avg_t)
        log(f"{op}: avg {avg_t * 1e3:.3f} ms/launch, {kern[op]['gbs']:.0f} GB/s algorithmic, "
            f"{kern[op]['mrays']:.0f} Mrays/s, {kern[op]['seg_per_s'] / 1e9:.1f} Gseg/s")
    dom = max(kern, key=lambda k: kern[k]["total_s"])
    alg_total = sum(kern[op]["alg_bytes"] for op in kern) * (1 if batched else len(cams))

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        kname = (batch_kernel_name(amr.batch_configs()[plans[dom].config], dom) if batched
                 else kernel_name(args.variant, dom))
        if tr.get("kernel_hash") == kernel_hash() and kname in tr.get("per_launch_bytes", {}):
            traffic = tr["per_launch_bytes"][kname]

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    lod_res = None
    if not args.no_lod:
        lod_res = lod_leg()

    cpu = None
    if not args.no_cpu_baseline:
        t1 = time.time()
        cpu = cpu_baseline(leaves, descs)
        log(f"cpu baseline: {cpu['value']:.3f} Mrays/s on {cpu['cores']} threads ({time.time() - t1:.1f} s)")

    line = {
        "metric": "Mrays/s + HBM GB/s; learned-LOD vs plain speedup at <=1e-3 rel err",
        "value": value,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "galaxy disk (seed 0, %d leaves, levels 7-16, density + velocity), 3 perspective "
                        "cameras 2048x2048 at inclinations 0/45/90 deg, ops sum(rho) and wmean(v_los; w=rho)"
                        % leaves.n,
            "leaves": int(leaves.n),
            "cells": int(tree.ncells),
            "rays_per_step": rays_per_step,
            "segments_per_camera": segs,
            "algorithmic_GB_per_step": alg_total / 1e9,
            "algorithmic_GBs": alg_total / (t_wall / args.steps) / 1e9,
            "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k, v in kern.items()},
            "launches": ("two batch launches per step (sum, wmean), three images each" if batched
                         else "six single-image launches per step"),
            "launch_shape": ({op: amr.batch_configs()[B.config] for op, B in plans.items()} if batched
                             else amr.variants()[args.variant if args.variant >= 0 else amr.default_variant()]),
            "single_image_ms_per_step": per_image_ms,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": (batch_kernel_name(amr.batch_configs()[plans[dom].config], dom) if batched
                       else kernel_name(args.variant, dom)),
            "achieved": kern[dom]["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": kern[dom]["gbs"] / HBM_PEAK_GBS,
            "traffic": traffic,
            # the algorithmic basis counts every segment's gather as HBM traffic; the
            # measured DRAM rate (traffic / launch time) shows how much the caches absorb
            "dram_GBs": (traffic / (kern[dom]["avg_ms"] * 1e-3) / 1e9) if traffic else None,
        },
        "cpu_baseline": cpu,
        "lod": lod_res,
    }
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """8 disk snapshots (seeds 0-7, 5-25M leaves) x 64 orbit cameras with
    image sides log-uniform in [512, 2048]: the 512 images in one
    graph-captured persistent launch vs 512 single-image launches."""
    import torch

    import amrgen
    import paper_1210_8014_amd as amr

    t0 = time.time()
    trees = []
    nleaves = []
    for sd in range(8):
        lv = amrgen.scene("batch", seed=sd)
        nleaves.append(int(lv.n))
        trees.append(amr.Tree(lv))
        del lv
        log(f"snapshot {sd}: {nleaves[-1]} leaves, {trees[-1].ncells} cells ({time.time() - t0:.1f} s)")
    descs = amrgen.orbit_cameras(64, seed=0, side_lo=512, side_hi=2048, multiple=16, max_level=16)
    cams = [amr.set_camera(d) for d in descs]
    pairs = [(t, c) for t in range(8) for c in range(64)]
    outs = [torch.empty(cams[c].W * cams[c].H, dtype=torch.float32, device="cuda") for _, c in pairs]
    rays = sum(cams[c].W * cams[c].H for _, c in pairs)
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    segs = 0
    for t, c in pairs:
        amr.count_segments(trees[t], cams[c], tot)
        torch.cuda.synchronize()
        segs += int(tot.item())
    log(f"{len(pairs)} images, {rays} rays, {segs} segments ({time.time() - t0:.1f} s)")
    B = amr.Batch(trees, cams, pairs, amr.SUM, outs)
    best, times = B.tune(reps=1)
    log(f"batch configurations (ms): {times}; chosen {amr.batch_configs()[best]}")
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        res = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res.append(e0.elapsed_time(e1) * 1e-3)
        return res

    for _ in range(args.warmup):
        B.run()
    t_batch = timed(B.run, args.steps)

    def per_image():
        for k, (t, c) in enumerate(pairs):
            amr.render(trees[t], cams[c], amr.SUM, outs[k])

    per_image()
    t_single = timed(per_image, max(1, args.steps // 4))
    tb, ts = sum(t_batch) / len(t_batch), sum(t_single) / len(t_single)
    alg = segs * B_SEG["sum"] + rays * B_PIX["sum"]
    line = {
        "metric": "Mrays/s + HBM GB/s; learned-LOD vs plain speedup at <=1e-3 rel err",
        "value": rays / tb / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tb * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched: 8 disk snapshots (seeds 0-7, %d-%d leaves) x 64 orbit cameras, sides "
                        "log-uniform in [512, 2048], op sum(rho), one graph launch (shape chosen by the tuner)"
                        % (min(nleaves), max(nleaves)),
            "images": len(pairs),
            "rays_per_step": rays,
            "segments_per_step": segs,
            "batch_config": amr.batch_configs()[best],
            "per_image_launches_ms": ts * 1e3,
            "batch_speedup_vs_per_image": ts / tb,
            "algorithmic_GBs": alg / tb / 1e9,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": batch_kernel_name(amr.batch_configs()[best], "sum"),
            "achieved": alg / tb / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": alg / tb / 1e9 / HBM_PEAK_GBS,
            "traffic": None,
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
