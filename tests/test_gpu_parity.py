"""GPU parity: the HIP library against the oracle on the same seeded inputs
(bars in tests/parity.py).  Run on an MI355X: pytest -m gpu."""
import numpy as np
import pytest

import amrgen
import oracle
from tests import parity
from tests.test_oracle_pins import degenerate_cams, rand_cams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_8014_amd as amr

    amr.lib()


def _R(*a, **k):
    from tests.gpu_render import GpuRenderer

    return GpuRenderer(*a, **k)


def _is_split(v):
    import paper_1210_8014_amd as amr

    return "split" in amr.variants()[v]


def log(*a):
    print(*a, flush=True)


def test_gpu_tiny_full_image_every_variant():
    import paper_1210_8014_amd as amr

    L = amrgen.scene("tiny")
    R = _R(L)
    OT = oracle.Tree(L)
    camd = amrgen.tiny_camera()
    cam, ocam = R.camera(camd), OT.camera(camd)
    ref_s = OT.render(ocam, oracle.SUM)
    ref_m = OT.render(ocam, oracle.MAX)["max"]
    base = None
    for v in range(len(amr.variants())):
        log("tiny variant", v, amr.variants()[v])
        s, _ = R.full(cam, amr.SUM, variant=v)
        m, _ = R.full(cam, amr.MAX, variant=v)
        parity.check_sum(s, ref_s["val"], f"tiny v{v}")
        parity.check_max(m, ref_m, f"tiny v{v}")
        if base is None:
            base, base_m = s, m
        assert np.array_equal(m.view(np.int32), base_m.view(np.int32)), f"variant {v} max not bit-identical"
        if not _is_split(v):
            assert np.array_equal(s.view(np.int32), base.view(np.int32)), f"variant {v} not bit-identical"
    cnt, tot = R.counts(cam)
    parity.check_counts(cnt, ref_s["count"], "tiny")
    assert tot == int(ref_s["count"].sum())
    rays = np.arange(65536)
    offs, cells = R.trace(cam, rays)
    ro, rc, _ = OT.trace(ocam, rays)
    parity.check_trace(offs, cells, ro, rc, "tiny all rays")


@pytest.mark.parametrize("seed", range(2))
def test_gpu_random_trees_and_degenerate_rays(seed):
    rng = np.random.default_rng(seed)
    L = amrgen.random_tree(200 + seed, lmax=5, p_refine=0.45, nfields=4)
    L.fields[1:] -= 5.0
    R = _R(L)
    OT = oracle.Tree(L)
    for k, camd in enumerate(rand_cams(rng, 6, W=9, H=7, inside=(seed == 1)) + degenerate_cams()):
        for ml in (OT.lmax, 2):
            d = dict(camd, max_level=ml)
            log("random tree", seed, "camera", k, "max_level", ml)
            parity.compare_all(R, OT, d, ops=("sum", "max", "wmean"), los_fields=(1, 0, True),
                               trace_rays=np.arange(d["W"] * d["H"]), what=f"seed{seed} cam{k} ml{ml}")


@pytest.mark.parametrize("name", ["p8x8_split2_fast", "p8x8_split4_fast", "p8x8_split2_fast_center"])
def test_gpu_split_rays_random_trees(name):
    """Rays cut into spans at base-level planes, one wave per span: every
    result against the oracle, including degenerate and inside cameras."""
    import paper_1210_8014_amd as amr

    v = amr.variants().index(name)
    K = len(name)
    rng = np.random.default_rng(10 + K)
    L = amrgen.random_tree(300 + K, lmax=6, p_refine=0.4, nfields=4)
    L.fields[1:] -= 5.0
    R = _R(L, variant=v)
    OT = oracle.Tree(L)
    for k, camd in enumerate(rand_cams(rng, 6, W=19, H=13, inside=("4" in name)) + degenerate_cams()):
        for ml in (OT.lmax, 3, 1):
            d = dict(camd, max_level=ml)
            log(name, "camera", k, "max_level", ml)
            parity.compare_all(R, OT, d, ops=("sum", "max", "wmean"), los_fields=(1, 0, True),
                               what=f"{name} cam{k} ml{ml}")


def test_gpu_every_truncation_level():
    L = amrgen.scene("tiny")
    R = _R(L)
    OT = oracle.Tree(L)
    for ml in range(0, 7):
        log("tiny max_level", ml)
        parity.compare_all(R, OT, amrgen.tiny_camera(128, 96, max_level=ml), ops=("sum", "max"),
                           trace_rays=np.arange(0, 128 * 96, 3), what=f"tiny L{ml}")


def test_gpu_edge_cases():
    L = amrgen.scene("tiny")
    R = _R(L)
    OT = oracle.Tree(L)
    cams = [
        amrgen.tiny_camera(1, 1),                                                   # one pixel
        amrgen.tiny_camera(37, 23),                                                 # ragged packets
        amrgen.camera("persp", (0.5, 0.5, 2.0), (0.5, 0.5, 3.0), (0, 1, 0), 33, 17, fov_y=1.0, max_level=6),  # misses
        amrgen.camera("persp", (0.41, 0.52, 0.47), (0.9, 0.1, 0.2), (0, 1, 0), 45, 31, fov_y=1.3, max_level=6),  # inside
        amrgen.camera("ortho", (0.5, 0.5, -0.5), (0.5, 0.5, 0.5), (0, 1, 0), 5, 5, ortho_height=1.25, max_level=6),
    ]
    for k, camd in enumerate(cams):
        log("edge camera", k)
        parity.compare_all(R, OT, camd, ops=("sum", "max"), trace_rays=np.arange(camd["W"] * camd["H"]),
                           what=f"edge{k}")
    out, _ = R.full(R.camera(cams[2]), 1)
    assert np.all(np.isneginf(out))


def test_gpu_deep_levels_fp64_boundaries():
    m_thr = 3e-3
    L = amrgen.generate(amrgen.DISK, 0, 7, 20, m_thr, True, False)
    R = _R(L)
    OT = oracle.Tree(L)
    tgt = amrgen.core_position(0, 20, m_thr, 0)
    s = 2.0 ** -13
    cam = amrgen.camera("persp", (tgt[0], tgt[1] - 0.8 * s, tgt[2] + 0.6 * s), tgt, (0, 0.6, 0.8), 256, 256,
                        fov_y=0.9, max_level=-1)
    assert R.camera(cam).max_level >= 18
    log("deep zoom", R.camera(cam).max_level)
    parity.compare_all(R, OT, cam, ops=("sum", "max"), trace_rays=np.arange(0, 65536, 11), what="deep")


@pytest.fixture(scope="module")
def disk_full():
    """The galaxy-disk scene at full size (library tree and oracle tree) and
    the seeded 1% sample of the 2048^2 pixels, shared by the tests below."""
    log("generating disk")
    L = amrgen.scene("disk")
    R = _R(L)
    OT = oracle.Tree(L)
    n = 2048 * 2048
    rays = np.sort(np.random.default_rng(1).choice(n, n // 100, replace=False))
    yield R, OT, rays
    R.T.close()


def test_gpu_disk_full_size_sampled(disk_full):
    """Galaxy disk, ~20.5M leaves, levels 7..16, 2048^2 perspective cameras at
    inclinations 0/45/90: sum and line-of-sight mass-weighted velocity on a
    seeded 1% ray sample; cell sequences of 2000 rays; determinism; every
    kernel variant bit-identical."""
    import paper_1210_8014_amd as amr

    R, OT, rays = disk_full
    for k, camd in enumerate(amrgen.disk_cameras()):
        log("disk camera", k)
        res = parity.compare_all(R, OT, camd, ops=("sum", "max", "wmean"), rays=rays, los_fields=(1, 0, True),
                                 trace_rays=rays[::21], what=f"disk cam{k}")
        log("  worst sum rel", res["sum"], "wmean", res["wmean"])
    cam = R.camera(amrgen.disk_cameras()[1])
    a, _ = R.full(cam, amr.SUM, variant=0)
    am, _ = R.full(cam, amr.MAX, variant=0)
    names = amr.variants()
    by_name = {}
    for v in range(len(names)):
        log("disk variant", v)
        b, _ = R.full(cam, amr.SUM, variant=v)
        by_name[names[v]] = b
        if names[v].endswith("_center"):
            # dispatch order only: equal to the same variant in plain order
            plain = by_name[names[v][: -len("_center")]]
            assert np.array_equal(plain.view(np.int32), b.view(np.int32)), f"variant {v} differs from plain order"
        if _is_split(v):
            # spans merged in order: same cells, sums differ by rounding only
            assert np.all(np.abs(b.astype(np.float64) - a) <= 2e-6 * np.abs(a)), f"variant {v} differs"
            bm, _ = R.full(cam, amr.MAX, variant=v)
            assert np.array_equal(am.view(np.int32), bm.view(np.int32)), f"variant {v} max differs"
        else:
            assert np.array_equal(a.view(np.int32), b.view(np.int32)), f"variant {v} differs"
    w1, x1 = R.full(cam, amr.WMEAN, field=1, weight=0, los=True)
    w2, x2 = R.full(cam, amr.WMEAN, field=1, weight=0, los=True)
    assert np.array_equal(w1.view(np.int32), w2.view(np.int32)) and np.array_equal(x1, x2)


def test_gpu_disk_batch_launch_as_benched(disk_full):
    """The benchmarked launch at full size: per op one batch over the three
    2048^2 disk views (sum of density; line-of-sight velocity weighted by
    density), in the grid shapes p8x8_fast_grid (the tuner's choice on this
    workload) and p8x8_split2_grid: against the oracle on the seeded 1% ray
    sample, and bit-identical to the per-image renders of the same walk."""
    import paper_1210_8014_amd as amr

    R, OT, rays = disk_full
    descs = amrgen.disk_cameras()
    cams = [R.camera(d) for d in descs]
    n = 2048 * 2048
    assert all(c.W * c.H == n for c in cams)
    pairs = [(0, k) for k in range(len(cams))]
    outs_s = [torch.full((n,), -7.0, device="cuda") for _ in cams]
    outs_w = [torch.full((n,), -7.0, device="cuda") for _ in cams]
    auxs = [torch.full((n,), -7.0, device="cuda") for _ in cams]
    Bs = amr.Batch([R.T], cams, pairs, amr.SUM, outs_s, field=0)
    Bw = amr.Batch([R.T], cams, pairs, amr.WMEAN, outs_w, auxs, field=1, weight=0, los=True)
    refs = []
    for k, camd in enumerate(descs):
        ocam = OT.camera(camd)
        refs.append((OT.render(ocam, oracle.SUM, rays=rays),
                     OT.render(ocam, oracle.WMEAN, field=1, weight=0, los=True, rays=rays)))
    names = amr.batch_configs()
    for cfg, variant in (("p8x8_fast_grid", 0), ("p8x8_split2_grid", amr.variants().index("p8x8_split2_fast"))):
        log("batch", cfg)
        for x in outs_s + outs_w + auxs:
            x.fill_(-7.0)
        for B in (Bs, Bw):
            B.set_config(names.index(cfg))
            B.run()
        torch.cuda.synchronize()
        for k in range(len(cams)):
            s_, w_, x_ = (t.cpu().numpy() for t in (outs_s[k], outs_w[k], auxs[k]))
            parity.check_sum(s_[rays], refs[k][0]["val"], f"batch {cfg} cam{k} sum")
            parity.check_wmean(w_[rays], x_[rays], refs[k][1], f"batch {cfg} cam{k} wmean")
            a, _ = R.full(cams[k], amr.SUM, variant=variant)
            w, x = R.full(cams[k], amr.WMEAN, field=1, weight=0, los=True, variant=variant)
            assert np.array_equal(a.view(np.int32), s_.view(np.int32)), f"{cfg} cam{k} sum differs from the single render"
            assert np.array_equal(w.view(np.int32), w_.view(np.int32)), f"{cfg} cam{k} wmean differs"
            assert np.array_equal(x.view(np.int32), x_.view(np.int32)), f"{cfg} cam{k} weight differs"
    Bs.close()
    Bw.close()


@pytest.mark.slow
def test_gpu_deepzoom_full_size_sampled():
    """Deep zoom at full size: ~201M leaves to level 22, the eye inside the disk
    2^-9 box from core 0, 4096^2 pixels, automatic maximum level 21, so cells
    at levels 18..21 (FP64 chords) are crossed.  Sum and max on a seeded 1% ray
    sample for the default, the unsplit walk and the unsplit walk with an
    ancestor stack (also bit-identical to the stackless one over the whole
    image); cell sequences of 1500 rays;
    the streamed render of the same image from the tree in host memory, in
    the bench's configuration, on the same sample (max also bit-identical to
    the in-memory render); slices at levels 22, 21 and 18."""
    import paper_1210_8014_amd as amr

    log("generating deep-zoom scene")
    L = amrgen.scene("deepzoom")
    log("leaves", L.n, "lmax", L.lmax)
    assert L.lmax == 22 and L.n > 150_000_000
    R = _R(L)
    log("library tree", R.T.ncells, "cells")
    OT = oracle.Tree(L)
    log("oracle tree", OT.nodes, "nodes")
    # the streamed render as the bench times it: the tree in pinned host
    # memory, chunks of at most 8M cells through four device buffers
    H = amr.Tree(L, host_only=True)
    P = amr.StreamPlan(H, 8 << 20, nbuffers=4)
    H.close()
    log("stream plan", P.nchunks, "chunks")
    del L
    camd = amrgen.deepzoom_camera()
    cam = R.camera(camd)
    assert cam.max_level == 21
    n = cam.W * cam.H
    rays = np.sort(np.random.default_rng(5).choice(n, n // 100, replace=False))
    lds = amr.variants().index("p8x8_w4_fastlds")  # the walk with an ancestor stack (the deep zoom's tuned choice)
    for v in (-1, 0, lds):
        R.variant = v
        log("variant", v)
        res = parity.compare_all(R, OT, camd, ops=("sum", "max"), rays=rays,
                                 trace_rays=rays[::112] if v == -1 else None, what=f"deepzoom v{v}")
        log("  worst sum rel", res["sum"])
    for op in (amr.SUM, amr.MAX):
        a, _ = R.full(cam, op, variant=0)
        b, _ = R.full(cam, op, variant=lds)
        assert np.array_equal(a.view(np.int32), b.view(np.int32)), "stack walk differs from the stackless walk"
        # 11 levels below the base level: the untuned default is the stack walk
        c, _ = R.full(cam, op, variant=-1)
        assert np.array_equal(b.view(np.int32), c.view(np.int32)), "deep default is not the stack walk"
    offs, cells = R.trace(cam, rays[::112])
    assert cells[:, 0].max() >= 18
    ocam = OT.camera(camd)
    ws = torch.empty(amr.StreamPlan.workspace_bytes(cam.W, cam.H) // 4, device="cuda")
    so = torch.empty(n, device="cuda")
    for op in (amr.SUM, amr.MAX):
        st = P.render(cam, op, so, ws)
        torch.cuda.synchronize()
        got = so.cpu().numpy()
        log("streamed", op, "chunks walked", st[0], "bytes copied", st[1])
        if op == amr.MAX:
            ref_in, _ = R.full(cam, op, variant=0)
            assert np.array_equal(got.view(np.int32), ref_in.view(np.int32)), "streamed max differs from in-memory"
            parity.check_max(got[rays], OT.render(ocam, oracle.MAX, rays=rays)["max"], "streamed deepzoom max")
        else:
            log("  worst sum rel", parity.check_sum(got[rays], OT.render(ocam, oracle.SUM, rays=rays)["val"],
                                                    "streamed deepzoom sum"))
    P.close()
    # slice maps through core 0 at the full depth and at the camera's level:
    # a 2048^2 plane 2^-10 box wide (pixel 2^-21 box), every point bit for bit
    import paper_1210_8014_amd as amr

    tgt = np.array(camd["target"])
    for ml in (22, 21, 18):
        sd = amrgen.camera("ortho", tgt, tgt + np.array([0.0, 0.0, 1.0]), (0, 1, 0), 2048, 2048,
                           ortho_height=2.0 ** -10, max_level=ml)
        scam, socam = R.camera(sd), OT.camera(sd)
        assert scam.as_dict() == socam.as_dict()
        out = torch.empty(2048 * 2048, device="cuda")
        amr.slice_map(R.T, scam, out)
        torch.cuda.synchronize()
        got, ref = out.cpu().numpy(), OT.slice(socam)
        assert not np.isnan(ref).any()
        assert np.array_equal(got.view(np.int32), ref.view(np.int32)), ml
        log("deep-zoom slice at level", ml, "bit-exact;", len(np.unique(ref)), "distinct values")


def test_gpu_rejects_bad_arguments():
    import paper_1210_8014_amd as amr

    R = _R(amrgen.scene("tiny"))
    cam = R.camera(amrgen.tiny_camera())
    out = torch.empty(cam.W * cam.H, dtype=torch.float32, device="cuda")
    for kw in (dict(field=1), dict(variant=99)):
        with pytest.raises(amr.AmrError) as e:
            amr.render(R.T, cam, amr.SUM, out, **kw)
        assert e.value.status == 1


def test_gpu_every_entry_point_rejects_out_of_range_records():
    """Every entry point that walks rays refuses a record outside the integer
    ranges the kernels rely on (AMR_EINVAL, nothing launched): the plain,
    batched, learned-LOD (both forms), streamed, resolution, slice and debug
    calls."""
    import paper_1210_8014_amd as amr
    from paper_1210_8014_amd import lod
    from tests.test_builder_cpu import _bad_records

    L = amrgen.scene("tiny")
    R = _R(L)
    H = amr.Tree(L, host_only=True)
    P = amr.StreamPlan(H, H.ncells)
    m = lod.LodModel()
    n = 1 << 16
    out = torch.empty(n, device="cuda")
    aux = torch.empty(n, device="cuda")
    ws = torch.empty(lod.workspace_bytes(256, 256), dtype=torch.uint8, device="cuda")
    sws = torch.empty(amr.StreamPlan.workspace_bytes(256, 256) // 4, device="cuda")
    st = torch.zeros(8, dtype=torch.int64, device="cuda")
    feat = torch.empty(lod.tiles(256, 256) * 32, dtype=torch.int16, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    bits = torch.zeros(R.T.ncells // 32 + 1, dtype=torch.int32, device="cuda")
    rays = torch.arange(4, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int32, device="cuda")
    offs = torch.zeros(5, dtype=torch.int64, device="cuda")
    cells = torch.zeros(64, dtype=torch.int32, device="cuda")
    calls = {
        "render": lambda c: amr.render(R.T, c, amr.SUM, out),
        "batch": lambda c: amr.Batch([R.T], [c], [(0, 0)], amr.SUM, [out]),
        "lod features": lambda c: lod.features(R.T, c, feat, coarse_level=4),
        "lod render": lambda c: lod.render_lod(R.T, c, amr.SUM, m, out, ws, st),
        "lod render noalloc": lambda c: lod.render_lod_noalloc(R.T, c, amr.SUM, m, out, st),
        "streamed": lambda c: P.render(c, amr.SUM, out, sws),
        "resolution": lambda c: amr.resolution(R.T, c, out),
        "slice": lambda c: amr.slice_map(R.T, c, out),
        "count segments": lambda c: amr.count_segments(R.T, c, tot),
        "mark cells": lambda c: amr.mark_cells(R.T, c, bits, tot),
        "count rays": lambda c: amr.count_rays(R.T, c, rays, cnt),
        "trace rays": lambda c: amr.trace_rays(R.T, c, rays, offs, cells),
    }
    for kind in ("ortho", "persp"):
        d = amrgen.tiny_camera() if kind == "ortho" else amrgen.camera(
            "persp", (0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0, 1, 0), 256, 256, fov_y=0.6, max_level=6)
        cam = R.camera(d)
        for what, bad in _bad_records(cam):
            if what == "zero orthographic direction":
                bad.F[1] = bad.F[2] = 0
            for name, f in calls.items():
                with pytest.raises(amr.AmrError) as e:
                    f(bad)
                assert e.value.status == 1, (kind, what, name)
    torch.cuda.synchronize()
    P.close()


def test_gpu_distinct_cells_match_oracle():
    """amr_mark_cells: the distinct cells met by all rays of an image (the
    basis of the compulsory traffic) equal the set of cells in the oracle's
    cell sequences; a second image accumulates onto the same bitmap."""
    import paper_1210_8014_amd as amr

    L = amrgen.scene("tiny")
    R = _R(L)
    OT = oracle.Tree(L)
    d1, d2 = amrgen.tiny_camera(), amrgen.camera("persp", (1.6, -0.7, 1.3), (0.5, 0.5, 0.5), (0, 0, 1), 97, 61,
                                                 fov_y=0.9, max_level=5)
    words = (R.T.ncells + 31) // 32
    bits = torch.zeros(words, dtype=torch.int32, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    seen = set()
    for k, d in enumerate((d1, d2)):
        cam, ocam = R.camera(d), OT.camera(d)
        amr.mark_cells(R.T, cam, bits, tot)
        torch.cuda.synchronize()
        _, cells, _ = OT.trace(ocam, np.arange(cam.W * cam.H))
        seen |= set(map(tuple, cells.tolist()))
        log("image", k, "distinct cells", int(tot.item()), "oracle", len(seen))
        assert int(tot.item()) == len(seen)
    # the bitmap holds exactly that many bits
    b = bits.cpu().numpy().view(np.uint32)
    assert int(np.unpackbits(b.view(np.uint8)).sum()) == len(seen)
