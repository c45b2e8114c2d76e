"""GPU: resolution plane, adaptive Gaussian post-filter and slice maps
against the oracle (oracle.Tree.resolution / slice, oracle/post.py)."""
import numpy as np
import pytest

import amrgen
import oracle
from oracle import post as OP
from tests import parity
from tests.test_oracle_pins import degenerate_cams, rand_cams

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(*a):
    print(*a, flush=True)


def _res(amr, T, cam):
    r = torch.empty(cam.W * cam.H, device="cuda")
    amr.resolution(T, cam, r)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def _check_res(got, ref, what):
    """Same bar as a sum (chord-weighted sums): 2e-6 relative, 0 for misses."""
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0), what
    rel = np.abs(got[~zero] - ref[~zero]) / ref[~zero]
    assert rel.size == 0 or rel.max() <= 2e-6, (what, rel.max())
    return float(rel.max()) if rel.size else 0.0


def test_gpu_resolution_matches_oracle():
    import paper_1210_8014_amd as amr

    worst = 0.0
    L = amrgen.scene("tiny")
    T, OT = amr.Tree(L), oracle.Tree(L)
    d = amrgen.tiny_camera(131, 97, max_level=6)
    worst = max(worst, _check_res(_res(amr, T, amr.set_camera(d, T)), OT.resolution(OT.camera(d)), "tiny"))
    rng = np.random.default_rng(4)
    Lr = amrgen.random_tree(77, lmax=5, p_refine=0.45, nfields=1)
    T, OT = amr.Tree(Lr), oracle.Tree(Lr)
    for k, d in enumerate(rand_cams(rng, 6, 23, 17) + degenerate_cams()[:6] + rand_cams(rng, 4, 19, 11, inside=True)):
        d = dict(d, max_level=int(rng.integers(2, 6)))
        worst = max(worst, _check_res(_res(amr, T, amr.set_camera(d, T)), OT.resolution(OT.camera(d)), f"random {k}"))
    Ld = amrgen.disk(seed=3, lmax=11, m_thr=2e-4)
    T, OT = amr.Tree(Ld), oracle.Tree(Ld)
    for inc in (0.0, 60.0):
        d = amrgen.disk_camera(inc, 150, 110, max_level=11)
        worst = max(worst, _check_res(_res(amr, T, amr.set_camera(d, T)), OT.resolution(OT.camera(d)), f"disk {inc}"))
    log("resolution: worst rel err", worst)


def _blur(amr, img, res, W, H, kappa):
    i = torch.as_tensor(np.ascontiguousarray(img, np.float32).ravel(), device="cuda")
    r = torch.as_tensor(np.ascontiguousarray(res, np.float32).ravel(), device="cuda")
    out = torch.full_like(i, -7.0)
    ws = torch.empty(amr.blur_workspace_bytes(W, H), dtype=torch.uint8, device="cuda")
    amr.blur_adaptive(i, r, W, H, kappa, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def test_gpu_blur_on_seeded_planes():
    """The filter alone, both sides on the same seeded fp32 image and
    resolution planes (ragged against both passes' tiles): zeros, values
    below the first level, exactly at ladder levels, between them and beyond
    the top.  Bound per pixel: 5e-7 of the largest level value (fp32 weights
    and stored row passes, fp64 sums, the final rounding) plus 4e-6 of the
    spread of the neighbouring levels (sigma and log2 sigma in fp32: the
    blend weight errs by ~2.4e-6 at 20 half-octaves)."""
    import paper_1210_8014_amd as amr

    rng = np.random.default_rng(9)
    H, W = 61, 293
    img = np.exp(rng.normal(size=(H, W))).astype(np.float32)
    img[:, 100:140] *= 30.0  # edges for the blur to smooth
    res = rng.uniform(0.0, 50.0, (H, W)).astype(np.float32)
    res[::7, :] = 0.0
    res[1::7, :] = rng.uniform(0.0, 1.0, (len(range(1, H, 7)), W))  # below the first level (kappa 0.5)
    lv = np.array([OP.sigma_level(k) / 0.5 for k in range(OP.NLEVELS)], np.float32)
    res[2::7, :] = lv[rng.integers(0, OP.NLEVELS, (len(range(2, H, 7)), W))]
    res[3::7, :] = 1e4
    got = _blur(amr, img, res, W, H, 0.5)
    ref, spread = OP.adaptive_blur_terms(img.astype(np.float64), res.astype(np.float64), float(np.float32(0.5)),
                                         np.arange(H * W))
    scale = np.maximum(np.abs(ref), np.abs(ref) + spread)
    err = np.abs(got - ref)
    bound = 5e-7 * scale + 4e-6 * spread
    log("blur: max err / bound", float((err / bound).max()), "max rel err", float((err / np.abs(ref)).max()))
    assert np.all(err <= bound)
    # sigma <= 0 is the image itself, bit for bit
    z = (res == 0.0).ravel()
    assert np.array_equal(got[z], img.ravel()[z].astype(np.float64))


def test_gpu_blur_end_to_end_matches_oracle_chain():
    """Render, resolution plane and blur on the GPU against the oracle's own
    render, resolution and blur of the same scene (a small disk).  Bound per
    pixel: the blur averages pixels each within 2e-6 of the oracle (the sum
    bar), plus the spread of the neighbouring levels times the blend weight's
    error (resolution within 2e-6: 2 x 2e-6 / ln 2 in u, plus the fp32 log2
    of the previous test)."""
    import paper_1210_8014_amd as amr

    Ld = amrgen.disk(seed=3, lmax=11, m_thr=2e-4)
    T, OT = amr.Tree(Ld), oracle.Tree(Ld)
    for ml in (5, 8):  # coarse truncations: cells of ~7 and ~1 pixels
        _chain(amr, T, OT, amrgen.disk_camera(50.0, 241, 171, max_level=ml))


def _chain(amr, T, OT, d):
    cam, ocam = amr.set_camera(d, T), OT.camera(d)
    W, H = cam.W, cam.H
    img = torch.empty(W * H, device="cuda")
    amr.render(T, cam, amr.SUM, img)
    res = torch.empty_like(img)
    amr.resolution(T, cam, res)
    out = torch.empty_like(img)
    ws = torch.empty(amr.blur_workspace_bytes(W, H), dtype=torch.uint8, device="cuda")
    amr.blur_adaptive(img, res, W, H, 0.5, out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    oimg = OT.render(ocam, oracle.SUM)["val"].reshape(H, W)
    ores = OT.resolution(ocam).reshape(H, W)
    log("resolution range", float(ores.min()), float(ores.max()))
    ref, spread = OP.adaptive_blur_terms(oimg, ores, 0.5, np.arange(H * W))
    err = np.abs(got - ref)
    bound = 2.5e-6 * (np.abs(ref) + spread) + 1e-5 * spread
    pos = bound > 0
    log("blur chain at level", cam.max_level, ": max err / bound", float((err[pos] / bound[pos]).max()),
        "max rel err", float((err[ref != 0] / np.abs(ref[ref != 0])).max()))
    assert np.all(err <= bound)


def test_gpu_slice_bit_exact():
    """Slice maps: every pixel's value bit for bit (NaN outside the box) on
    the tiny scene, random trees (second field) with face-aligned and random
    orthographic planes at several truncation levels, and the disk midplane
    z = 1/2 (a face at every level) at 512^2."""
    import paper_1210_8014_amd as amr

    def check(T, OT, d, field=0, what=""):
        cam, ocam = amr.set_camera(d, T), OT.camera(d)
        assert cam.as_dict() == ocam.as_dict()
        out = torch.full((cam.W * cam.H,), -7.0, device="cuda")
        amr.slice_map(T, cam, out, field=field)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = OT.slice(ocam, field=field)
        nan = np.isnan(ref)
        assert np.array_equal(np.isnan(got), nan), what
        assert np.array_equal(got[~nan].view(np.int32), ref[~nan].view(np.int32)), what
        return int((~nan).sum())

    L = amrgen.scene("tiny")
    T, OT = amr.Tree(L), oracle.Tree(L)
    n = check(T, OT, amrgen.camera("ortho", (0.5, 0.5, 0.37), (0.5, 0.5, 1.0), (0, 1, 0), 256, 256,
                                   ortho_height=1.0, max_level=6), what="tiny")
    rng = np.random.default_rng(12)
    Lr = amrgen.random_tree(91, lmax=5, p_refine=0.45, nfields=2)
    T, OT = amr.Tree(Lr), oracle.Tree(Lr)
    cams = [c for c in rand_cams(rng, 20, 37, 29) if c["kind"] == "ortho"] + \
        [c for c in degenerate_cams() if c["kind"] == "ortho"]
    for k, d in enumerate(cams):
        for ml in (1, 3, 5):
            n += check(T, OT, dict(d, max_level=ml), field=1, what=f"random {k} level {ml}")
    Ld = amrgen.disk(seed=3, lmax=12, m_thr=1e-4)
    T, OT = amr.Tree(Ld), oracle.Tree(Ld)
    for ml in (7, 12):
        n += check(T, OT, amrgen.camera("ortho", (0.5, 0.5, 0.5), (0.5, 0.5, 1.5), (0, 1, 0), 512, 512,
                                        ortho_height=1.0, max_level=ml), what=f"disk midplane {ml}")
    log("slices: points compared", n)
    with pytest.raises(amr.AmrError) as e:  # perspective records have no plane
        amr.slice_map(T, amr.set_camera(amrgen.disk_camera(10.0, 8, 8), T), torch.empty(64, device="cuda"))
    assert e.value.status == 1


def test_gpu_render_with_resolution_equals_the_two_walks():
    """amr_render_with_resolution: the image bit-identical to amr_render with
    the unsplit variant p8x8_w1_fast and the plane bit-identical to
    amr_render_resolution, for every op, on the tiny scene, random trees
    with degenerate and inside cameras, and the disk at 2048^2 (both already
    checked against the oracle by the tests of those two calls)."""
    import paper_1210_8014_amd as amr

    v0 = amr.variants().index("p8x8_w1_fast")

    def same(T, d, what):
        cam = amr.set_camera(d, T)
        n = cam.W * cam.H
        nf = int(T.info.nfields)
        jobs = [(amr.SUM, {}), (amr.MAX, {})]
        if nf >= 4:
            jobs += [(amr.WMEAN, dict(field=1, weight=0, los=True)), (amr.SUM, dict(field=2)),
                     (amr.WMEAN, dict(field=3, weight=1, los=False))]
        ref_res = torch.empty(n, device="cuda")
        amr.resolution(T, cam, ref_res)
        for op, kw in jobs:
            a, x = torch.full((n,), -7.0, device="cuda"), torch.full((n,), -7.0, device="cuda")
            b, y, r = (torch.full((n,), -7.0, device="cuda") for _ in range(3))
            amr.render(T, cam, op, a, x if op == amr.WMEAN else None, variant=v0, **kw)
            amr.render_with_resolution(T, cam, op, b, r, y if op == amr.WMEAN else None, **kw)
            torch.cuda.synchronize()
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (what, op, kw)
            if op == amr.WMEAN:
                assert torch.equal(x.view(torch.int32), y.view(torch.int32)), (what, op, kw)
            assert torch.equal(ref_res.view(torch.int32), r.view(torch.int32)), (what, op, kw)

    L = amrgen.scene("tiny")
    same(amr.Tree(L), amrgen.tiny_camera(131, 97, max_level=6), "tiny")
    rng = np.random.default_rng(8)
    Lr = amrgen.random_tree(78, lmax=5, p_refine=0.45, nfields=4)
    Lr.fields[1:] -= 5.0
    T = amr.Tree(Lr)
    for k, d in enumerate(rand_cams(rng, 4, 23, 17) + degenerate_cams()[:6] + rand_cams(rng, 3, 19, 11, inside=True)):
        same(T, dict(d, max_level=int(rng.integers(2, 6))), f"random {k}")
    T = amr.Tree(amrgen.scene("disk"))
    same(T, amrgen.disk_camera(45.0, 2048, 2048, max_level=16), "disk 2048")
    T.close()
