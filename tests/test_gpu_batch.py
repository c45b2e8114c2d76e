"""GPU: batched persistent hipGraph launch is bit-identical to unsplit per-image
renders, on every replay; stale trees are refused; the tuners return valid
choices that render identically."""
import numpy as np
import pytest

import amrgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(*a):
    print(*a, flush=True)


def _mixed_batch():
    import paper_1210_8014_amd as amr

    trees = [amr.Tree(amrgen.scene("tiny")), amr.Tree(amrgen.disk(seed=3, lmax=11, m_thr=2e-4)),
             amr.Tree(amrgen.disk(seed=4, lmax=12, m_thr=1e-4))]
    descs = [amrgen.tiny_camera(37, 23), amrgen.tiny_camera(256, 256)]
    descs += amrgen.orbit_cameras(8, seed=1, side_lo=40, side_hi=300, multiple=1, max_level=12)
    cams = [amr.set_camera(d) for d in descs]
    pairs = [(t, c) for t in range(3) for c in range(len(cams))]
    return trees, cams, pairs


@pytest.mark.parametrize("op", ["sum", "max", "wmean", "sum_field1", "wmean_los"])
def test_batch_matches_single_renders_on_every_replay(op):
    """sum and max of field 0 and wmean with the line of sight on the
    interleaved records run the grid kernels specialised for that layout;
    sum of field 1 and wmean of a scalar field run the general ones."""
    import paper_1210_8014_amd as amr

    trees, cams, pairs = _mixed_batch()
    o = {"sum": amr.SUM, "max": amr.MAX, "wmean": amr.WMEAN, "sum_field1": amr.SUM, "wmean_los": amr.WMEAN}[op]
    kw = {"sum": dict(field=0), "max": dict(field=0), "sum_field1": dict(field=1),
          "wmean": dict(field=1, weight=0, los=False), "wmean_los": dict(field=1, weight=0, los=True)}[op]
    if op in ("wmean", "sum_field1", "wmean_los"):
        # tiny has one field: restrict to the disks (four fields)
        pairs = [p for p in pairs if p[0] > 0]
    outs = [torch.full((cams[c].W * cams[c].H,), -7.0, device="cuda") for _, c in pairs]
    auxs = [torch.full_like(x, -7.0) for x in outs] if o == amr.WMEAN else None
    B = amr.Batch(trees, cams, pairs, o, outs, auxs, **kw)
    split_variant = amr.variants().index("p8x8_split2_fast")

    def singles(variant):
        out = []
        for (t, c) in pairs:
            r = torch.empty(cams[c].W * cams[c].H, device="cuda")
            a = torch.empty_like(r) if o == amr.WMEAN else None
            amr.render(trees[t], cams[c], o, r, a, variant=variant, **kw)
            out.append((r, a))
        return out

    ref = singles(0)  # the unsplit walk of the persistent configurations
    ref_split = singles(split_variant)
    torch.cuda.synchronize()
    for rep in range(3):
        log("replay", rep)
        for x in outs:
            x.fill_(-7.0)  # eager work between replays
        torch.cuda.synchronize()
        B.run()
        torch.cuda.synchronize()
        for k, ((r, a), x) in enumerate(zip(ref, outs)):
            assert torch.equal(r.view(torch.int32), x.view(torch.int32)), f"image {k} differs on replay {rep}"
            if a is not None:
                assert torch.equal(a.view(torch.int32), auxs[k].view(torch.int32))
    for cfg in range(len(amr.batch_configs())):
        name = amr.batch_configs()[cfg]
        log("config", cfg, name)
        B.set_config(cfg)
        for x in outs:
            x.fill_(-7.0)
        B.run()
        torch.cuda.synchronize()
        want = ref_split if "split" in name else ref
        for k, ((r, _), x) in enumerate(zip(want, outs)):
            assert torch.equal(r.view(torch.int32), x.view(torch.int32)), f"config {name} image {k} differs"
    B.close()


def test_batch_refuses_freed_tree():
    import paper_1210_8014_amd as amr

    trees, cams, pairs = _mixed_batch()
    outs = [torch.empty(cams[c].W * cams[c].H, device="cuda") for _, c in pairs]
    B = amr.Batch(trees, cams, pairs, amr.SUM, outs)
    B.run()
    torch.cuda.synchronize()
    trees[1].close()
    with pytest.raises(amr.AmrError) as e:
        B.run()
    assert e.value.status == 6
    B.close()


def test_tuners_choose_valid_configurations(tmp_path):
    import paper_1210_8014_amd as amr

    trees, cams, pairs = _mixed_batch()
    outs = [torch.empty(cams[c].W * cams[c].H, device="cuda") for _, c in pairs]
    B = amr.Batch(trees, cams, pairs, amr.SUM, outs)
    best, times = B.tune(reps=1)
    assert 0 <= best < len(amr.batch_configs()) and B.config == best
    assert all(t > 0 for t in times.values())
    t = trees[1]
    cam = amr.set_camera(amrgen.disk_camera(45.0, 300, 200, max_level=11), t)
    out = torch.empty(300 * 200, device="cuda")
    cache = str(tmp_path / "tune.json")
    v, tv = amr.tune(t, cam, amr.SUM, out, reps=1, cache=cache)
    assert 0 <= v < len(amr.variants())
    a = torch.empty_like(out)
    amr.render(t, cam, amr.SUM, a)  # default variant = the tuned one
    b = torch.empty_like(out)
    amr.render(t, cam, amr.SUM, b, variant=v)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    assert amr.apply_tuning(t, cam, amr.SUM, cache=cache) == v


def test_batched_disk_snapshots_match_oracle_on_sampled_rays():
    """A slice of the batched workload at its real shape: two disk snapshots
    (seeds 0 and 1: 5.3M and 8.2M leaves, density and velocity) under all
    64 orbit cameras (sides 512..2048, multiples of 16) = 128 images in one
    graph launch of the benchmarked grid configuration, sum and the
    line-of-sight weighted mean; every 8th image is checked against the
    oracle on a seeded 1% ray sample."""
    import oracle
    import paper_1210_8014_amd as amr
    from tests import parity

    leaves = [amrgen.scene("batch", seed=s) for s in (0, 1)]
    trees = [amr.Tree(L) for L in leaves]
    descs = amrgen.orbit_cameras(64, seed=0)
    cams = [amr.set_camera(d) for d in descs]
    pairs = [(t, c) for t in range(2) for c in range(64)]
    checked = list(range(0, len(pairs), 8))
    OTs = [oracle.Tree(L) for L in leaves]
    rng = np.random.default_rng(42)
    samples = {k: np.sort(rng.choice(cams[pairs[k][1]].W * cams[pairs[k][1]].H,
                                     cams[pairs[k][1]].W * cams[pairs[k][1]].H // 100, replace=False))
               for k in checked}
    for op in ("sum", "wmean"):
        o = amr.SUM if op == "sum" else amr.WMEAN
        kw = dict(field=1, weight=0, los=True) if op == "wmean" else {}
        outs = [torch.empty(cams[c].W * cams[c].H, device="cuda") for _, c in pairs]
        auxs = [torch.empty_like(x) for x in outs] if op == "wmean" else None
        B = amr.Batch(trees, cams, pairs, o, outs, auxs, **kw)
        B.set_config(amr.batch_configs().index("p8x8_fast_grid"))
        B.run()
        torch.cuda.synchronize()
        worst = 0.0
        for k in checked:
            t, c = pairs[k]
            ocam = OTs[t].camera(descs[c])
            assert ocam.as_dict() == cams[c].as_dict()
            r = samples[k]
            got = outs[k].cpu().numpy()[r]
            if op == "sum":
                worst = max(worst, parity.check_sum(got, OTs[t].render(ocam, oracle.SUM, rays=r)["val"], f"image {k}"))
            else:
                ref = OTs[t].render(ocam, oracle.WMEAN, field=1, weight=0, los=True, rays=r)
                worst = max(worst, parity.check_wmean(got, auxs[k].cpu().numpy()[r], ref, f"image {k}"))
        log(op, "batch of", len(pairs), "images:", len(checked), "checked on 1% samples, worst", f"{worst:.2e}")
        B.close()


def test_weight_plane_of_wmean_is_the_sum_projection_of_the_weight():
    """The weighted mean accumulates the weight integral with exactly the sum
    projection's arithmetic (product of the cell's weight and the chord,
    Kahan-added in walk order, spans merged alike), so its weight plane is
    the sum image of the weight field bit for bit: for the specialised and
    the general kernels, every batch configuration and the single-image
    variants."""
    import paper_1210_8014_amd as amr

    trees, cams, pairs = _mixed_batch()
    pairs = [p for p in pairs if p[0] > 0]  # the disks (four fields)
    for los in (True, False):
        kw = dict(field=1, weight=0, los=los)
        sums = [torch.empty(cams[c].W * cams[c].H, device="cuda") for _, c in pairs]
        means = [torch.empty_like(x) for x in sums]
        weights = [torch.empty_like(x) for x in sums]
        S = amr.Batch(trees, cams, pairs, amr.SUM, sums, field=0)
        M = amr.Batch(trees, cams, pairs, amr.WMEAN, means, weights, **kw)
        for cfg in range(len(amr.batch_configs())):
            S.set_config(cfg)
            M.set_config(cfg)
            for x in sums + weights:
                x.fill_(-7.0)
            S.run()
            M.run()
            torch.cuda.synchronize()
            for k, (s, w) in enumerate(zip(sums, weights)):
                assert torch.equal(s.view(torch.int32), w.view(torch.int32)), \
                    f"los {los} config {amr.batch_configs()[cfg]} image {k}"
        S.close()
        M.close()
        for v in range(len(amr.variants())):
            for (t, c) in pairs[:4]:
                s = torch.empty(cams[c].W * cams[c].H, device="cuda")
                m, w = torch.empty_like(s), torch.empty_like(s)
                amr.render(trees[t], cams[c], amr.SUM, s, variant=v, field=0)
                amr.render(trees[t], cams[c], amr.WMEAN, m, w, variant=v, **kw)
                torch.cuda.synchronize()
                assert torch.equal(s.view(torch.int32), w.view(torch.int32)), \
                    f"los {los} variant {amr.variants()[v]} tree {t} camera {c}"
        log("los", los, "weight plane equals the sum image on", len(pairs), "images")


def test_deep_batch_with_ancestor_stack_matches_single_renders():
    """A batch whose maximum level lies 10 levels below the tree's base level
    (a disk refined to level 17, base level 7) runs the grid kernels that
    keep an ancestor stack; every image equals the stackless single render of
    the same shape bit for bit (sum, max, wmean; both grid shapes)."""
    import paper_1210_8014_amd as amr

    T = amr.Tree(amrgen.disk(seed=5, lmax=17, m_thr=2e-5))
    assert T.lmax == 17
    descs = amrgen.orbit_cameras(6, seed=3, side_lo=96, side_hi=256, multiple=1, max_level=17)
    cams = [amr.set_camera(d) for d in descs]
    assert all(c.max_level == 17 for c in cams)
    pairs = [(0, c) for c in range(len(cams))]
    split_variant = amr.variants().index("p8x8_split2_fast")
    for o, kw in ((amr.SUM, {}), (amr.MAX, {}), (amr.WMEAN, dict(field=1, weight=0, los=True))):
        outs = [torch.full((c.W * c.H,), -7.0, device="cuda") for c in cams]
        auxs = [torch.full_like(x, -7.0) for x in outs] if o == amr.WMEAN else None
        B = amr.Batch([T], cams, pairs, o, outs, auxs, **kw)
        for cfg, variant in (("p8x8_fast_grid", 0), ("p8x8_split2_grid", split_variant)):
            B.set_config(amr.batch_configs().index(cfg))
            B.run()
            torch.cuda.synchronize()
            for k, c in enumerate(cams):
                r = torch.empty(c.W * c.H, device="cuda")
                a = torch.empty_like(r) if o == amr.WMEAN else None
                amr.render(T, c, o, r, a, variant=variant, **kw)
                torch.cuda.synchronize()
                assert torch.equal(r.view(torch.int32), outs[k].view(torch.int32)), f"op {o} {cfg} image {k}"
                if a is not None:
                    assert torch.equal(a.view(torch.int32), auxs[k].view(torch.int32)), f"op {o} {cfg} image {k}"
        B.close()
        log("deep batch op", o, "matches single renders")
