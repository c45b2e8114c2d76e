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
