"""GPU: the allocation-free LOD render (amr_render_lod_noalloc, fixed device
scratch) against amr_render_lod on a caller workspace: bit-identical
outputs, levels and statistics on two calls in a row, the second on a
smaller image, and a clear error for images beyond the fixed size."""
import numpy as np
import pytest

import amrgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(lod, amr, T, m, cam, op, kw, forced=None):
    n, nt = cam.W * cam.H, lod.tiles(cam.W, cam.H)
    res = []
    for noalloc in (False, True):
        out = torch.full((n,), -7.0, device="cuda")
        aux = torch.full((n,), -7.0, device="cuda") if op == amr.WMEAN else None
        st = torch.full((8,), -1, dtype=torch.int64, device="cuda")
        lev = torch.full((nt,), -1, dtype=torch.int8, device="cuda")
        if noalloc:
            lod.render_lod_noalloc(T, cam, op, m, out, st, aux=aux, tile_levels=lev, forced=forced, **kw)
        else:
            ws = torch.empty(lod.workspace_bytes(cam.W, cam.H), dtype=torch.uint8, device="cuda")
            lod.render_lod(T, cam, op, m, out, ws, st, aux=aux, tile_levels=lev, forced=forced, **kw)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), None if aux is None else aux.cpu().numpy(), st.cpu().numpy(),
                    lev.cpu().numpy()))
    return res


@pytest.mark.parametrize("op", ["sum", "wmean"])
def test_noalloc_lod_render_equals_workspace_render(op):
    import paper_1210_8014_amd as amr
    from paper_1210_8014_amd import lod

    T = amr.Tree(amrgen.disk(seed=6, lmax=14, m_thr=3e-5))
    m = lod.LodModel(path=lod.MODEL_PATH)
    m.config = dict(audit_frac=0.25)  # exercise the audit planes of the scratch too
    code = amr.SUM if op == "sum" else amr.WMEAN
    kw = dict(field=1, weight=0, los=True) if op == "wmean" else {}
    # two calls in a row, the second smaller (its scratch holds the first's leftovers)
    for W, H in ((640, 480), (200, 136)):
        cam = amr.set_camera(amrgen.disk_camera(60.0, W, H, max_level=14), T)
        (o0, a0, s0, l0), (o1, a1, s1, l1) = _pair(lod, amr, T, m, cam, code, kw)
        assert np.array_equal(o0.view(np.int32), o1.view(np.int32)), (W, H)
        if a0 is not None:
            assert np.array_equal(a0.view(np.int32), a1.view(np.int32)), (W, H)
        assert np.array_equal(s0, s1) and np.array_equal(l0, l1), (W, H)
        assert s1[0] == lod.tiles(W, H) and s1[2] > 0
        print(op, W, H, "stats", s1.tolist(), flush=True)
    # forced levels through the fixed scratch as well
    cam = amr.set_camera(amrgen.disk_camera(60.0, 200, 136, max_level=14), T)
    forced = torch.full((lod.tiles(200, 136),), 7, dtype=torch.int8, device="cuda")
    (o0, _, s0, _), (o1, _, s1, _) = _pair(lod, amr, T, m, cam, code, kw, forced=forced)
    assert np.array_equal(o0.view(np.int32), o1.view(np.int32)) and np.array_equal(s0, s1)


def test_noalloc_lod_render_rejects_images_beyond_the_scratch():
    import paper_1210_8014_amd as amr
    from paper_1210_8014_amd import lod

    T = amr.Tree(amrgen.disk(seed=6, lmax=12, m_thr=1e-4))
    m = lod.LodModel(path=lod.MODEL_PATH)
    assert lod.workspace_bytes(2048, 2048) <= lod.noalloc_max_bytes() < lod.workspace_bytes(4096, 4096)
    cam = amr.set_camera(amrgen.disk_camera(45.0, 4096, 4096, max_level=12), T)
    out = torch.empty(4096 * 4096, device="cuda")
    st = torch.zeros(8, dtype=torch.int64, device="cuda")
    with pytest.raises(amr.AmrError) as e:
        lod.render_lod_noalloc(T, cam, amr.SUM, m, out, st)
    assert e.value.status == 5  # AMR_ECAPACITY
