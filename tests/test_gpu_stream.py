"""GPU parity of the streamed render (trees kept in host memory, streamed
through the GPU in chunks) through amr_render_streamed: values against the
oracle on the same seeded inputs (bars in tests/parity.py), the maximum
bit-identical to the in-memory render, back-to-back renders on one plan,
and the argument checks.  Run on an MI355X: pytest -m gpu."""
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


def log(*a):
    print(*a, flush=True)


class StreamedRenderer:
    """Values from amr_render_streamed over a plan of `cap` cells per chunk;
    cell counts and sequences from the in-memory library tree (the streamed
    walk's own cells are checked against the oracle on the CPU).  Every MAX
    image must equal the in-memory render bit for bit."""

    def __init__(self, leaves, cap, restrict=None):
        import paper_1210_8014_amd as amr
        from tests.gpu_render import GpuRenderer

        H = amr.Tree(leaves, restrict=restrict, host_only=True)
        self.P = amr.StreamPlan(H, cap)
        self.lmax = H.lmax
        H.close()
        self.G = GpuRenderer(leaves, restrict=restrict)
        self.stats = []

    @property
    def chunk_level(self):
        return int(self.P.info.max_chunk_level)

    def camera(self, d):
        return self.G.camera(d)

    def full(self, cam, op, field=0, weight=0, los=False):
        import paper_1210_8014_amd as amr

        n = cam.W * cam.H
        out = torch.full((n,), -7.0, dtype=torch.float32, device="cuda")
        aux = torch.full((n,), -7.0, dtype=torch.float32, device="cuda") if op == amr.WMEAN else None
        ws = torch.empty(amr.StreamPlan.workspace_bytes(cam.W, cam.H) // 4, dtype=torch.float32, device="cuda")
        self.stats.append(self.P.render(cam, op, out, ws, aux, field=field, weight=weight, los=los))
        torch.cuda.synchronize()
        return out.cpu().numpy(), (aux.cpu().numpy() if aux is not None else None)

    def render(self, cam, op, field=0, weight=0, los=False, rays=None):
        import paper_1210_8014_amd as amr

        out, aux = self.full(cam, op, field, weight, los)
        ref, _ = self.G.full(cam, op, field, weight, los)
        if op == amr.MAX:
            assert np.array_equal(out.view(np.int32), ref.view(np.int32)), "streamed max differs from in-memory"
        cnt, _ = self.G.counts(cam)
        if rays is not None:
            out, cnt = out[rays], cnt[rays]
            aux = aux[rays] if aux is not None else None
        return out, aux, cnt

    def trace(self, cam, rays):
        return self.G.trace(cam, rays)

    def close(self):
        self.P.close()
        self.G.T.close()


@pytest.mark.parametrize("seed", range(3))
def test_gpu_streamed_random_trees(seed):
    rng = np.random.default_rng(70 + seed)
    L = amrgen.random_tree(600 + seed, lmax=6, p_refine=0.42, levelmin=3, nfields=4)
    L.fields[1:] -= 5.0
    OT = oracle.Tree(L)
    cams = rand_cams(rng, 5, W=21, H=17, inside=(seed % 2 == 1)) + degenerate_cams()
    for frac in (8, 40):
        log("seed", seed, "chunks of", len(L.level) // frac)
        R = StreamedRenderer(L, max(len(L.level) // frac, 400))
        assert R.P.nchunks > 1
        for camd in cams:
            for ml in sorted({OT.lmax, R.chunk_level}):
                if ml < R.chunk_level:
                    continue
                d = dict(camd, max_level=ml)
                n = d["W"] * d["H"]
                parity.compare_all(R, OT, d, ops=("sum", "max", "wmean"), los_fields=(1, 0, True),
                                   trace_rays=np.arange(n)[::4], what=f"streamed/{frac} seed{seed} ml{ml}")
        R.close()


def test_gpu_streamed_tiny_full_image_and_fields():
    """256^2 orthographic image of the tiny scene over chunks of levels up to
    3, every op, a non-zero sum field and a scalar weighted mean (the
    per-field arrays instead of the interleaved records)."""
    import paper_1210_8014_amd as amr

    L = amrgen.scene("tiny")
    OT = oracle.Tree(L)
    R = StreamedRenderer(L, 1500)
    assert R.chunk_level >= 2
    d = amrgen.tiny_camera(256, 256, 6)
    parity.compare_all(R, OT, d, ops=("sum", "max"), trace_rays=np.arange(256 * 256)[::97], what="streamed tiny")
    R.close()
    # positive fields: the relative bar of a sum assumes no cancellation
    L = amrgen.random_tree(77, lmax=6, p_refine=0.42, levelmin=3, nfields=4)
    assert (L.fields > 0).all()
    OT = oracle.Tree(L)
    R = StreamedRenderer(L, len(L.level) // 30)
    rng = np.random.default_rng(3)
    for camd in rand_cams(rng, 3, W=40, H=30):
        cam, ocam = R.camera(camd), OT.camera(camd)
        got, _ = R.full(cam, amr.SUM, field=2)
        parity.check_sum(got, OT.render(ocam, oracle.SUM, field=2)["val"], "streamed sum of field 2")
        got, _ = R.full(cam, amr.MAX, field=3)
        parity.check_max(got, OT.render(ocam, oracle.MAX, field=3)["max"], "streamed max of field 3")
        got, aux = R.full(cam, amr.WMEAN, field=3, weight=1, los=False)
        parity.check_wmean(got, aux, OT.render(ocam, oracle.WMEAN, field=3, weight=1, los=False),
                           "streamed wmean of field 3 by field 1")
    R.close()


def test_gpu_streamed_disk_sampled_and_back_to_back():
    """The galaxy disk (20.5M leaves) cut into chunks of at most 2M cells:
    the three 2048^2 views against the oracle on a seeded 1% ray sample,
    the maximum bit-identical to the in-memory render, and three renders
    queued back to back on one plan (buffers reused through its events)
    equal to the same renders one at a time."""
    import paper_1210_8014_amd as amr

    L = amrgen.scene("disk")
    OT = oracle.Tree(L)
    R = StreamedRenderer(L, 2_000_000)
    I = R.P.info
    log("disk plan", I.nchunks, "chunks, levels", I.min_chunk_level, "-", I.max_chunk_level, "device MB",
        I.device_bytes / 1e6)
    # four buffers of 2M cells (40 B each) against the ~45 B per cell the tree needs in memory
    assert I.nchunks >= 10 and I.nbuffers == 4 and I.device_bytes < 0.35 * 45 * len(L.level)
    n = 2048 * 2048
    rays = np.sort(np.random.default_rng(1).choice(n, n // 100, replace=False))
    descs = amrgen.disk_cameras()
    for k, camd in enumerate(descs):
        log("disk camera", k)
        parity.compare_all(R, OT, camd, ops=("sum", "max", "wmean"), rays=rays, los_fields=(1, 0, True),
                           what=f"streamed disk cam{k}")
        st = R.stats[-1]
        assert 0 < st[0] <= I.nchunks
    # back to back
    cams = [R.camera(d) for d in descs]
    jobs = [(cams[0], amr.SUM, {}), (cams[1], amr.WMEAN, dict(field=1, weight=0, los=True)), (cams[2], amr.MAX, {})]
    singles = [R.full(c, op, **kw) for c, op, kw in jobs]
    outs, auxs, wss = [], [], []
    for c, op, kw in jobs:
        outs.append(torch.full((n,), -7.0, device="cuda"))
        auxs.append(torch.full((n,), -7.0, device="cuda") if op == amr.WMEAN else None)
        wss.append(torch.empty(amr.StreamPlan.workspace_bytes(c.W, c.H) // 4, device="cuda"))
        R.P.render(c, op, outs[-1], wss[-1], auxs[-1], **kw)
    torch.cuda.synchronize()
    for (a, x), o, ax in zip(singles, outs, auxs):
        assert np.array_equal(a.view(np.int32), o.cpu().numpy().view(np.int32))
        if x is not None:
            assert np.array_equal(x.view(np.int32), ax.cpu().numpy().view(np.int32))
    R.close()


def test_gpu_streamed_rejects():
    import paper_1210_8014_amd as amr

    L = amrgen.random_tree(9, lmax=6, p_refine=0.45, levelmin=3, nfields=1)
    H = amr.Tree(L, host_only=True)
    P = amr.StreamPlan(H, len(L.level) // 20)
    lc = int(P.info.max_chunk_level)
    assert lc >= 1
    cam = amr.set_camera(amrgen.tiny_camera(32, 32, lc - 1))
    out = torch.empty(32 * 32, device="cuda")
    ws = torch.empty(amr.StreamPlan.workspace_bytes(32, 32) // 4, device="cuda")
    with pytest.raises(amr.AmrError) as e:
        P.render(cam, amr.SUM, out, ws)  # shallower than the deepest chunk
    assert e.value.status == amr._abi.AMR_EINVAL
    cam = amr.set_camera(amrgen.tiny_camera(32, 32, 6))
    with pytest.raises(amr.AmrError) as e:
        P.render(cam, amr.SUM, out, ws[:100])
    assert e.value.status == amr._abi.AMR_ECAPACITY
    with pytest.raises(amr.AmrError) as e:
        P.render(cam, amr.WMEAN, out, ws, field=0, weight=0, los=True)  # needs 3 velocity fields
    assert e.value.status == amr._abi.AMR_EINVAL
    with pytest.raises(amr.AmrError) as e:
        amr.StreamPlan(amr.Tree(L), 1000)  # a device tree
    assert e.value.status == amr._abi.AMR_EINVAL
    P.render(cam, amr.SUM, out, ws)
    torch.cuda.synchronize()
    P.close()
    H.close()
