"""Host-side parity of the library (no GPU): the linear-octree builder and the
camera quantiser against the oracle, error handling, and the C ABI exports."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import amrgen
import paper_1210_8014_amd as amr
from paper_1210_8014_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    amr.lib()


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "amr.h")).read()
    names = sorted(set(re.findall(r"\b(amr_[a-z_]+)\(", hdr)))
    assert len(names) >= 10
    lib = ctypes.CDLL(amr.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each
    from paper_1210_8014_amd import lod

    declared = set(_abi.SIGNATURES) | set(lod._SIGS)
    assert set(names) <= declared, set(names) - declared


def test_issue_probe_library_exports_its_calls():
    # the measurement aid built beside the library (not part of the C ABI)
    from paper_1210_8014_amd import build as amr_build

    if not os.path.exists(amr_build.PROBE_LIB):
        pytest.skip("libamrprobe.so not built")
    lib = ctypes.CDLL(amr_build.PROBE_LIB)
    for n in ("amrprobe_kinds", "amrprobe_name", "amrprobe_per_iter", "amrprobe_run"):
        assert hasattr(lib, n), n
    lib.amrprobe_name.restype = ctypes.c_char_p
    assert lib.amrprobe_kinds() >= 10 and lib.amrprobe_per_iter(0) == 32
    assert lib.amrprobe_per_iter(lib.amrprobe_kinds()) == 0
    assert lib.amrprobe_name(0) == b"v_add_u32" and lib.amrprobe_name(-1) == b"invalid"
    # argument errors are returned before any device call
    ms = (ctypes.c_float * 1)()
    lib.amrprobe_run.argtypes = [ctypes.c_int32] * 4 + [ctypes.POINTER(ctypes.c_float)] * 2
    assert lib.amrprobe_run(lib.amrprobe_kinds(), 1, 1, 1, ms, ms) != 0
    assert lib.amrprobe_run(0, 0, 1, 1, ms, ms) != 0


def _cells_by_level(T):
    child, vals, md = T.host_arrays()
    off = np.array(list(T.info.level_offset))
    return child, vals, md, off


def test_builder_layout_matches_oracle_cells_and_values(oracle_lib):
    L = amrgen.random_tree(3, lmax=5, p_refine=0.45, nfields=4)
    L.fields[1:] -= 5.0
    T = amr.Tree(L, host_only=True)
    O = oracle_lib.Tree(L)
    child, vals, md, off = _cells_by_level(T)
    assert T.ncells == O.nodes
    # walk every cell: level-major Morton order, 8 children contiguous
    seen = 0
    for lvl in range(T.lmax + 1):
        n = off[lvl + 1] - off[lvl]
        for k in range(n):
            c = off[lvl] + k
            seen += 1
    assert seen == T.ncells
    # reconstruct coordinates top-down and compare every value with the oracle (bit-exact)
    coords = {0: (0, 0, 0, 0)}
    for c in range(T.ncells):
        lv, x, y, z = coords[c]
        v32, _ = O.lookup(lv, x, y, z)
        assert np.array_equal(vals[:, c], v32), (c, lv, x, y, z)
        if child[c] >= 0:
            assert off[lv + 1] <= child[c] < off[lv + 2]
            for o in range(8):
                coords[child[c] + o] = (lv + 1, 2 * x + (o & 1), 2 * y + ((o >> 1) & 1), 2 * z + ((o >> 2) & 1))
        else:
            assert md[c] == lv
    assert len(coords) == T.ncells
    # within a level, cells are in Morton order
    for lvl in range(T.lmax + 1):
        keys = []
        for c in range(off[lvl], off[lvl + 1]):
            _, x, y, z = coords[c]
            keys.append(sum((((x >> b) & 1) | (((y >> b) & 1) << 1) | (((z >> b) & 1) << 2)) << (3 * b)
                            for b in range(lvl)))
        assert keys == sorted(keys)


def test_builder_is_order_independent():
    L = amrgen.blobs(0)
    a = amr.Tree(L, host_only=True).host_arrays()
    b = amr.Tree(L.permuted(5), host_only=True).host_arrays()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_builder_maxdepth_and_levels():
    L = amrgen.blobs(0)
    T = amr.Tree(L, host_only=True)
    child, vals, md, off = _cells_by_level(T)
    assert T.info.levelmin == 3 and T.info.lmax == 6
    assert md[0] == 6
    for l in range(4):
        assert off[l + 1] - off[l] == 8 ** l
    # maxdepth of a refined cell is the max over its children
    ref = np.nonzero(child >= 0)[0]
    kids = child[ref][:, None] + np.arange(8)[None, :]
    assert np.array_equal(md[ref], md[kids].max(axis=1))


def _bad(lv, x, y, z, v=None):
    n = len(lv)
    v = np.ones((1, n), np.float32) if v is None else v
    return amrgen.Leaves(np.array(lv, np.int32), np.array(x, np.int32), np.array(y, np.int32),
                         np.array(z, np.int32), v)


def test_builder_rejects_bad_leaf_sets():
    c = np.arange(8)
    x, y, z = c & 1, (c >> 1) & 1, (c >> 2) & 1
    cases = [
        (_bad([1] * 7, x[:7], y[:7], z[:7]), _abi.AMR_ETREE),                  # gap
        (_bad([1] * 8 + [0], list(x) + [0], list(y) + [0], list(z) + [0]), _abi.AMR_ETREE),  # overlap
        (_bad([1] * 9, list(x) + [0], list(y) + [0], list(z) + [0]), _abi.AMR_ETREE),        # duplicate
        (_bad([0], [1], [0], [0]), _abi.AMR_ETREE),                            # coordinate out of range
        (_bad([25], [0], [0], [0]), _abi.AMR_EINVAL),                          # level out of range
        (_bad([0], [0], [0], [0], np.array([[np.inf]], np.float32)), _abi.AMR_EINVAL),
    ]
    for leaves, st in cases:
        with pytest.raises(amr.AmrError) as e:
            amr.Tree(leaves, host_only=True)
        assert e.value.status == st
    with pytest.raises(amr.AmrError) as e:
        amr.Tree(amrgen.blobs(0), restrict=[3], host_only=True)
    assert e.value.status == _abi.AMR_EINVAL


def _random_desc(rng):
    eye = rng.uniform(-2.0, 3.0, 3)
    tgt = rng.uniform(0.0, 1.0, 3)
    up = rng.normal(size=3)
    W, H = (int(v) for v in rng.integers(1, 3000, 2))
    if rng.random() < 0.5:
        return amrgen.camera("persp", eye, tgt, up, W, H, fov_y=rng.uniform(0.05, 1.4), max_level=-1,
                             level_bias=int(rng.integers(-2, 3)))
    return amrgen.camera("ortho", eye, tgt, up, W, H, ortho_height=rng.uniform(0.01, 1.2), max_level=-1)


def test_camera_records_match_oracle(oracle_lib):
    rng = np.random.default_rng(0)
    n_ok = 0
    for _ in range(3000):
        d = _random_desc(rng)
        try:
            ref = oracle_lib.set_camera(d, 16)
        except ValueError:
            with pytest.raises(amr.AmrError):
                _set_with_lmax(d, 16)
            continue
        got = _set_with_lmax(d, 16)
        assert got.as_dict() == ref.as_dict(), d
        n_ok += 1
    assert n_ok > 1000
    for name in ("tiny_camera.json", "two_level.json", "persp_axis.json", "persp_oblique.json"):
        import json
        g = json.load(open(os.path.join(ROOT, "tests", "golden", name)))
        c = amr.set_camera(g["camera"])
        for k in ("O", "F", "U", "V"):
            assert list(getattr(c, k)) == g["record"][k], (name, k)
        if "auto_level" in g:
            assert c.max_level == g["auto_level"], name


_lmax_trees = {}


def _set_with_lmax(d, lmax):
    if lmax not in _lmax_trees:
        _lmax_trees[lmax] = amr.Tree(amrgen.uniform(1) if lmax == 1 else _deep_leaf_set(lmax), host_only=True)
    return amr.set_camera(d, _lmax_trees[lmax])


def _deep_leaf_set(lmax):
    """Smallest complete octree with one leaf at depth lmax."""
    lv, xs, ys, zs = [], [], [], []
    for l in range(1, lmax + 1):
        for c in range(1, 8):
            lv.append(l)
            xs.append(c & 1)
            ys.append((c >> 1) & 1)
            zs.append((c >> 2) & 1)
    lv.append(lmax)
    xs.append(0)
    ys.append(0)
    zs.append(0)
    return amrgen.Leaves(np.array(lv, np.int32), np.array(xs, np.int32), np.array(ys, np.int32),
                         np.array(zs, np.int32), np.ones((1, len(lv)), np.float32))


def test_camera_rejections_match_oracle(oracle_lib):
    base = amrgen.camera("persp", (0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0, 1, 0), 64, 64, fov_y=0.5)
    bad = [dict(base, fov_y=2.9), dict(base, eye=[0.5, 0.5, 4.5]), dict(base, target=list(base["eye"])),
           dict(base, up=[0.0, 0.0, 1.0]), dict(base, W=0), dict(base, fov_y=0.0),
           dict(base, kind="ortho", ortho_height=-1.0), dict(base, max_level=25)]
    for b in bad:
        with pytest.raises(ValueError):
            oracle_lib.set_camera(b)
        with pytest.raises(amr.AmrError) as e:
            amr.set_camera(b)
        assert e.value.status == _abi.AMR_EINVAL


def test_render_rejects_bad_arguments_without_gpu():
    T = amr.Tree(amrgen.blobs(0), host_only=True)
    cam = amr.set_camera(amrgen.tiny_camera(), T)
    out = np.zeros(cam.W * cam.H, np.float32)
    with pytest.raises(amr.AmrError) as e:  # host-only trees cannot be rendered
        amr.render(T, cam, amr.SUM, out, stream=0)
    assert e.value.status == _abi.AMR_EINVAL


def _bad_records(cam):
    """Hand-made records outside the integer ranges the kernels rely on, each
    with what it breaks."""
    import copy

    def mod(**kw):
        c = copy.deepcopy(cam)
        for k, v in kw.items():
            if isinstance(v, tuple):
                getattr(c, k)[v[0]] = v[1]
            else:
                setattr(c, k, v)
        return c

    return [("image width 0", mod(W=0)), ("image height 32769", mod(H=32769)),
            ("max_level 25", mod(max_level=25)), ("max_level -1", mod(max_level=-1)), ("kind 2", mod(kind=2)),
            ("origin beyond 2^30", mod(O=(0, 1 << 30))), ("origin below -2^30", mod(O=(1, -(1 << 30) - 1))),
            ("direction at 2^30", mod(F=(2, 1 << 30))),
            ("pixel span beyond 2^30", mod(U=(0, 1 << 25))),
            ("zero orthographic direction", mod(F=(0, 0)) if cam.kind == 1 else mod(kind=1, F=(0, 0)))]


def test_every_out_of_range_record_is_rejected_without_gpu():
    """The camera checks shared by every entry point that walks rays (here
    reached through a host-only stream plan, which needs no GPU): each
    out-of-range record is refused with AMR_EINVAL before any launch."""
    T = amr.Tree(amrgen.blobs(0), host_only=True)
    P = amr.StreamPlan(T, T.ncells, host_only=True)
    for kind in ("ortho", "persp"):
        d = amrgen.tiny_camera() if kind == "ortho" else amrgen.camera(
            "persp", (0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0, 1, 0), 64, 48, fov_y=0.6, max_level=6)
        cam = amr.set_camera(d, T)
        assert P.rect(0, cam)[2] >= 0
        for what, bad in _bad_records(cam):
            if what == "zero orthographic direction":
                bad.F[1] = bad.F[2] = 0
            with pytest.raises(amr.AmrError) as e:
                P.rect(0, bad)
            assert e.value.status == _abi.AMR_EINVAL, what
