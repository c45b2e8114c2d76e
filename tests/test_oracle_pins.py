"""Pins for the CPU oracle against things other than itself: hand-worked
closed forms, exact brute force over every leaf, a textbook grid DDA,
conservation laws and algebraic identities.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import amrgen
from tests import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def two_level_leaves():
    lv = np.ones(8, np.int32)
    c = np.arange(8)
    return amrgen.Leaves(lv, (c & 1).astype(np.int32), ((c >> 1) & 1).astype(np.int32),
                         ((c >> 2) & 1).astype(np.int32), (c + 1).astype(np.float32).reshape(1, 8), 1)


def rand_cams(rng, n, W=3, H=2, inside=False):
    cams = []
    for _ in range(n):
        if inside:
            eye = rng.uniform(0.05, 0.95, 3)
        else:
            eye = rng.uniform(-1.5, 2.5, 3)
        tgt = rng.uniform(0.1, 0.9, 3)
        if np.linalg.norm(tgt - eye) < 1e-3:
            continue
        up = rng.normal(size=3)
        if rng.random() < 0.5:
            cams.append(amrgen.camera("persp", eye, tgt, up, W, H, fov_y=rng.uniform(0.2, 1.2)))
        else:
            cams.append(amrgen.camera("ortho", eye, tgt, up, W, H, ortho_height=rng.uniform(0.2, 1.5)))
    return cams


def degenerate_cams():
    """Rays along cell faces and edges, grazing the box, missing it, and
    starting on a face or inside the box."""
    cams = []
    for axis in range(3):
        for sgn in (1, -1):
            f = np.zeros(3)
            f[axis] = sgn
            eye = np.full(3, 0.5)
            eye[axis] = 0.5 - 1.0 * sgn
            up = np.zeros(3)
            up[(axis + 1) % 3] = 1.0
            # 5x5 pixels of 0.25 box: centres on level-2 faces (0, .25, .5, .75, 1)
            cams.append(amrgen.camera("ortho", eye, eye + f, up, 5, 5, ortho_height=1.25))
            # 4x4 pixels of 0.25 box: centres inside cells
            cams.append(amrgen.camera("ortho", eye, eye + f, up, 4, 4, ortho_height=1.0))
    # diagonal through box corners, eye on a face, eye inside, looking away
    cams.append(amrgen.camera("persp", (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5), (0, 0, 1), 1, 1, fov_y=0.5))
    cams.append(amrgen.camera("persp", (0.5, 0.25, 0.0), (0.5, 0.25, 1.0), (0, 1, 0), 3, 3, fov_y=1.0))
    cams.append(amrgen.camera("persp", (0.3, 0.6, 0.45), (0.9, 0.1, 0.2), (0, 1, 0), 3, 3, fov_y=1.2))
    cams.append(amrgen.camera("persp", (0.5, 0.5, 2.0), (0.5, 0.5, 3.0), (0, 1, 0), 3, 3, fov_y=1.0))
    cams.append(amrgen.camera("ortho", (1.0, 0.5, -1.0), (1.0, 0.5, 1.0), (0, 1, 0), 3, 1, ortho_height=0.5))
    cams.append(amrgen.camera("ortho", (0.25, 0.75, 1.5), (0.25, 0.75, 0.5), (1, 0, 0), 1, 1, ortho_height=0.5))
    return cams


def check_against_bruteforce(oracle, T, leaves, camd):
    cam = T.camera(camd)
    rays = np.arange(cam.W * cam.H)
    offs, cells, tq = T.trace(cam, rays, with_t=True)
    tc = bf.truncated_cells(leaves.level, leaves.ix, leaves.iy, leaves.iz, cam.max_level)
    for r in rays:
        o, d = oracle.pixel_ray(cam, r % cam.W, r // cam.W)
        ref = bf.brute_segments(tc, o.tolist(), d.tolist())
        got = cells[offs[r]:offs[r + 1]]
        assert len(ref) == len(got), (camd, r)
        for (c, t0, t1), g, q in zip(ref, got, tq[offs[r]:offs[r + 1]]):
            assert tuple(int(v) for v in g) == c
            assert Fraction(int(q[0]), int(q[1])) == t0
            assert Fraction(int(q[2]), int(q[3])) == t1


# ------------------------------------------------------------------ golden

def test_golden_two_level(oracle_lib):
    g = _golden("two_level.json")
    L = two_level_leaves()
    T = oracle_lib.Tree(L)
    cam = T.camera(g["camera"])
    for k in ("O", "F", "U", "V"):
        assert list(getattr(cam, k)) == g["record"][k]
    offs, cells, _ = T.trace(cam, np.array([0]))
    assert cells.tolist() == g["cells"]
    assert T.render(cam, oracle_lib.SUM)["val"][0] == g["sum"]
    assert T.render(cam, oracle_lib.MAX)["max"][0] == g["max"]
    d0 = dict(g["camera"], max_level=0)
    cam0 = T.camera(d0)
    assert T.render(cam0, oracle_lib.SUM)["val"][0] == g["sum_level0"]
    assert T.render(cam0, oracle_lib.MAX)["max"][0] == g["max_level0"]


def test_golden_tiny_camera(oracle_lib):
    g = _golden("tiny_camera.json")
    cam = oracle_lib.set_camera(g["camera"])
    for k in ("O", "F", "U", "V"):
        assert list(getattr(cam, k)) == g["record"][k]
    assert cam.max_level == g["auto_level"]
    assert oracle_lib.set_camera(g["camera"], 6).max_level == 6
    # pixel (i, j) starts at its centre, (2i + 1) 2^19 units
    for i, j in [(0, 0), (255, 0), (17, 200), (255, 255)]:
        o, d = oracle_lib.pixel_ray(cam, i, j)
        assert o.tolist() == [(2 * i + 1) << 19, (2 * j + 1) << 19, -(1 << 27)]
        assert d.tolist() == [0, 0, 1 << 28]


@pytest.mark.parametrize("name", ["persp_axis.json", "persp_oblique.json"])
def test_golden_perspective_records(oracle_lib, name):
    """Hand-derived perspective records: pins the half-pixel step
    tan(fov_y/2)/H (vertical field of view), the image axes and the
    automatic level."""
    g = _golden(name)
    cam = oracle_lib.set_camera(g["camera"])
    for k in ("O", "F", "U", "V"):
        assert list(getattr(cam, k)) == g["record"][k], k
    assert cam.max_level == g["auto_level"]
    # pixel (0, 0) looks through the lower-left pixel centre: a = 1 - W, b = 1 - H
    o, d = oracle_lib.pixel_ray(cam, 0, 0)
    W, H = g["camera"]["W"], g["camera"]["H"]
    F, U, V = (np.array(g["record"][k]) for k in ("F", "U", "V"))
    assert o.tolist() == g["record"]["O"]
    assert d.tolist() == (F + (1 - W) * U + (1 - H) * V).tolist()


def test_field_of_view_edge_ray(oracle_lib):
    """The top edge of the image (b = H) lies fov_y/2 off the view axis and
    the right edge (a = W) atan(W/H tan(fov_y/2)) off it, to within the
    rounding of the integer record: |H |V| / |F| - tan(fov_y/2)| is at most
    (H + 1) sqrt(3)/2 / (|F| - 1)."""
    rng = np.random.default_rng(7)
    n = 0
    for _ in range(400):
        eye = rng.uniform(-1.0, 2.0, 3)
        tgt = rng.uniform(0.2, 0.8, 3)
        W, H = (int(v) for v in rng.integers(1, 4000, 2))
        fov = rng.uniform(0.05, 1.5)
        d = amrgen.camera("persp", eye, tgt, rng.normal(size=3), W, H, fov_y=fov)
        try:
            c = oracle_lib.set_camera(d)
        except ValueError:
            continue
        F, U, V = (np.array(list(getattr(c, k)), np.float64) for k in ("F", "U", "V"))
        nF = np.linalg.norm(F)
        bound = (H + 1) * math.sqrt(3) / 2 / (nF - 1)
        assert abs(H * np.linalg.norm(V) / nF - math.tan(fov / 2)) <= bound + 1e-15
        assert abs(H * np.linalg.norm(U) / nF - math.tan(fov / 2)) <= bound + 1e-15
        # the three axes are orthogonal to within the rounding
        assert abs(F @ U) <= 0.87 * (np.abs(F).sum() + np.abs(U).sum())
        assert abs(F @ V) <= 0.87 * (np.abs(F).sum() + np.abs(V).sum())
        n += 1
    assert n > 300


def test_camera_rejects(oracle_lib):
    base = amrgen.camera("persp", (0.5, 0.5, 2.0), (0.5, 0.5, 0.5), (0, 1, 0), 64, 64, fov_y=0.5)
    oracle_lib.set_camera(base)
    bad = [dict(base, fov_y=2.9),                            # directions beyond 2^30
           dict(base, eye=[0.5, 0.5, 4.5]),                 # eye outside [-4, 4)
           dict(base, target=list(base["eye"])),            # zero view direction
           dict(base, up=[0.0, 0.0, 1.0]),                  # up parallel to the view
           dict(base, W=0), dict(base, fov_y=0.0),
           dict(base, kind="ortho", ortho_height=-1.0),
           dict(base, max_level=25)]
    for b in bad:
        with pytest.raises(ValueError):
            oracle_lib.set_camera(b)


def test_camera_auto_level_perspective(oracle_lib):
    # footprint 2 D tan(fov/2) / H with D = 1.02, tan = 0.5, H = 2^k -> 1.02 * 2^-k
    for k in range(3, 12):
        d = amrgen.camera("persp", (0.5, 0.5, 1.52), (0.5, 0.5, 0.5), (0, 1, 0), 1 << k, 1 << k,
                          fov_y=2 * math.atan(0.5))
        assert oracle_lib.set_camera(d).max_level == k
        assert oracle_lib.set_camera(dict(d, level_bias=-1)).max_level == k - 1
        assert oracle_lib.set_camera(d, 5).max_level == min(k, 5)


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("seed", range(6))
def test_segments_match_bruteforce_random(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    L = amrgen.random_tree(seed, lmax=4, p_refine=0.4)
    T = oracle_lib.Tree(L)
    for camd in rand_cams(rng, 6, inside=(seed % 2 == 1)):
        for ml in (T.lmax, max(0, T.lmax - 2)):
            check_against_bruteforce(oracle_lib, T, L, dict(camd, max_level=ml))


@pytest.mark.parametrize("seed", range(3))
def test_segments_match_bruteforce_degenerate(oracle_lib, seed):
    L = amrgen.random_tree(100 + seed, lmax=4, p_refine=0.45)
    T = oracle_lib.Tree(L)
    for camd in degenerate_cams():
        for ml in (T.lmax, 2):
            check_against_bruteforce(oracle_lib, T, L, dict(camd, max_level=ml))


def test_values_match_bruteforce(oracle_lib):
    """Sum and max recomputed from brute-force segments and the input leaf
    values (no truncation, so no restriction involved)."""
    rng = np.random.default_rng(7)
    L = amrgen.random_tree(7, lmax=4, p_refine=0.4)
    T = oracle_lib.Tree(L)
    val = {(int(a), int(b), int(c), int(d)): float(v)
           for a, b, c, d, v in zip(L.level, L.ix, L.iy, L.iz, L.fields[0])}
    cells = list(val.keys())
    for camd in rand_cams(rng, 6, W=4, H=3) + degenerate_cams()[:4]:
        cam = T.camera(dict(camd, max_level=T.lmax))
        s = T.render(cam, oracle_lib.SUM)["val"]
        m = T.render(cam, oracle_lib.MAX)["max"]
        for r in range(cam.W * cam.H):
            o, d = oracle_lib.pixel_ray(cam, r % cam.W, r // cam.W)
            segs = bf.brute_segments(cells, o.tolist(), d.tolist())
            u = bf.ray_length_unit(d.tolist())
            ref = math.fsum(val[c] * float(t1 - t0) * u for c, t0, t1 in segs)
            assert s[r] == pytest.approx(ref, rel=1e-13, abs=1e-300)
            refm = max((np.float32(val[c]) for c, _, _ in segs), default=np.float32(-np.inf))
            assert m[r] == refm


# ------------------------------------------------------------ textbook DDA

@pytest.mark.parametrize("level", [1, 2, 3])
def test_uniform_tree_matches_grid_dda(oracle_lib, level):
    L = amrgen.uniform(level, seed=level)
    T = oracle_lib.Tree(L)
    rng = np.random.default_rng(level)
    for camd in rand_cams(rng, 5, W=3, H=3) + degenerate_cams():
        cam = T.camera(dict(camd, max_level=level))
        rays = np.arange(cam.W * cam.H)
        offs, cells, tq = T.trace(cam, rays, with_t=True)
        for r in rays:
            o, d = oracle_lib.pixel_ray(cam, r % cam.W, r // cam.W)
            ref = bf.grid_dda(level, o.tolist(), d.tolist())
            got = cells[offs[r]:offs[r + 1]]
            assert [c for c, _, _ in ref] == [tuple(int(v) for v in g) for g in got]
            assert [(a, b) for _, a, b in ref] == [
                (Fraction(int(q[0]), int(q[1])), Fraction(int(q[2]), int(q[3]))) for q in tq[offs[r]:offs[r + 1]]]


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("level", [2, 4, 5])
def test_axis_aligned_ray_crosses_2_to_the_l_cells(oracle_lib, level):
    L = amrgen.uniform(level, values=np.ones(8 ** level))
    T = oracle_lib.Tree(L)
    cam = T.camera(amrgen.tiny_camera(32, 32, max_level=level))
    r = T.render(cam, oracle_lib.SUM)
    assert np.all(r["count"] == 2 ** level)
    assert np.all(r["val"] == 1.0)


@pytest.mark.parametrize("level", [1, 3, 5])
def test_diagonal_ray_crosses_2_to_the_l_cells(oracle_lib, level):
    L = amrgen.uniform(level, seed=3)
    T = oracle_lib.Tree(L)
    cam = T.camera(amrgen.camera("persp", (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5), (0, 0, 1), 1, 1, fov_y=0.5,
                                 max_level=level))
    offs, cells, _ = T.trace(cam, np.array([0]))
    assert cells.tolist() == [[level, i, i, i] for i in range(2 ** level)]


def test_constant_field_sum_is_value_times_box_chord(oracle_lib):
    rng = np.random.default_rng(11)
    L = amrgen.random_tree(11, lmax=5, p_refine=0.45)
    L.fields[:] = np.float32(0.7)
    T = oracle_lib.Tree(L)
    for camd in rand_cams(rng, 8, W=8, H=8) + degenerate_cams():
        for ml in (T.lmax, 1):
            cam = T.camera(dict(camd, max_level=ml))
            s = T.render(cam, oracle_lib.SUM)["val"]
            for r in range(cam.W * cam.H):
                o, d = oracle_lib.pixel_ray(cam, r % cam.W, r // cam.W)
                lb = bf.box_chord(o.tolist(), d.tolist())
                assert s[r] == pytest.approx(float(np.float32(0.7)) * lb, rel=1e-14, abs=1e-300)


def test_mass_conserved_at_every_truncation_level(oracle_lib):
    """Orthographic, full domain, pixels finer than the finest cell: the
    image-integrated column times the pixel area is the total mass, at every
    maximum level (restriction conserves mass).  Truncated cells carry fp32
    roundings of the fp64 restricted values, so the identity holds to 2^-24
    relative; without truncation it holds to fp64 rounding."""
    L = amrgen.blobs(0)
    T = oracle_lib.Tree(L)
    mass = math.fsum((L.fields[0].astype(np.float64) * 8.0 ** (-L.level)).tolist())
    for ml in range(0, T.lmax + 1):
        cam = T.camera(amrgen.tiny_camera(64, 64, max_level=ml))
        s = T.render(cam, oracle_lib.SUM)["val"]
        tol = 1e-12 if ml == T.lmax else 2.0 ** -24
        assert math.fsum(s.tolist()) / 64 ** 2 == pytest.approx(mass, rel=tol)


def test_momentum_conserved_at_every_truncation_level(oracle_lib):
    """Mass-weighted restriction conserves momentum: sum over pixels of
    wmean * weight * area equals sum over leaves of rho v V."""
    L = amrgen.random_tree(5, lmax=4, p_refine=0.5, nfields=4)
    L.fields[1:] -= 5.0  # signed velocities
    T = oracle_lib.Tree(L)
    for comp in (1, 2, 3):
        mom = math.fsum((L.fields[0].astype(np.float64) * L.fields[comp].astype(np.float64)
                         * 8.0 ** (-L.level)).tolist())
        for ml in range(0, T.lmax + 1):
            cam = T.camera(amrgen.tiny_camera(16, 16, max_level=ml))
            r = T.render(cam, oracle_lib.WMEAN, field=comp, weight=0)
            tol = 1e-11 if ml == T.lmax else 2.0 ** -22  # fp32 roundings of rho and v
            got = math.fsum((r["val"] * r["aux"]).tolist()) / 16 ** 2
            scale = math.fsum((L.fields[0].astype(np.float64) * np.abs(L.fields[comp].astype(np.float64))
                               * 8.0 ** (-L.level)).tolist())
            assert abs(got - mom) <= tol * scale


def test_uniform_tree_equals_dense_grid_sum(oracle_lib):
    level = 3
    L = amrgen.uniform(level, seed=9)
    T = oracle_lib.Tree(L)
    n = 2 ** level
    grid = np.zeros((n, n, n))
    grid[L.iz, L.iy, L.ix] = L.fields[0]
    cam = T.camera(amrgen.tiny_camera(16, 16, max_level=level))
    s = T.render(cam, oracle_lib.SUM)["val"].reshape(16, 16)
    dense = grid.sum(axis=0) / n  # column sums times the cell side, indexed [y, x]
    assert np.allclose(s, np.repeat(np.repeat(dense, 2, axis=0), 2, axis=1), rtol=1e-14)


# ------------------------------------------------------------ wmean identities

def test_wmean_identities(oracle_lib):
    rng = np.random.default_rng(3)
    L = amrgen.random_tree(21, lmax=4, p_refine=0.45, nfields=3)
    L.fields[2] = np.float32(2.5)
    T = oracle_lib.Tree(L, restrict=[-1, 0, 0])
    for camd in rand_cams(rng, 6, W=6, H=5):
        cam = T.camera(dict(camd, max_level=T.lmax))
        const = T.render(cam, oracle_lib.WMEAN, field=2, weight=0)
        hit = const["aux"] > 0
        assert np.allclose(const["val"][hit], 2.5, rtol=1e-14)
        assert np.all(const["val"][~hit] == 0.0)
        r = T.render(cam, oracle_lib.WMEAN, field=1, weight=0)
        mx = T.render(cam, oracle_lib.MAX, field=1)["max"]
        offs, cells, _ = T.trace(cam, np.arange(cam.W * cam.H))
        for k in np.nonzero(hit)[0]:
            vs = [T.lookup(*c)[0][1] for c in cells[offs[k]:offs[k + 1]]]
            assert min(vs) - 1e-6 <= r["val"][k] <= max(vs) + 1e-6
            assert max(vs) == mx[k]


def test_wmean_unit_weight_is_sum_over_length(oracle_lib):
    rng = np.random.default_rng(4)
    L = amrgen.random_tree(22, lmax=4, p_refine=0.45, nfields=2)
    L.fields[0] = np.float32(1.0)
    T = oracle_lib.Tree(L, restrict=[-1, -1])
    for camd in rand_cams(rng, 6, W=5, H=5):
        cam = T.camera(dict(camd, max_level=T.lmax))
        w = T.render(cam, oracle_lib.WMEAN, field=1, weight=0)
        s = T.render(cam, oracle_lib.SUM, field=1)["val"]
        for r in range(cam.W * cam.H):
            o, d = oracle_lib.pixel_ray(cam, r % cam.W, r // cam.W)
            lb = bf.box_chord(o.tolist(), d.tolist())
            if lb > 0:
                assert w["val"][r] == pytest.approx(s[r] / lb, rel=1e-13)
                assert w["aux"][r] == pytest.approx(lb, rel=1e-13)


def test_los_velocity_picks_the_view_component(oracle_lib):
    L = amrgen.random_tree(23, lmax=3, p_refine=0.5, nfields=4)
    L.fields[1:] -= 5.0
    T = oracle_lib.Tree(L)
    for axis in range(3):
        for sgn in (1.0, -1.0):
            eye = np.full(3, 0.5)
            eye[axis] -= 1.0 * sgn
            tgt = np.full(3, 0.5)
            up = np.zeros(3)
            up[(axis + 1) % 3] = 1.0
            cam = T.camera(amrgen.camera("ortho", eye, tgt, up, 8, 8, ortho_height=1.0, max_level=3))
            a = T.render(cam, oracle_lib.WMEAN, field=1, weight=0, los=True)["val"]
            b = T.render(cam, oracle_lib.WMEAN, field=1 + axis, weight=0)["val"]
            assert np.allclose(a, sgn * b, rtol=1e-14, atol=1e-12)


# ------------------------------------------------------------ truncation

def test_truncation_equals_rendering_the_collapsed_tree(oracle_lib):
    L = amrgen.random_tree(31, lmax=5, p_refine=0.5)
    T = oracle_lib.Tree(L)
    rng = np.random.default_rng(31)
    for ml in range(0, T.lmax):
        cells = bf.truncated_cells(L.level, L.ix, L.iy, L.iz, ml)
        arr = np.array(cells, np.int32)
        vals = np.array([[T.lookup(*c)[0][0] for c in cells]], np.float32)
        C = oracle_lib.Tree(amrgen.Leaves(arr[:, 0].copy(), arr[:, 1].copy(), arr[:, 2].copy(), arr[:, 3].copy(), vals))
        for camd in rand_cams(rng, 3, W=8, H=8):
            c1 = T.camera(dict(camd, max_level=ml))
            c2 = C.camera(dict(camd, max_level=24))
            a = T.render(c1, oracle_lib.SUM)
            b = C.render(c2, oracle_lib.SUM)
            assert np.array_equal(a["val"], b["val"]) and np.array_equal(a["count"], b["count"])
            assert np.array_equal(T.render(c1, oracle_lib.MAX)["max"], C.render(c2, oracle_lib.MAX)["max"])


def test_mirrored_view_gives_mirrored_image(oracle_lib):
    L = amrgen.blobs(0)
    T = oracle_lib.Tree(L)
    a = T.camera(amrgen.camera("ortho", (0.5, 0.5, -0.5), (0.5, 0.5, 0.5), (0, 1, 0), 64, 64, ortho_height=1.0,
                               max_level=6))
    b = T.camera(amrgen.camera("ortho", (0.5, 0.5, 1.5), (0.5, 0.5, 0.5), (0, 1, 0), 64, 64, ortho_height=1.0,
                               max_level=6))
    ma = T.render(a, oracle_lib.MAX)["max"].reshape(64, 64)
    mb = T.render(b, oracle_lib.MAX)["max"].reshape(64, 64)
    assert np.array_equal(ma, mb[:, ::-1])
    sa = T.render(a, oracle_lib.SUM)["val"].reshape(64, 64)
    sb = T.render(b, oracle_lib.SUM)["val"].reshape(64, 64)
    assert np.allclose(sa, sb[:, ::-1], rtol=1e-14)


# ------------------------------------------------------------ tree validation

def test_tree_rejects_bad_leaf_sets(oracle_lib):
    L = two_level_leaves()

    def mk(lv, x, y, z, v=None):
        n = len(lv)
        v = np.ones((1, n), np.float32) if v is None else v
        return amrgen.Leaves(np.array(lv, np.int32), np.array(x, np.int32), np.array(y, np.int32),
                             np.array(z, np.int32), v)

    with pytest.raises(ValueError):  # gap: one octant missing
        oracle_lib.Tree(mk(L.level[:7], L.ix[:7], L.iy[:7], L.iz[:7]))
    with pytest.raises(ValueError):  # overlap: the root and its children
        oracle_lib.Tree(mk(list(L.level) + [0], list(L.ix) + [0], list(L.iy) + [0], list(L.iz) + [0]))
    with pytest.raises(ValueError):  # duplicate leaf
        oracle_lib.Tree(mk(list(L.level) + [1], list(L.ix) + [0], list(L.iy) + [0], list(L.iz) + [0]))
    with pytest.raises(ValueError):  # coordinate outside 0..2^l-1
        oracle_lib.Tree(mk([0], [1], [0], [0]))
    with pytest.raises(ValueError):  # NaN field
        oracle_lib.Tree(mk([0], [0], [0], [0], np.array([[np.nan]], np.float32)))
    T = oracle_lib.Tree(L.permuted(3))
    assert T.nodes == 9


# ------------------------------------------------- hand-worked sums

def _leaves_level(level, fields_of):
    """Uniform level-`level` tree; fields_of(ix, iy, iz) -> list of fields."""
    n = 1 << level
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    vals = np.array([fields_of(int(a), int(b), int(c)) for a, b, c in zip(ix, iy, iz)], np.float32).T
    return amrgen.Leaves(np.full(ix.size, level, np.int32), ix.astype(np.int32), iy.astype(np.int32),
                         iz.astype(np.int32), np.ascontiguousarray(vals), vals.shape[0])


def test_golden_wmean_three_cells(oracle_lib):
    """Hand-worked sum, maximum, line-of-sight weighted mean and both of its
    error scales on three cells (pins the projection, the weights and the
    absf / absdot scales term by term)."""
    g = _golden("wmean_three_cells.json")
    cells = {tuple(int(v) for v in k.split(",")): v for k, v in g["cells"].items()}
    L = _leaves_level(1, lambda a, b, c: cells.get((a, b, c), g["other"]))
    T = oracle_lib.Tree(L)
    cam = T.camera(g["camera"])
    e = g["expect"]
    r2 = math.sqrt(2.0)
    s = T.render(cam, oracle_lib.SUM)
    assert s["count"][0] == e["count"]
    assert s["val"][0] == pytest.approx(e["sum_over_sqrt2"] * r2, rel=1e-15)
    assert T.render(cam, oracle_lib.MAX)["max"][0] == e["max"]
    w = T.render(cam, oracle_lib.WMEAN, field=1, weight=0, los=True)
    assert w["val"][0] == pytest.approx(e["wmean_over_sqrt2"] * r2, rel=1e-14)
    assert w["aux"][0] == pytest.approx(e["weight_over_sqrt2"] * r2, rel=1e-15)
    assert w["absf"][0] == pytest.approx(e["absf_over_sqrt2"] * r2, rel=1e-14)
    assert w["absdot"][0] == pytest.approx(e["absdot_over_sqrt2"] * r2, rel=1e-14)
    sc = T.render(cam, oracle_lib.WMEAN, field=1, weight=0, los=False)
    assert abs(sc["val"][0]) <= 1e-15
    assert sc["absf"][0] == pytest.approx(e["scalar_vx"]["absf"], rel=1e-15)
    assert sc["absdot"][0] == pytest.approx(e["scalar_vx"]["absf"], rel=1e-15)


def test_golden_cancelling_sum_needs_compensation(oracle_lib):
    """A sum whose exact value plain fp64 accumulation loses: the oracle's
    compensated sum returns it exactly (pins the compensation)."""
    g = _golden("cancelling_sum.json")
    pat = g["pattern"]
    L = _leaves_level(g["level"], lambda a, b, c: [pat[a % 4]])
    T = oracle_lib.Tree(L)
    cam = T.camera(g["camera"])
    r = T.render(cam, oracle_lib.SUM)
    assert r["count"][0] == 1 << g["level"]
    assert r["val"][0] == g["expect"]["sum"]
    # the fixture's premise: plain left-to-right fp64 gets it wrong
    acc = 0.0
    for k in range(1 << g["level"]):
        acc += float(np.float32(pat[k % 4])) * 2.0 ** -g["level"]
    assert acc == g["expect"]["plain_left_to_right"]
