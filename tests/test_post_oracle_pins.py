"""Pins (CPU) for the oracle's slice maps, resolution plane and adaptive
Gaussian post-filter: closed forms, brute force over every leaf and hand-made
cases, independent of the code they check."""
import math

import numpy as np
import pytest

import amrgen
from oracle import post as OP
from tests.test_oracle_pins import degenerate_cams, rand_cams


@pytest.fixture(scope="module")
def O():
    import oracle

    oracle.build()
    return oracle


def _uniform(level, seed=0):
    n = 1 << level
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    vals = (1.0 + ix + 7.0 * iy + 53.0 * iz).astype(np.float32).ravel()[None, :]
    return amrgen.Leaves(np.full(n ** 3, level, np.int32), ix.ravel().astype(np.int32), iy.ravel().astype(np.int32),
                         iz.ravel().astype(np.int32), vals, 1)


def _ortho_cams(rng, n, W=7, H=5):
    return [c for c in rand_cams(rng, 3 * n, W, H) if c["kind"] == "ortho"][:n]


# ------------------------------------------------------------------ slices

def test_slice_uniform_tree_closed_form(O):
    """Uniform level-l tree: the value at point p is that of cell floor(p 2^l)
    (half-open cells), NaN outside the box; faces included."""
    rng = np.random.default_rng(1)
    for level in (0, 2, 3):
        L = _uniform(level)
        T = O.Tree(L)
        cams = _ortho_cams(rng, 6) + [c for c in degenerate_cams() if c["kind"] == "ortho"]
        for d in cams:
            cam = T.camera(dict(d, max_level=level))
            got = T.slice(cam)
            for pix in range(cam.W * cam.H):
                p, _ = O.pixel_ray(cam, pix % cam.W, pix // cam.W)
                if np.any(p < 0) or np.any(p >= 1 << 28):
                    assert np.isnan(got[pix])
                    continue
                c = p >> (28 - level)
                assert got[pix] == np.float32(1.0 + c[0] + 7.0 * c[1] + 53.0 * c[2]), (level, pix)


@pytest.mark.parametrize("seed", range(3))
def test_slice_random_tree_bruteforce(O, seed):
    """Random trees: the leaf whose box holds the point, found by testing
    every leaf, then its ancestor at the truncation level (restricted value
    from the oracle's lookup)."""
    rng = np.random.default_rng(seed)
    L = amrgen.random_tree(300 + seed, lmax=5, p_refine=0.45, nfields=2)
    T = O.Tree(L)
    lo = [L.ix.astype(np.int64) << (28 - L.level), L.iy.astype(np.int64) << (28 - L.level),
          L.iz.astype(np.int64) << (28 - L.level)]
    side = np.int64(1) << (28 - L.level.astype(np.int64))
    for d in _ortho_cams(rng, 4) + [c for c in degenerate_cams() if c["kind"] == "ortho"][:4]:
        for ml in (1, 3, 5):
            cam = T.camera(dict(d, max_level=ml))
            got = T.slice(cam, field=1)
            for pix in range(cam.W * cam.H):
                p, _ = O.pixel_ray(cam, pix % cam.W, pix // cam.W)
                inside = np.ones(L.n, bool)
                for k in range(3):
                    inside &= (lo[k] <= p[k]) & (p[k] < lo[k] + side)
                hits = np.flatnonzero(inside)
                if hits.size == 0:
                    assert np.isnan(got[pix])
                    continue
                assert hits.size == 1
                q = hits[0]
                lv = min(int(L.level[q]), ml)
                sh = int(L.level[q]) - lv
                v32, _ = T.lookup(lv, int(L.ix[q]) >> sh, int(L.iy[q]) >> sh, int(L.iz[q]) >> sh)
                assert got[pix] == v32[1], (seed, ml, pix)


# ------------------------------------------------------------ resolution

def test_resolution_uniform_tree_orthographic(O):
    """Every cell of a uniform level-l tree has side 2^-l, so every ray that
    meets the box has r = 2^-l / (2 |U| 2^-28) pixels; misses give 0."""
    rng = np.random.default_rng(2)
    for level in (1, 3):
        T = O.Tree(_uniform(level))
        for d in _ortho_cams(rng, 5, 9, 6):
            cam = T.camera(dict(d, max_level=level))
            r = T.resolution(cam)
            cnt = T.render(cam, O.SUM)["count"]
            w = 2.0 * math.sqrt(sum(float(u) ** 2 for u in cam.U)) * 2.0 ** -28
            assert np.all(r[cnt == 0] == 0.0)
            assert np.allclose(r[cnt > 0], 2.0 ** -level / w, rtol=1e-14)


def test_resolution_single_cell_perspective(O):
    """The root alone, eye inside it: one segment from t = 0 to the box exit
    t1 = min_k (face_k - o_k) / d_k, so r = 2^0 / (w0 t1 / 2) with
    w0 = 2 |U| 2^-28."""
    T = O.Tree(_uniform(0))
    d = amrgen.camera("persp", (0.3, 0.6, 0.45), (0.9, 0.1, 0.7), (0, 0, 1), 5, 4, fov_y=1.1, max_level=0)
    cam = T.camera(d)
    r = T.resolution(cam)
    w0 = 2.0 * math.sqrt(sum(float(u) ** 2 for u in cam.U)) * 2.0 ** -28
    for pix in range(cam.W * cam.H):
        o, dv = O.pixel_ray(cam, pix % cam.W, pix // cam.W)
        t1 = min(((1 << 28) - o[k]) / dv[k] if dv[k] > 0 else (-o[k] / dv[k]) for k in range(3) if dv[k] != 0)
        assert r[pix] == pytest.approx(2.0 / (w0 * t1), rel=1e-13)


def test_resolution_two_level_hand_case(O):
    """Ray along +x at y = z = 0.3: the half x < 0.5 is one level-1 cell, the
    half x >= 0.5 two level-2 cells: r = (0.5 x 0.5 + 0.25 x 0.25 + 0.25 x
    0.25) / 1 / w = 0.375 / w."""
    lv, xs, ys, zs = [], [], [], []
    for c in range(8):
        x, y, z = c & 1, (c >> 1) & 1, (c >> 2) & 1
        if x == 1:
            for cc in range(8):
                lv.append(2)
                xs.append(2 * x + (cc & 1))
                ys.append(2 * y + ((cc >> 1) & 1))
                zs.append(2 * z + ((cc >> 2) & 1))
        else:
            lv.append(1)
            xs.append(x)
            ys.append(y)
            zs.append(z)
    L = amrgen.Leaves(np.array(lv, np.int32), np.array(xs, np.int32), np.array(ys, np.int32), np.array(zs, np.int32),
                      np.ones((1, len(lv)), np.float32), 1)
    T = O.Tree(L)
    cam = T.camera(amrgen.camera("ortho", (-0.5, 0.3, 0.3), (0.5, 0.3, 0.3), (0, 0, 1), 1, 1, ortho_height=0.25,
                                 max_level=2))
    w = 2.0 * math.sqrt(sum(float(u) ** 2 for u in cam.U)) * 2.0 ** -28
    assert T.render(cam, O.SUM)["count"][0] == 3
    assert T.resolution(cam)[0] == pytest.approx(0.375 / w, rel=1e-14)


# ------------------------------------------------------------------- blur

def _gauss_norm(s, R):
    return sum(math.exp(-i * i / (2 * s * s)) for i in range(-R, R + 1))


def test_blur_constant_image_is_unchanged():
    rng = np.random.default_rng(3)
    img = np.full((23, 31), 2.5)
    res = rng.uniform(0.0, 40.0, img.shape)
    out = OP.adaptive_blur(img, res, 0.5)
    assert np.allclose(out, 2.5, rtol=1e-14)


def test_blur_preserves_linear_ramps_away_from_borders():
    H, W = 41, 45
    yy, xx = np.mgrid[0:H, 0:W]
    img = 0.3 * xx - 0.7 * yy + 5.0
    for k in (0, 2, 4):
        res = np.full((H, W), OP.sigma_level(k) / 0.5)  # kappa 0.5 -> sigma = sigma_k
        R = OP.radius(k)
        pix = [y * W + x for y in range(R, H - R) for x in range(R, W - R)][::7]
        out = OP.adaptive_blur(img, res, 0.5, np.array(pix))
        assert np.allclose(out, img.ravel()[pix], rtol=0, atol=1e-11), k


def test_blur_impulse_response_closed_form():
    """An impulse at (20, 20): B_k at (20 + dx, 20 + dy) is
    exp(-(dx^2 + dy^2) / (2 s^2)) / (sum_{|i| <= R} exp(-i^2 / (2 s^2)))^2
    inside the image; half way (in log2 sigma) between two levels the output
    is the mean of the two levels' responses; at sigma = SIGMA0 / 2 half the
    image plus half of level 0."""
    H = W = 41
    img = np.zeros((H, W))
    img[20, 20] = 1.0
    for k in (1, 3):
        s, R = OP.sigma_level(k), OP.radius(k)
        res = np.full((H, W), s / 0.5)
        for dx, dy in ((0, 0), (1, 0), (2, -3), (R, R)):
            got = OP.adaptive_blur(img, res, 0.5, np.array([(20 + dy) * W + 20 + dx]))[0]
            want = math.exp(-(dx * dx + dy * dy) / (2 * s * s)) / _gauss_norm(s, R) ** 2
            assert got == pytest.approx(want, rel=1e-12), (k, dx, dy)
    # between levels 2 and 3
    s2, s3 = OP.sigma_level(2), OP.sigma_level(3)
    res = np.full((H, W), s2 * 2 ** 0.25 / 0.5)
    for dx, dy in ((0, 0), (1, 2)):
        got = OP.adaptive_blur(img, res, 0.5, np.array([(20 + dy) * W + 20 + dx]))[0]
        want = 0.5 * sum(math.exp(-(dx * dx + dy * dy) / (2 * s * s)) / _gauss_norm(s, OP.radius(k)) ** 2
                         for k, s in ((2, s2), (3, s3)))
        assert got == pytest.approx(want, rel=1e-12)
    # below the first level: from the image itself
    res = np.full((H, W), OP.SIGMA0 / 2 / 0.5)
    got = OP.adaptive_blur(img, res, 0.5, np.array([20 * W + 20]))[0]
    assert got == pytest.approx(0.5 + 0.5 / _gauss_norm(OP.SIGMA0, OP.radius(0)) ** 2, rel=1e-12)
    # zero resolution (rays that miss the box): the image itself
    assert OP.adaptive_blur(img, np.zeros((H, W)), 0.5, np.array([20 * W + 20]))[0] == 1.0


def test_blur_normalises_over_the_image_at_borders():
    """At a corner the window is cut by the image: a constant image stays
    constant and an impulse at the corner gets weight 1 / (sum of the
    weights of the window's pixels inside the image)."""
    img = np.zeros((30, 30))
    img[0, 0] = 1.0
    k = 4
    s, R = OP.sigma_level(k), OP.radius(k)
    res = np.full(img.shape, s / 0.5)
    got = OP.adaptive_blur(img, res, 0.5, np.array([0]))[0]
    half = sum(math.exp(-i * i / (2 * s * s)) for i in range(0, R + 1))
    assert got == pytest.approx(1.0 / half ** 2, rel=1e-12)
    # beyond the top of the ladder: the top level
    res = np.full(img.shape, 1e4)
    top = OP.NLEVELS - 1
    s, R = OP.sigma_level(top), OP.radius(top)
    half = sum(math.exp(-i * i / (2 * s * s)) for i in range(0, min(R, 29) + 1))
    assert OP.adaptive_blur(img, res, 0.5, np.array([0]))[0] == pytest.approx(1.0 / half ** 2, rel=1e-12)
