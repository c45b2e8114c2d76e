"""Pins for the learned-LOD oracle (CPU): finite differences, closed forms,
hand-made label cases, and probe statistics against the pinned renderer."""
import math

import numpy as np
import pytest

import amrgen
from tests import bruteforce as bf


@pytest.fixture(scope="module")
def L():
    import oracle
    import oracle.lod as lod

    oracle.build()
    return lod


def test_bf16_rounding_cases(L):
    one = 1.0
    # bf16 keeps 8 significand bits: ulp(1) = 2^-7; ties go to even
    cases = {one: one, one + 2 ** -9: one, one + 3 * 2 ** -9: one + 2 ** -7, one + 2 ** -8: one,
             one + 2 ** -8 + 2 ** -20: one + 2 ** -7, one + 3 * 2 ** -8: one + 2 ** -6, -2.5: -2.5}
    for x, want in cases.items():
        assert L.bf16(np.float32(x)) == want, x


def test_loss_closed_forms(L):
    z = np.zeros((3, 16))
    y = np.array([0, 4, 15])
    loss, g = L.loss_and_grad(z, y, 0.5)
    u = 1.0 / 16
    assert np.allclose(loss, math.log(16) + 0.5 * y * u)
    for k, yy in enumerate(y):
        want = np.array([u - (j == yy) + 0.5 * u * ((j < yy) - u * yy) for j in range(16)])
        assert np.allclose(g[k], want)
    p = L.softmax10(np.random.default_rng(0).normal(size=(5, 16)))
    assert np.allclose(p.sum(axis=1), 1.0)


def test_loss_gradient_matches_finite_differences(L):
    rng = np.random.default_rng(1)
    z = rng.normal(size=(6, 16)) * 2
    y = rng.integers(0, 16, 6)
    for lam in (0.0, 2.0):
        _, g = L.loss_and_grad(z, y, lam)
        num = np.zeros_like(z)
        h = 1e-6
        for i in range(6):
            for c in range(16):
                zp, zm = z.copy(), z.copy()
                zp[i, c] += h
                zm[i, c] -= h
                num[i, c] = (L.loss_and_grad(zp, y, lam)[0][i] - L.loss_and_grad(zm, y, lam)[0][i]) / (2 * h)
        assert np.allclose(g, num, atol=1e-8)


def test_parameter_gradients_match_finite_differences(L):
    rng = np.random.default_rng(2)
    params = rng.normal(size=L.NPARAMS) * 0.3
    X = rng.normal(size=(7, 32))
    y = rng.integers(0, 16, 7)
    lam = 1.5
    logits, acts = L.forward(params, X, emulate=False)
    _, dl = L.loss_and_grad(logits, y, lam)
    g = L.backward(params, X, acts, dl, emulate=False)
    idx = rng.choice(L.NPARAMS, 200, replace=False)
    h = 1e-6
    for k in idx:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        num = (L.total_loss(pp, X, y, lam) - L.total_loss(pm, X, y, lam)) / (2 * h)
        assert g[k] == pytest.approx(num, rel=1e-5, abs=1e-7), k


def test_labels_hand_made(L):
    W = H = 32  # 4 tiles; 16 renders (levels 1..16), the last is the reference
    ref = np.ones((H, W))
    imgs = [ref.copy() * 2 for _ in range(15)] + [ref]
    # tile 0: exact from class 3; tile 1: within tol from class 5; tile 2: never; tile 3: exact everywhere
    for c in range(3, 15):
        imgs[c][0:16, 0:16] = 1.0
    for c in range(5, 15):
        imgs[c][0:16, 16:32] = 1.0 + 0.9e-3
    for c in range(15):
        imgs[c][16:32, 16:32] = 1.0
    imgs[4][0:16, 16:32] = 1.0 + 1.1e-3  # class 4 just outside the tolerance
    lab = L.labels_from_renders([x.ravel() for x in imgs], W, H, 1e-3)
    assert lab.tolist() == [3, 5, 15, 0]


def test_plan_quantile_and_fallback(L):
    z = np.full((3, 16), -20.0)
    z[0, 2] = 10.0                     # confident class 2 -> level 3
    z[1, :] = 0.0                      # uniform -> low confidence -> full
    z[2, 4] = 3.0
    z[2, 6] = 3.0                      # two equal peaks: cdf reaches 0.99 at class 6 -> level 7
    lev, fb = L.plan(z, 0.99, 0.4, 16)
    assert lev.tolist() == [3, 16, 7] and fb.tolist() == [False, True, False]
    lev2, fb2 = L.plan(z, 0.99, 0.6, 16)
    assert lev2.tolist() == [3, 16, 16] and fb2.tolist() == [False, True, True]
    lev3, fb3 = L.plan(z, 0.99, 1.0, 16)
    assert np.all(lev3 == 16) and np.all(fb3)


def test_probe_stats_against_pinned_render(L):
    import oracle

    leaves = amrgen.random_tree(41, lmax=5, p_refine=0.45)
    T = oracle.Tree(leaves)
    cam = T.camera(amrgen.camera("persp", (0.5, -1.0, 0.7), (0.5, 0.5, 0.5), (0, 0, 1), 24, 20, fov_y=0.8,
                                 max_level=3))
    ids, nt = L.probe_pixels(24, 20)
    st = T.probe_stats(cam, ids)
    ref = T.render(cam, oracle.SUM, rays=ids)
    assert np.allclose(st[:, 0], ref["val"], rtol=1e-12)
    assert np.array_equal(st[:, 15].astype(np.int64), ref["count"])
    assert np.allclose(st[:, 5:15].sum(axis=1), st[:, 1], rtol=1e-12)
    for r, pid in enumerate(ids):
        o, d = oracle.pixel_ray(cam, pid % 24, pid // 24)
        assert st[r, 1] == pytest.approx(bf.box_chord(o.tolist(), d.tolist()), rel=1e-12, abs=1e-300)
        assert st[r, 4] == (1.0 if st[r, 1] > 0 else 0.0)
    f = L.tile_features(st, None, 0.5, nt)
    hit = f[:, 15] > 0
    assert np.allclose(f[hit, 2:12].sum(axis=1), 1.0)


def test_adam_constant_gradient_closed_form(L):
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2 at every step, so each step moves a parameter by
    -lr g / (|g| + eps): after t steps p = p0 - t lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50) * np.logspace(-6, 2, 50)
    lr, eps = 3e-3, 1e-8
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 41):
        p, m, v = L.adam(p, g, m, v, t, lr, eps=eps)
        want = p0 - t * lr * g / (np.abs(g) + eps)
        assert np.allclose(p, want, rtol=1e-12, atol=1e-14), t
    # the moments themselves: m_t = g (1 - 0.9^t), v_t = g^2 (1 - 0.999^t)
    assert np.allclose(m, g * (1 - 0.9 ** 40), rtol=1e-12)
    assert np.allclose(v, g * g * (1 - 0.999 ** 40), rtol=1e-12)


def test_adam_alternating_gradient_closed_form(L):
    """g_k = (-1)^k g: m_t = (1 - b1) (-1)^t g (1 - (-b1)^t) / (1 + b1),
    v_t = g^2 (1 - b2^t), and the step uses both bias corrections."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-2, 1e-8
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    want_p = np.zeros(3)
    for t in range(1, 25):
        p, m, v = L.adam(p, (-1.0) ** t * g, m, v, t, lr)
        mt = (1 - b1) * (-1.0) ** t * g * (1 - (-b1) ** t) / (1 + b1)
        vt = g * g * (1 - b2 ** t)
        assert np.allclose(m, mt, rtol=1e-12) and np.allclose(v, vt, rtol=1e-12)
        want_p = want_p - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(p, want_p, rtol=1e-12, atol=1e-15)
    # the first step is -lr sign(g) (up to eps)
    p1, _, _ = L.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr)
    assert np.allclose(p1, -lr * g / (np.abs(g) + eps), rtol=1e-12)
