"""CPU check of the render kernels' grid -> pixel mapping for every variant:
each pixel is written by exactly one lane and no lane writes outside the
image.  Mirrors the index arithmetic of k_render (block remap over the 8
XCDs or centre-out packet rows, packets of PW x 64/PW pixels, WPB waves per
block) and of k_render_split (one 8 x 8 packet per block, K span waves,
wave 0 writes)."""
import numpy as np
import pytest

import paper_1210_8014_amd as amr

# (packet width, waves per block, remap, spans per ray) per variant, in library order;
# remap: None, "xcd" (bands over the 8 XCDs) or "center" (packet rows from the middle out)
VARIANTS = [(8, 1, None, 1), (8, 2, None, 1), (8, 4, None, 1), (16, 4, None, 1), (32, 2, None, 1),
            (8, 1, None, 1), (8, 4, None, 1), (8, 1, None, 1), (8, 4, "xcd", 1), (8, 2, None, 2), (8, 4, None, 4),
            (8, 1, "center", 1), (8, 2, "center", 2), (8, 4, None, 1), (8, 2, None, 1)]


def xcd_remap(b, nb):
    full = nb - nb % 8
    if b >= full:
        return b
    return (b % 8) * (full // 8) + b // 8


def center_out(b, px, py):
    k, x = divmod(b, px)
    row = py // 2 + (-((k + 1) >> 1) if k & 1 else (k >> 1))
    return row * px + x


def covered_split(W, H, k, remap=None):
    px, py = -(-W // 8), -(-H // 8)
    hits = np.zeros(W * H, np.int64)
    for b in range(px * py):
        ty, tx = divmod(center_out(b, px, py) if remap == "center" else b, px)
        for t in range(64 * k):
            lane, w = t % 64, t // 64
            i, j = tx * 8 + lane % 8, ty * 8 + lane // 8
            if w != 0 or ty >= py or i >= W or j >= H:
                continue
            hits[j * W + i] += 1
    return hits


def covered(W, H, pw, wpb, remap, split=1):
    if split > 1:
        return covered_split(W, H, split, remap)
    ph = 64 // pw
    px, py = -(-W // pw), -(-H // ph)
    blocks = -(-(px * py) // wpb)
    hits = np.zeros(W * H, np.int64)
    for b in range(blocks):
        blk = xcd_remap(b, blocks) if remap == "xcd" else b
        for w in range(wpb):
            packet = blk * wpb + w
            if remap == "center" and packet < px * py:
                packet = center_out(packet, px, py)
            ty, tx = divmod(packet, px)
            for lane in range(64):
                i, j = tx * pw + lane % pw, ty * ph + lane // pw
                if ty >= py or i >= W or j >= H:
                    continue
                hits[j * W + i] += 1
    return hits


def test_variant_table_matches_library():
    names = amr.variants()
    assert len(names) == len(VARIANTS)
    for (pw, wpb, remap, split), n in zip(VARIANTS, names):
        head = f"p{pw}x{64 // pw}_split{split}_" if split > 1 else f"p{pw}x{64 // pw}_w{wpb}_"
        assert n.startswith(head)
        assert n.endswith("xcdband") == (remap == "xcd")
        assert n.endswith("center") == (remap == "center")


@pytest.mark.parametrize("W,H", [(1, 1), (37, 23), (64, 64), (256, 256), (130, 9), (9, 130), (517, 211)])
def test_every_pixel_written_once(W, H):
    for v in VARIANTS:
        assert np.all(covered(W, H, *v) == 1), (W, H, v)


def test_xcd_remap_is_a_permutation():
    for nb in [1, 7, 8, 9, 64, 1000, 16384, 16389]:
        r = [xcd_remap(b, nb) for b in range(nb)]
        assert sorted(r) == list(range(nb))


def test_center_out_is_a_permutation_middle_first():
    for px, py in [(1, 1), (3, 1), (1, 2), (5, 7), (4, 8), (256, 256), (17, 33)]:
        r = [center_out(b, px, py) for b in range(px * py)]
        assert sorted(r) == list(range(px * py))
        assert r[0] // px == py // 2
        # rows leave the middle in order of distance
        d = [abs(q // px - py // 2) for q in r]
        assert d == sorted(d)
