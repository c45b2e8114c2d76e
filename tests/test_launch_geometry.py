"""CPU check of the render kernels' grid -> pixel mapping for every variant:
each pixel is written by exactly one lane and no lane writes outside the
image.  Mirrors the index arithmetic of k_render (block remap over the 8
XCDs, packets of PW x 64/PW pixels, WPB waves per block) and of
k_render_split (one 8 x 8 packet per block, K span waves, wave 0 writes)."""
import numpy as np
import pytest

import paper_1210_8014_amd as amr

# (packet width, waves per block, XCD remap, spans per ray) per variant, in library order
VARIANTS = [(8, 1, False, 1), (8, 2, False, 1), (8, 4, False, 1), (16, 4, False, 1), (32, 2, False, 1),
            (8, 1, False, 1), (8, 4, False, 1), (8, 1, False, 1), (8, 4, True, 1), (8, 2, False, 2), (8, 4, False, 4)]


def xcd_remap(b, nb):
    full = nb - nb % 8
    if b >= full:
        return b
    return (b % 8) * (full // 8) + b // 8


def covered_split(W, H, k):
    px, py = -(-W // 8), -(-H // 8)
    hits = np.zeros(W * H, np.int64)
    for b in range(px * py):
        ty, tx = divmod(b, px)
        for t in range(64 * k):
            lane, w = t % 64, t // 64
            i, j = tx * 8 + lane % 8, ty * 8 + lane // 8
            if w != 0 or ty >= py or i >= W or j >= H:
                continue
            hits[j * W + i] += 1
    return hits


def covered(W, H, pw, wpb, remap, split=1):
    if split > 1:
        return covered_split(W, H, split)
    ph = 64 // pw
    px, py = -(-W // pw), -(-H // ph)
    blocks = -(-(px * py) // wpb)
    hits = np.zeros(W * H, np.int64)
    for b in range(blocks):
        blk = xcd_remap(b, blocks) if remap else b
        for w in range(wpb):
            packet = blk * wpb + w
            ty, tx = divmod(packet, px)
            for lane in range(64):
                i, j = tx * pw + lane % pw, ty * ph + lane // pw
                if ty >= py or i >= W or j >= H:
                    continue
                hits[j * W + i] += 1
    return hits


def test_variant_table_matches_library():
    names = amr.variants()
    for (pw, wpb, remap, split), n in zip(VARIANTS, names):
        head = f"p{pw}x{64 // pw}_split{split}_" if split > 1 else f"p{pw}x{64 // pw}_w{wpb}_"
        assert n.startswith(head)
        assert n.endswith("xcdband") == remap


@pytest.mark.parametrize("W,H", [(1, 1), (37, 23), (64, 64), (256, 256), (130, 9), (9, 130), (517, 211)])
def test_every_pixel_written_once(W, H):
    for v in VARIANTS:
        assert np.all(covered(W, H, *v) == 1), (W, H, v)


def test_xcd_remap_is_a_permutation():
    for nb in [1, 7, 8, 9, 64, 1000, 16384, 16389]:
        r = [xcd_remap(b, nb) for b in range(nb)]
        assert sorted(r) == list(range(nb))
