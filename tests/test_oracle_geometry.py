"""Pins of the oracle's level and block geometry (Sections 3.1, 4.3 and 4.4). CPU only."""
import numpy as np
import pytest

import oracle


def test_4k_has_eight_levels_down_to_one_block():
    """Section 4.4: halving until a single 32x32 block remains gives 8 levels at 4K."""
    sizes = oracle.level_sizes(3840, 2160, 32)
    assert len(sizes) == 8
    assert sizes[-1] == (30, 17)
    assert sizes[1] == (1920, 1080) and sizes[4] == (240, 135) and sizes[5] == (120, 68)


def test_256_has_four_levels():
    """The mask-restriction figure of Section 4.3 shows a 256x256 mask at 256, 128, 64
    and 32 pixels."""
    assert oracle.level_sizes(256, 256, 32) == [(256, 256), (128, 128), (64, 64), (32, 32)]


def test_36852_local_problems_for_4k_rgb():
    """Section 3.1: 32x32 blocks with a 6-pixel overlap give 36852 local problems
    per ORAS iteration for a 4K colour image."""
    n = oracle.num_blocks(3840, 32, 6) * oracle.num_blocks(2160, 32, 6) * 3
    assert n == 36852
    # the alternative of ceil(n / stride) blocks would give a different count
    assert -(-3840 // 26) * -(-2160 // 26) * 3 != 36852


@pytest.mark.parametrize("n", [1, 2, 17, 31, 32, 33, 38, 39, 58, 59, 100, 255, 256, 1080, 2160, 3840])
@pytest.mark.parametrize("B,o", [(32, 6), (32, 2), (16, 4), (24, 8), (64, 6), (32, 16), (16, 2)])
def test_blocks_cover_axis_with_uniform_overlap(n, B, o):
    blocks = oracle.block_starts(n, B, o)
    assert blocks[0][0] == 0
    assert blocks[-1][0] + blocks[-1][1] == n
    for (s0, w0), (s1, w1) in zip(blocks, blocks[1:]):
        assert s1 - s0 == B - o and w0 == B
        assert s0 + w0 - s1 == o           # neighbours share exactly o pixels
        assert w1 > o                      # the clipped last block is wider than the overlap
    for (s0, w0), (s2, _) in zip(blocks, blocks[2:]):
        assert s2 >= s0 + w0               # no pixel lies in three blocks along an axis


@pytest.mark.parametrize("n", [1, 20, 32, 33, 59, 100, 257, 3840])
@pytest.mark.parametrize("B,o", [(32, 6), (32, 2), (16, 4), (24, 8), (32, 16)])
def test_partition_of_unity_1d(n, B, o):
    """Partition of unity of discrete ORAS (Section 3): sum_i R_i^T D_i R_i = I, with
    weight 0 at the outermost and 1 at
    the innermost overlap pixel and linear in between (Section 3.1)."""
    blocks = oracle.block_starts(n, B, o)
    wts = oracle.pou_weights_1d(n, B, o)
    acc = np.zeros(n)
    for (s0, w), wt in zip(blocks, wts):
        assert wt.shape == (w,)
        assert np.all(wt >= 0) and np.all(wt <= 1)
        acc[s0:s0 + w] += wt
    np.testing.assert_allclose(acc, 1.0, rtol=0, atol=1e-15)
    if len(blocks) > 1:
        first, second = wts[0], wts[1]
        assert first[B - 1] == 0.0 and first[B - o] == 1.0
        assert second[0] == 0.0 and second[o - 1] == 1.0
        np.testing.assert_allclose(np.diff(second[:o]), 1.0 / (o - 1), atol=1e-15)
        # toward the image edge the weight stays 1
        assert first[0] == 1.0 and wts[-1][-1] == 1.0


@pytest.mark.parametrize("W,H,B,o", [(100, 70, 32, 6), (33, 97, 16, 4), (3840 // 16, 2160 // 16, 32, 6)])
def test_partition_of_unity_2d(W, H, B, o):
    acc = np.zeros((H, W))
    for by, (y0, h) in enumerate(oracle.block_starts(H, B, o)):
        for bx, (x0, w) in enumerate(oracle.block_starts(W, B, o)):
            acc[y0:y0 + h, x0:x0 + w] += oracle.block_weight_2d(W, H, B, o, bx, by)
    np.testing.assert_allclose(acc, 1.0, rtol=0, atol=1e-15)
