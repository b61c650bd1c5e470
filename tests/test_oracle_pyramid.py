"""Pins of the oracle's coarse problems and grid transfers (Sections 4.1, 4.3, 4.4). CPU only."""
import numpy as np
import pytest

import oracle
from golden_io import pyramid_cases


@pytest.mark.parametrize("k", range(len(pyramid_cases())))
def test_worked_pyramid_cases(k):
    case = pyramid_cases()[k]
    cf = case["fine_mask"].astype(np.uint8)
    b = case["fine_b"]
    np.testing.assert_array_equal(oracle.mask_down(cf), case["coarse_mask"])
    np.testing.assert_allclose(oracle.rhs_down_naive(cf, b), case["naive"], atol=1e-12)
    np.testing.assert_allclose(oracle.rhs_down_modified(cf, b), case["modified"], atol=1e-12)


def _printed_top_left_weight(cf):
    """Printed weight of the top-left child (2,2) of coarse cell (1,1) of a 6x6
    fine mask (Section 4.3): ``c (4 - c_H(left) - c_H(up) - c_h(right) - c_h(down))``.
    This is the one printed weight without an index typo."""
    cc = oracle.mask_down(cf)
    return int(cf[2, 2]) * (4 - int(cc[1, 0]) - int(cc[0, 1]) - int(cf[2, 3]) - int(cf[3, 2]))


def test_modified_weights_from_printed_top_left_formula():
    """The other three children's weights are mirror images of the top-left one,
    so each is the printed top-left formula applied to the flipped mask.  The
    oracle must agree with that on random masks (this pins all four weights
    without using the three printed formulas that carry typos)."""
    rng = np.random.default_rng(0)
    for _ in range(400):
        cf = (rng.random((6, 6)) < 0.5).astype(np.uint8)
        bb = rng.uniform(0, 255, size=(6, 6))
        w = {
            (2, 2): _printed_top_left_weight(cf),
            (2, 3): _printed_top_left_weight(cf[:, ::-1]),
            (3, 2): _printed_top_left_weight(cf[::-1]),
            (3, 3): _printed_top_left_weight(cf[::-1, ::-1]),
        }
        den = sum(w.values())
        known = [(y, x) for (y, x) in w if cf[y, x]]
        got = oracle.rhs_down_modified(cf, bb)[1, 1]
        if den > 0:
            assert got == pytest.approx(sum(w[k] * bb[k] for k in w) / den, rel=1e-12)
        elif known:
            assert got == pytest.approx(np.mean([bb[k] for k in known]), rel=1e-12)
        else:
            assert got == 0.0


def test_modified_downsampling_is_flip_equivariant():
    rng = np.random.default_rng(5)
    for _ in range(50):
        cf = (rng.random((10, 14)) < 0.4).astype(np.uint8)
        bb = rng.uniform(0, 255, size=(10, 14))
        out = oracle.rhs_down_modified(cf, bb)
        np.testing.assert_allclose(oracle.rhs_down_modified(cf[:, ::-1], bb[:, ::-1]), out[:, ::-1], atol=1e-12)
        np.testing.assert_allclose(oracle.rhs_down_modified(cf[::-1], bb[::-1]), out[::-1], atol=1e-12)
        np.testing.assert_allclose(oracle.rhs_down_modified(cf.T, bb.T), out.T, atol=1e-12)


def test_mask_down_odd_sizes_and_density():
    rng = np.random.default_rng(1)
    c = (rng.random((37, 23)) < 0.03).astype(np.uint8)
    cc = oracle.mask_down(c)
    assert cc.shape == (19, 12)
    # brute force over the children, including partial cells at the edges
    for Y in range(19):
        for X in range(12):
            assert cc[Y, X] == int(c[2 * Y:2 * Y + 2, 2 * X:2 * X + 2].any())
    assert cc.mean() >= c.mean()


def test_rhs_down_constant_values():
    """Any positive weighting of equal values returns that value."""
    rng = np.random.default_rng(2)
    c = (rng.random((41, 30)) < 0.2).astype(np.uint8)
    b = np.where(c != 0, 9.5, 0.0)
    cc = oracle.mask_down(c) != 0
    for fn in (oracle.rhs_down_naive, oracle.rhs_down_modified):
        out = fn(c, b)
        np.testing.assert_allclose(out[cc], 9.5, atol=1e-12)
        assert np.all(out[~cc] == 0)


def test_prolong_closed_forms():
    # constants are reproduced everywhere
    np.testing.assert_allclose(oracle.prolong_bilinear(np.full((5, 7), 3.0), 13, 9), 3.0, atol=1e-15)
    # a linear function sampled at coarse cell centres is reproduced at fine
    # cell centres away from the clamped edge rows/columns
    Hc, Wc = 9, 11
    Y, X = np.mgrid[0:Hc, 0:Wc].astype(np.float64)
    uc = 2.0 + 0.5 * (2 * X + 0.5) - 1.25 * (2 * Y + 0.5)
    uf = oracle.prolong_bilinear(uc, 2 * Wc, 2 * Hc)
    y, x = np.mgrid[0:2 * Hc, 0:2 * Wc].astype(np.float64)
    ef = 2.0 + 0.5 * x - 1.25 * y
    np.testing.assert_allclose(uf[1:-1, 1:-1], ef[1:-1, 1:-1], atol=1e-12)
    # a single interior coarse value spreads as the tensor product of (1/4, 3/4, 3/4, 1/4)
    d = np.zeros((7, 7))
    d[3, 3] = 1.0
    uf = oracle.prolong_bilinear(d, 14, 14)
    k = np.array([0.25, 0.75, 0.75, 0.25])
    np.testing.assert_allclose(uf[5:9, 5:9], np.outer(k, k), atol=1e-15)
    assert np.count_nonzero(uf) == 16


def test_restrict_residual_closed_forms():
    r = np.full((9, 12), 2.0)
    cc = np.zeros((5, 6), np.uint8)
    cc[1, 2] = 1
    out = oracle.restrict_residual(r, cc)
    assert out[1, 2] == 0.0
    expect = np.full((5, 6), 8.0)
    expect[1, 2] = 0.0
    np.testing.assert_allclose(out, expect, atol=1e-15)
    # partial edge cells use the mean of the children that exist
    r2 = np.arange(9 * 12, dtype=np.float64).reshape(9, 12)
    out2 = oracle.restrict_residual(r2, np.zeros((5, 6), np.uint8))
    assert out2[4, 0] == pytest.approx(4.0 * (r2[8, 0] + r2[8, 1]) / 2)


@pytest.mark.parametrize("coef", [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.3, -0.7, 0.5), (2.0, 1.5, -1.0)])
def test_restricted_residual_is_the_coarse_residual_of_a_quadratic(coef):
    """Two-grid consistency, independent of the restriction's own definition:
    for a quadratic error e(x, y) (pixel-centre coordinates, cell-centred
    grids, so a coarse centre sits at fine coordinate 2X + 1/2), the fine
    integer-stencil residual of e, restricted, equals the coarse
    integer-stencil residual of e sampled at the coarse centres.  The
    quadratic part makes the fine residual a constant -2(a + b); on the
    coarse grid the same function is 4 times as curved per cell, so any
    other factor than 4 (reading A2: H^2/h^2) fails."""
    a, b, c = coef
    Hf, Wf = 24, 32

    def e(x, y):
        return a * x * x + b * y * y + c * x * y + 0.25 * x - 3.0 * y + 1.0

    yf, xf = np.mgrid[0:Hf, 0:Wf].astype(np.float64)
    Yc, Xc = np.mgrid[0:Hf // 2, 0:Wf // 2].astype(np.float64)
    rf = oracle.apply_L(e(xf, yf))
    rc = oracle.apply_L(e(2 * Xc + 0.5, 2 * Yc + 0.5))
    out = oracle.restrict_residual(rf, np.zeros((Hf // 2, Wf // 2), np.uint8))
    # interior coarse cells: their children and the children's neighbours are
    # inside the image, where the reflecting boundary does not enter
    np.testing.assert_allclose(out[1:-1, 1:-1], rc[1:-1, 1:-1], rtol=0, atol=1e-9)
    np.testing.assert_allclose(rc[1:-1, 1:-1], -8.0 * (a + b), rtol=0, atol=1e-9)
