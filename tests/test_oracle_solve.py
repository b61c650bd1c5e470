"""Pins of the oracle's solver against closed forms, hand-worked cases, brute force
and invariants of the discrete system of Section 2.2.  CPU only."""
import numpy as np
import pytest

import oracle
from golden_io import small_systems


def _random_case(rng, H, W, dens=0.2):
    f = rng.uniform(0, 255, size=(H, W))
    m = (rng.random((H, W)) < dens).astype(np.uint8)
    if not m.any():
        m[rng.integers(H), rng.integers(W)] = 1
    return f, m


# ---------------------------------------------------------------- worked cases

@pytest.mark.parametrize("case", small_systems(), ids=lambda c: c[0])
def test_hand_worked_systems(case):
    _, mask, f, u = case
    got = oracle.solve_pcg(f, mask)[0]
    np.testing.assert_allclose(got, u, rtol=0, atol=1e-10)
    got_d = oracle.solve_dense(f, mask)[0]
    np.testing.assert_allclose(got_d, u, rtol=0, atol=1e-10)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("W,seed", [(7, 0), (40, 1), (257, 2), (1000, 3)])
def test_single_row_is_piecewise_linear(W, seed):
    """A 1-pixel-high image: the solution interpolates linearly between known
    pixels and is constant beyond the first and last one (reflecting ends)."""
    rng = np.random.default_rng(seed)
    f, m = _random_case(rng, 1, W, dens=0.1)
    xs = np.nonzero(m[0])[0]
    expect = np.interp(np.arange(W), xs, f[0, xs])
    got = oracle.solve_pcg(f, m)[0, 0]
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-8)


@pytest.mark.parametrize("H,seed", [(9, 4), (300, 5)])
def test_single_column_is_piecewise_linear(H, seed):
    rng = np.random.default_rng(seed)
    f, m = _random_case(rng, H, 1, dens=0.1)
    ys = np.nonzero(m[:, 0])[0]
    expect = np.interp(np.arange(H), ys, f[ys, 0])
    got = oracle.solve_pcg(f, m)[0, :, 0]
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-8)


@pytest.mark.parametrize("transpose", [False, True])
def test_whole_known_columns(transpose):
    """Known data on whole columns, constant along each: the solution does not
    vary along y and interpolates linearly in x between the columns."""
    rng = np.random.default_rng(6)
    H, W = 23, 61
    cols = np.sort(rng.choice(W, size=5, replace=False))
    vals = rng.uniform(0, 255, size=5)
    m = np.zeros((H, W), np.uint8)
    f = np.full((H, W), np.nan)
    m[:, cols] = 1
    f[:, cols] = vals[None, :]
    expect = np.broadcast_to(np.interp(np.arange(W), cols, vals)[None, :], (H, W))
    if transpose:
        m, f, expect = m.T.copy(), f.T.copy(), expect.T
    got = oracle.solve_pcg(f, m)[0]
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-8)


def test_single_known_pixel_gives_constant():
    m = np.zeros((19, 33), np.uint8)
    m[7, 21] = 1
    f = np.full(m.shape, np.nan)
    f[7, 21] = 123.25
    np.testing.assert_allclose(oracle.solve_pcg(f, m)[0], 123.25, rtol=0, atol=1e-9)


def test_constant_data_gives_constant():
    rng = np.random.default_rng(7)
    _, m = _random_case(rng, 31, 45, dens=0.03)
    f = np.full(m.shape, 42.0)
    np.testing.assert_allclose(oracle.solve_pcg(f, m)[0], 42.0, rtol=0, atol=1e-9)


def test_linear_ramp_with_known_border_is_exact():
    """A linear ramp is discrete-harmonic; with every border pixel known the
    reflecting boundary plays no part and the ramp is reproduced exactly."""
    rng = np.random.default_rng(8)
    H, W = 48, 48
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = 17.0 + 1.5 * x - 0.75 * y
    m = (rng.random((H, W)) < 0.05).astype(np.uint8)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = 1
    np.testing.assert_allclose(oracle.solve_pcg(f, m)[0], f, rtol=0, atol=1e-9)


def test_ramp_with_random_mask_only_is_not_exact():
    """Without the known border the reflecting boundary bends the ramp: this is
    the condition under which the ramp pin holds, checked from the other side."""
    rng = np.random.default_rng(8)
    H, W = 48, 48
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = 17.0 + 1.5 * x - 0.75 * y
    m = (rng.random((H, W)) < 0.05).astype(np.uint8)
    assert np.abs(oracle.solve_pcg(f, m)[0] - f).max() > 1.0


# ---------------------------------------------------------------- brute force

def _random_walk_solution(f, m):
    """Brute force from a different formulation: u(i) is the expected known value
    where a random walk from i first meets a known pixel.  Each step goes to one
    of the 4 directions with probability 1/4; a step that would leave the image
    stays put (reflection).  Solved as an absorbing Markov chain."""
    H, W = m.shape
    idx = [(y, x) for y in range(H) for x in range(W)]
    unk = [k for k, (y, x) in enumerate(idx) if not m[y, x]]
    pos = {k: j for j, k in enumerate(unk)}
    n = len(unk)
    Q = np.zeros((n, n))
    R = np.zeros(n)
    for j, k in enumerate(unk):
        y, x = idx[k]
        for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            yy, xx = y + dy, x + dx
            if not (0 <= yy < H and 0 <= xx < W):
                yy, xx = y, x
            kk = yy * W + xx
            if m[yy, xx]:
                R[j] += 0.25 * f[yy, xx]
            else:
                Q[j, pos[kk]] += 0.25
    u = np.array(f, dtype=np.float64, copy=True)
    sol = np.linalg.solve(np.eye(n) - Q, R) if n else np.zeros(0)
    for j, k in enumerate(unk):
        u[idx[k]] = sol[j]
    return u


@pytest.mark.parametrize("H,W,dens,seed", [
    (1, 1, 1.0, 0), (1, 9, 0.3, 1), (9, 1, 0.3, 2), (5, 9, 0.2, 3), (16, 16, 0.05, 4),
    (17, 23, 0.1, 5), (32, 32, 0.05, 6), (32, 32, 1.0, 7), (2, 31, 0.1, 8),
])
def test_pcg_and_dense_match_random_walk(H, W, dens, seed):
    rng = np.random.default_rng(seed)
    f, m = _random_case(rng, H, W, dens)
    ref = _random_walk_solution(f, m)
    np.testing.assert_allclose(oracle.solve_pcg(f, m)[0], ref, rtol=0, atol=1e-8)
    if H * W <= 1024:
        np.testing.assert_allclose(oracle.solve_dense(f, m)[0], ref, rtol=0, atol=1e-8)


# ---------------------------------------------------------------- invariants

def test_invariants_on_random_image():
    rng = np.random.default_rng(9)
    H, W = 40, 57
    f, m = _random_case(rng, H, W, dens=0.04)
    u = oracle.solve_pcg(f, m)[0]
    k = m != 0
    # known pixels reproduced bit-exactly
    assert np.array_equal(u[k], f[k])
    # maximum principle
    assert u.min() >= f[k].min() - 1e-9 and u.max() <= f[k].max() + 1e-9
    # values at unknown pixels are never read
    g = f.copy()
    g[~k] = np.nan
    assert np.array_equal(oracle.solve_pcg(g, m)[0], u)
    # linearity in f for a fixed mask
    f2 = rng.uniform(0, 255, size=(H, W))
    u2 = oracle.solve_pcg(f2, m)[0]
    u3 = oracle.solve_pcg(0.3 * f - 2.0 * f2, m)[0]
    np.testing.assert_allclose(u3, 0.3 * u - 2.0 * u2, atol=1e-7)
    # equivariance under flips and transposition
    np.testing.assert_allclose(oracle.solve_pcg(f[:, ::-1], m[:, ::-1])[0], u[:, ::-1], atol=1e-8)
    np.testing.assert_allclose(oracle.solve_pcg(f[::-1], m[::-1])[0], u[::-1], atol=1e-8)
    np.testing.assert_allclose(oracle.solve_pcg(f.T, m.T)[0], u.T, atol=1e-8)


def test_channels_are_independent():
    rng = np.random.default_rng(10)
    f = rng.uniform(0, 255, size=(3, 20, 30))
    m = (rng.random((20, 30)) < 0.1).astype(np.uint8)
    u = oracle.solve_pcg(f, m)
    for ch in range(3):
        np.testing.assert_array_equal(u[ch], oracle.solve_pcg(f[ch], m)[0])


def test_empty_mask_is_rejected():
    with pytest.raises(ValueError):
        oracle.solve_pcg(np.zeros((4, 4)), np.zeros((4, 4), np.uint8))
    with pytest.raises(ValueError):
        oracle.solve_dense(np.zeros((4, 4)), np.zeros((4, 4), np.uint8))


def test_all_known_returns_f():
    rng = np.random.default_rng(11)
    f = rng.uniform(0, 255, size=(6, 7))
    m = np.ones((6, 7), np.uint8)
    assert np.array_equal(oracle.solve_pcg(f, m)[0], f)


# ---------------------------------------------------------------- rel_res

def test_rel_res_reference_points():
    rng = np.random.default_rng(12)
    f, m = _random_case(rng, 33, 35, dens=0.05)
    cf = np.where(m != 0, f, 0.0)
    assert oracle.rel_res(cf, f, m)[0] == pytest.approx(1.0, rel=1e-14)
    u = oracle.solve_pcg(f, m)[0]
    assert oracle.rel_res(u, f, m)[0] < 1e-11
    # scale invariance: rel_res(a u; a f) == rel_res(u; f)
    assert oracle.rel_res(3.0 * cf, 3.0 * f, m)[0] == pytest.approx(1.0, rel=1e-14)
    # a perturbation of one unknown pixel by d raises the residual by d*|N(i)| there
    # and by d at each unknown neighbour
    y, x = np.argwhere(m == 0)[0]
    v = u.copy()
    v[y, x] += 1.0
    r = oracle.residual(v, f, m)
    assert r[y, x] == pytest.approx(-oracle.neighbour_count(*m.shape)[y, x], abs=1e-9)
