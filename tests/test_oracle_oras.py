"""Pins of the oracle's ORAS iteration (Algorithm 2, Section 3). CPU only."""
import numpy as np
import pytest

import oracle


def _case(seed, H, W, dens):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 255, size=(H, W))
    m = (rng.random((H, W)) < dens).astype(np.uint8)
    m[0, 0] = 1
    return f, m


def test_one_block_is_a_direct_solve():
    """With a single block covering the image the local problem is the global
    one, so one iteration from any admissible start gives the solution."""
    f, m = _case(0, 29, 31, 0.05)
    u0 = np.where(m != 0, f, 0.0)
    u1 = oracle.oras_step(u0, f, m, B=32, o=6, gamma=0.5)
    np.testing.assert_allclose(u1, oracle.solve_pcg(f, m)[0], atol=1e-9)


def test_solution_is_a_fixed_point():
    f, m = _case(1, 70, 45, 0.05)
    u = oracle.solve_pcg(f, m)[0]
    np.testing.assert_allclose(oracle.oras_step(u, f, m, B=16, o=4, gamma=0.4), u, atol=1e-9)


@pytest.mark.parametrize("gamma", [0.3, 1.0])
def test_iteration_converges_to_solution(gamma):
    f, m = _case(2, 40, 52, 0.08)
    exact = oracle.solve_pcg(f, m)[0]
    u = np.where(m != 0, f, 0.0)
    errs = []
    for _ in range(60):
        u = oracle.oras_step(u, f, m, B=16, o=4, gamma=gamma)
        errs.append(np.abs(u - exact).max())
    assert errs[-1] < 1e-6 * max(errs[0], 1.0)
    assert np.array_equal(u[m != 0], f[m != 0])


def test_local_matrix_rows():
    """Row sums of A_i: gamma per cut edge for unknown pixels with no known
    neighbour; RAS (gamma = 1) gives the principal submatrix of A."""
    rng = np.random.default_rng(3)
    H, W = 20, 20
    m = (rng.random((H, W)) < 0.1).astype(np.uint8)
    x0, y0, w, h = 4, 6, 8, 9
    Ai = oracle.oras_local_matrix(m, x0, y0, w, h, 1.0).toarray()
    A = oracle.dense_matrix(m)
    idx = [(y0 + ly) * W + (x0 + lx) for ly in range(h) for lx in range(w)]
    np.testing.assert_array_equal(Ai, A[np.ix_(idx, idx)])
    g = 0.37
    Ag = oracle.oras_local_matrix(np.zeros_like(m), x0, y0, w, h, g).toarray()
    rows = Ag.sum(axis=1).reshape(h, w)
    cuts = np.zeros((h, w))
    cuts[:, 0] += 1
    cuts[:, -1] += 1
    cuts[0, :] += 1
    cuts[-1, :] += 1
    np.testing.assert_allclose(rows, g * cuts, atol=1e-14)
