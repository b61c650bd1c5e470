"""Step-level parity of the HIP kernels against the oracle (coarse problems, grid
transfers and one ORAS iteration), through the C ABI's step entry points."""
import numpy as np
import pytest

import oracle
from paper_2401_06744_amd import binding, synth

pytestmark = pytest.mark.gpu


def _f32_close(got, ref, ulps=1):
    """float32 result vs a float64 reference rounded to float32, within `ulps`."""
    ref32 = np.asarray(ref, dtype=np.float64).astype(np.float32)
    got = np.asarray(got, dtype=np.float32)
    sp = np.spacing(np.maximum(np.abs(ref32), np.float32(1e-30)).astype(np.float32))
    assert np.all(np.abs(got.astype(np.float64) - ref32.astype(np.float64)) <= ulps * sp.astype(np.float64))


@pytest.mark.parametrize("W,H,dens,rhs", [
    (256, 256, 0.05, binding.RHS_MODIFIED), (301, 157, 0.02, binding.RHS_MODIFIED),
    (97, 33, 0.3, binding.RHS_NAIVE), (640, 360, 0.01, binding.RHS_MODIFIED),
])
def test_pyramid_matches_oracle(W, H, dens, rhs):
    f = synth.frame_image(W, H, 2, seed=7)
    m = synth.bernoulli_mask(W, H, dens, seed=8)
    levels = binding.inpaint_debug_pyramid(f, m, block=32, rhs_restriction=rhs)
    sizes = oracle.level_sizes(W, H, 32)
    assert [(lv[0].shape[1], lv[0].shape[0]) for lv in levels] == sizes
    assert np.array_equal(levels[0][0], (m != 0).astype(np.uint8))
    assert np.array_equal(levels[0][1], np.where(m[None] != 0, f, 0))
    down = oracle.rhs_down_naive if rhs == binding.RHS_NAIVE else oracle.rhs_down_modified
    for l in range(1, len(levels)):
        cf, bf = levels[l - 1]
        cc, bc = levels[l]
        assert np.array_equal(cc, oracle.mask_down(cf)), f"mask level {l}"
        for ch in range(bf.shape[0]):
            _f32_close(bc[ch], down(cf, bf[ch].astype(np.float64)), ulps=1)


@pytest.mark.parametrize("Wf,Hf,seed", [(64, 64, 1), (77, 39, 2), (3, 200, 3), (130, 1, 4)])
def test_restrict_matches_oracle(Wf, Hf, seed):
    rng = np.random.default_rng(seed)
    r = rng.normal(0, 10, (Hf, Wf)).astype(np.float32)
    cc = (rng.random(((Hf + 1) // 2, (Wf + 1) // 2)) < 0.2).astype(np.uint8)
    got = binding.inpaint_debug_restrict(r, cc)
    _f32_close(got, oracle.restrict_residual(r.astype(np.float64), cc), ulps=1)


@pytest.mark.parametrize("Wf,Hf,seed", [(64, 64, 1), (77, 39, 2), (5, 130, 3), (131, 2, 4)])
def test_prolong_matches_oracle(Wf, Hf, seed):
    rng = np.random.default_rng(seed)
    Wc, Hc = (Wf + 1) // 2, (Hf + 1) // 2
    uc = rng.uniform(0, 255, (Hc, Wc)).astype(np.float32)
    mf = (rng.random((Hf, Wf)) < 0.1).astype(np.uint8)
    bf = np.where(mf != 0, rng.uniform(0, 255, (Hf, Wf)), 0).astype(np.float32)
    p = oracle.prolong_bilinear(uc.astype(np.float64), Wf, Hf)
    got0 = binding.inpaint_debug_prolong(uc, mf, bf, mode=0)
    assert np.array_equal(got0[mf != 0], bf[mf != 0])
    _f32_close(got0[mf == 0], p[mf == 0], ulps=1)
    uin = rng.uniform(0, 255, (Hf, Wf)).astype(np.float32)
    got1 = binding.inpaint_debug_prolong(uc, mf, bf, u_in=uin, mode=1)
    assert np.array_equal(got1[mf != 0], uin[mf != 0])
    _f32_close(got1[mf == 0], (uin.astype(np.float64) + p)[mf == 0], ulps=1)


@pytest.mark.parametrize("W,H,B,o,gamma", [
    (100, 70, 32, 6, 0.5), (64, 64, 16, 4, 1.0), (45, 90, 32, 2, 0.3), (31, 29, 32, 6, 0.5),
    (150, 33, 16, 8, 0.7), (150, 100, 64, 8, 0.5), (61, 130, 64, 6, 0.3),
])
def test_oras_step_matches_oracle(W, H, B, o, gamma):
    """With the local CG run to convergence, one GPU ORAS iteration equals the
    oracle's iteration with exact local solves (Algorithm 2)."""
    f = synth.frame_image(W, H, 1, seed=3)
    m = synth.bernoulli_mask(W, H, 0.05, seed=4)
    rng = np.random.default_rng(5)
    u0 = np.where(m != 0, f[0], rng.uniform(0, 255, (H, W))).astype(np.float32)
    opts = binding.make_opts(block=B, overlap=o, gamma=gamma, tau=1e-14, max_local_iters=4 * B * B)
    got = binding.inpaint_debug_oras_step(u0[None], f, m, opts)[0]
    ref = oracle.oras_step(u0.astype(np.float64), f[0].astype(np.float64), m, B=B, o=o, gamma=gamma)
    assert np.array_equal(got[m != 0], f[0][m != 0])
    np.testing.assert_allclose(got, ref, atol=2e-3, rtol=0)
