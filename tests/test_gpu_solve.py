"""GPU solve vs the CPU oracle through the C ABI (parity gate: max abs error <= 0.5
grey levels on [0, 255], relative residual <= 1e-6, known pixels bit-exact)."""
import numpy as np
import pytest

import oracle
from paper_2401_06744_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = 1e-6
MAX_ERR = 0.5


def _torch():
    import torch
    return torch


def _check(u, f, m, ref=None, rr_tol=TOL, err_tol=MAX_ERR):
    u = np.asarray(u, dtype=np.float32)
    f3 = f if f.ndim == 3 else f[None]
    u3 = u if u.ndim == 3 else u[None]
    k = m != 0
    for ch in range(f3.shape[0]):
        assert np.array_equal(u3[ch][k], f3[ch][k]), "known pixels must be reproduced bit-exactly"
    rr = oracle.rel_res(u3.astype(np.float64), f3.astype(np.float64), m)
    assert np.all(rr <= rr_tol), rr
    if ref is None:
        ref = oracle.solve_pcg(f3.astype(np.float64), m)
    err = np.abs(u3.astype(np.float64) - ref).max()
    assert err <= err_tol, err
    return rr, err


def _solve(f, m, tol=TOL, **kw):
    opts = binding.make_opts(**kw) if kw else None
    out, st, stats = binding.inpaint_solve_ex(f, m, tol, opts=opts)
    return out, st, stats


def test_small_config_256():
    f, m = synth.config_small()
    out, st, stats = _solve(f, m)
    assert st == binding.OK
    assert stats["levels"] == 4
    _check(out, f, m)


@pytest.mark.parametrize("W,H,C,dens,seed", [
    (77, 53, 1, 0.05, 1), (33, 33, 3, 0.04, 2), (65, 31, 2, 0.1, 3), (300, 17, 1, 0.05, 4),
    (129, 257, 4, 0.02, 5), (1, 100, 1, 0.1, 6), (100, 1, 1, 0.1, 7), (32, 32, 1, 0.05, 8),
    (58, 59, 1, 0.01, 9), (511, 383, 3, 0.04, 10), (1000, 3, 1, 0.05, 11), (2, 2, 1, 0.5, 12),
])
def test_ragged_sizes(W, H, C, dens, seed):
    f = synth.frame_image(W, H, C, seed=seed)
    m = synth.bernoulli_mask(W, H, dens, seed=seed + 100)
    out, st, _ = _solve(f, m)
    assert st == binding.OK
    _check(out, f, m)


def test_local_residuals_reaching_subnormal_range():
    """Regression: in this problem (659x467 RGB, 9.4 % mask) some local CG
    solves drive their squared residual norm below the smallest normal
    float32; a hardware reciprocal of such a value is inf and used to turn the
    whole solve into NaN."""
    f, m = synth.batched_problems()[60]
    assert f.shape == (3, 467, 659)
    out, st, stats = _solve(f, m)
    assert st == binding.OK and np.isfinite(out).all()
    assert np.array_equal(out[:, m != 0], f[:, m != 0])
    rr = oracle.rel_res(out.astype(np.float64), f.astype(np.float64), m)
    assert np.all(rr <= TOL), rr


CG_TOL = 1e-5


@pytest.mark.parametrize("W,H,C,dens,seed", [
    (77, 53, 1, 0.05, 1), (300, 17, 3, 0.05, 4), (129, 257, 2, 0.02, 5), (1, 100, 1, 0.1, 6),
    (256, 256, 1, 0.05, 2),
])
def test_cg_schedule_matches_oracle(W, H, C, dens, seed):
    """The comparison schedule (plain CG on the finest grid) reaches the oracle's
    solution within the 0.5 grey-level bound.  Its gate is 1e-5: in FP32, CG's
    updates round away against |u| once the relative residual nears 1e-6 (more
    so the sparser the mask), so it can stall between 1e-6 and 1e-5."""
    f = synth.frame_image(W, H, C, seed=seed)
    m = synth.bernoulli_mask(W, H, dens, seed=seed + 100)
    out, st, stats = _solve(f, m, tol=CG_TOL, schedule=binding.SCHED_CG)
    assert st == binding.OK
    assert stats["cycles"] >= 1 and stats["oras_iters"] == C * (8 * stats["cycles"] + 1)
    _check(out, f, m, rr_tol=CG_TOL)


@pytest.mark.parametrize("sched", ["CG_MULTILEVEL", "CG_MULTIGRID"])
@pytest.mark.parametrize("W,H,C,dens,seed", [
    (77, 53, 1, 0.05, 1), (300, 17, 3, 0.05, 4), (129, 257, 2, 0.02, 5), (1, 100, 1, 0.1, 6),
    (20, 24, 1, 0.2, 7), (256, 256, 1, 0.05, 2), (2048, 64, 1, 0.04, 8),
])
def test_cg_counterparts_match_oracle(sched, W, H, C, dens, seed):
    """The multilevel and multigrid CG counterparts (CG in place of ORAS in
    the same cascade and V-cycles; 20x24 is a single-level problem) reach the
    oracle's solution, held to the same gate as plain CG.  On 2048x64 the
    max-pooled masks of the deepest levels are fully known, so CG there starts
    from r = 0."""
    f = synth.frame_image(W, H, C, seed=seed)
    m = synth.bernoulli_mask(W, H, dens, seed=seed + 100)
    out, st, stats = _solve(f, m, tol=CG_TOL, schedule=getattr(binding, "SCHED_" + sched))
    assert st == binding.OK
    _check(out, f, m, rr_tol=CG_TOL)


@pytest.mark.parametrize("sched", ["CG_MULTILEVEL", "CG_MULTIGRID"])
@pytest.mark.parametrize("nu", [1, 2, 8])
def test_cg_counterparts_smoothing_counts(sched, nu):
    """Any number of CG iterations per smoothing, on a frame deep enough
    (960x540, six levels) that its coarse levels are fully known."""
    f = synth.frame_image(960, 540, 1, seed=9)
    m = synth.bernoulli_mask(960, 540, 0.04, seed=109)
    out, st, stats = _solve(f, m, tol=CG_TOL, schedule=getattr(binding, "SCHED_" + sched),
                            pre_smooth=nu, post_smooth=nu)
    assert st == binding.OK
    _check(out, f, m, rr_tol=CG_TOL)


def test_cg_schedule_stops_when_it_stalls():
    """On a 1 % mask float32 CG stalls above 1e-6: the solve gives up after 16
    tests without a 1 % improvement (long before the 500-cycle cap), reports
    NOT_CONVERGED with the relative residual it reached, and its output still
    meets the grey-level bound."""
    f = synth.frame_image(640, 360, 1, seed=71)
    m = synth.bernoulli_mask(640, 360, 0.01, seed=72)
    out, st, stats = _solve(f, m, tol=TOL, schedule=binding.SCHED_CG)
    assert st == binding.NOT_CONVERGED
    assert 16 < stats["cycles"] < 120
    assert TOL < stats["rel_res"] <= CG_TOL
    _check(out, f, m, rr_tol=CG_TOL)


def test_cg_schedule_is_float32_only():
    f, m = synth.config_small()
    with pytest.raises(binding.InpaintError) as e:
        _solve(f, m, schedule=binding.SCHED_CG, precision=binding.PREC_FP16)
    assert e.value.code == binding.E_INVALID
    with pytest.raises(binding.InpaintError) as e:
        _solve(f, m, schedule=binding.SCHED_CG_MULTIGRID, precision=binding.PREC_BF16)
    assert e.value.code == binding.E_INVALID


def test_single_pixel_and_all_known():
    f = synth.plain_image(40, 30, seed=3)
    m = np.zeros((30, 40), np.uint8)
    m[11, 7] = 1
    out, st, _ = _solve(f, m)
    assert st == binding.OK
    np.testing.assert_allclose(out[0], f[0, 11, 7], atol=1e-3)
    m1 = np.ones((30, 40), np.uint8)
    out1, st1, _ = _solve(f, m1)
    assert st1 == binding.OK and np.array_equal(out1, f)
    one = np.array([[[5.0]]], np.float32)
    o1, s1, _ = _solve(one, np.ones((1, 1), np.uint8))
    assert s1 == binding.OK and o1[0, 0, 0] == 5.0


@pytest.mark.parametrize("sched", ["CG", "CG_MULTILEVEL", "CG_MULTIGRID"])
def test_cg_schedules_all_known_and_one_pixel(sched):
    """Degenerate inputs of the comparison schedules: with every pixel known
    the residual and every CG scalar are 0 from the start (no 0/0 may leak
    into the output), and a 1x1 image is its own coarsest level."""
    kw = {"schedule": getattr(binding, "SCHED_" + sched)}
    f = synth.plain_image(40, 30, seed=3)
    out1, st1, _ = _solve(f, np.ones((30, 40), np.uint8), tol=CG_TOL, **kw)
    assert st1 == binding.OK and np.array_equal(out1, f)
    one = np.array([[[5.0]]], np.float32)
    o1, s1, _ = _solve(one, np.ones((1, 1), np.uint8), tol=CG_TOL, **kw)
    assert s1 == binding.OK and o1[0, 0, 0] == 5.0


def test_ramp_with_known_border():
    H, W = 96, 130
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = (20.0 + 1.2 * x + 0.5 * y).astype(np.float32)[None]
    m = synth.bernoulli_mask(W, H, 0.03, seed=4)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = 1
    out, st, _ = _solve(f, m)
    assert st == binding.OK
    np.testing.assert_allclose(out[0], f[0], atol=5e-3)


def test_row_closed_form():
    W = 700
    rng = np.random.default_rng(5)
    f = rng.uniform(0, 255, (1, 1, W)).astype(np.float32)
    m = (rng.random((1, W)) < 0.05).astype(np.uint8)
    m[0, 3] = 1
    out, st, _ = _solve(f, m)
    xs = np.nonzero(m[0])[0]
    expect = np.interp(np.arange(W), xs, f[0, 0, xs].astype(np.float64))
    assert st == binding.OK
    np.testing.assert_allclose(out[0, 0], expect, atol=1e-2)


def test_errors():
    f, m = synth.config_small(40, 40)
    with pytest.raises(binding.InpaintError) as e:
        _solve(f, np.zeros_like(m))
    assert e.value.code == binding.E_EMPTY_MASK
    g = f.copy()
    k = np.argwhere(m)[0]
    g[0, k[0], k[1]] = np.nan
    with pytest.raises(binding.InpaintError) as e:
        _solve(g, m)
    assert e.value.code == binding.E_INVALID
    for bad in ({"block": 24}, {"block": 128}, {"overlap": 1}, {"overlap": 3}, {"overlap": 17}, {"gamma": 1.5}, {"schedule": 9}):
        with pytest.raises(binding.InpaintError) as e:
            _solve(f, m, **bad)
        assert e.value.code == binding.E_INVALID
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_ex(f, m, 0.0)
    assert e.value.code == binding.E_INVALID


def test_not_converged_writes_iterate():
    f, m = synth.config_small(128, 128, 0.01)
    out, st, stats = _solve(f, m, tol=1e-15, max_cycles=2)
    assert st == binding.NOT_CONVERGED
    assert stats["cycles"] == 2
    assert np.array_equal(out[0][m != 0], f[0][m != 0])
    assert oracle.rel_res(out.astype(np.float64), f.astype(np.float64), m)[0] < 1e-2


def test_unknown_values_never_read_and_channels_independent():
    f = synth.frame_image(150, 90, 3, seed=21)
    m = synth.bernoulli_mask(150, 90, 0.04, seed=22)
    out, _, _ = _solve(f, m)
    g = f.copy()
    g[:, m == 0] = np.nan
    out2, _, _ = _solve(g, m)
    assert np.array_equal(out, out2)
    for ch in range(3):
        single, _, _ = _solve(np.ascontiguousarray(f[ch:ch + 1]), m)
        assert np.array_equal(single[0], out[ch])


def _overflowing(f, m, ch, value=1e6):
    """f with the known pixels of channel ch set to +-value in a checkerboard:
    finite data beyond the float16 range (65504), which the float16 form's
    coarse known values and iterates (stored unscaled) cannot hold."""
    g = f.copy()
    ys, xs = np.nonzero(m)
    g[ch, ys, xs] = np.where((ys + xs) % 2 == 0, value, -value).astype(np.float32)
    return g


def test_overflowing_known_values_diverge_alone():
    """A channel whose residual becomes non-finite stops as diverged: in the
    float16 form, known values beyond the float16 range overflow the coarse
    levels' 16-bit fields, and the solve returns E_DIVERGED with rel_res NaN,
    while the problem's other channels and the other problems of a batch are
    solved exactly as alone."""
    opts = binding.make_opts(precision=binding.PREC_FP16)
    f = synth.frame_image(150, 90, 3, seed=41)
    m = synth.bernoulli_mask(150, 90, 0.05, seed=42)
    g = _overflowing(f, m, 1)
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_ex(g, m, TOL, opts=opts)
    assert e.value.code == binding.E_DIVERGED
    a = (synth.frame_image(97, 61, 1, seed=43), synth.bernoulli_mask(97, 61, 0.03, seed=44))
    outs, st, stats = binding.inpaint_solve_batched([a, (g, m)], TOL, opts=opts, raise_on_error=False)
    assert st == binding.E_DIVERGED
    assert stats[0]["status"] == binding.OK and stats[1]["status"] == binding.E_DIVERGED
    assert np.isnan(stats[1]["rel_res"])
    assert np.array_equal(outs[0], binding.inpaint_solve_ex(*a, TOL, opts=opts)[0])
    for ch in (0, 2):
        single, st1, _ = binding.inpaint_solve_ex(np.ascontiguousarray(f[ch:ch + 1]), m, TOL, opts=opts)
        assert st1 == binding.OK and np.array_equal(outs[1][ch], single[0]), ch
    # the diverged channel stops at its first non-finite test, not at the cycle cap
    assert stats[1]["cycles"] < 30
    # the same values are within float32's range: the float32 form does not diverge
    out32, st32, _ = binding.inpaint_solve_ex(g, m, TOL)
    assert st32 in (binding.OK, binding.NOT_CONVERGED)
    assert np.array_equal(out32[:, m != 0], g[:, m != 0])


def test_repeatable_and_device_pointers_and_alias():
    torch = _torch()
    f = synth.frame_image(200, 120, 3, seed=31)
    m = synth.bernoulli_mask(200, 120, 0.05, seed=32)
    a, _, _ = _solve(f, m)
    b, _, _ = _solve(f, m)
    assert np.array_equal(a, b), "run-to-run results must be bitwise identical"
    fd = torch.from_numpy(f).cuda()
    md = torch.from_numpy(m).cuda()
    od, st, _ = binding.inpaint_solve_ex(fd, md, TOL)
    torch.cuda.synchronize()
    assert st == binding.OK and np.array_equal(od.cpu().numpy(), a)
    al = fd.clone()
    binding.inpaint_solve_ex(al, md, TOL, out=al)
    torch.cuda.synchronize()
    assert np.array_equal(al.cpu().numpy(), a)


@pytest.mark.parametrize("kw", [
    {"schedule": binding.SCHED_FMG}, {"schedule": binding.SCHED_MULTILEVEL},
    {"block": 16, "overlap": 4}, {"overlap": 2}, {"overlap": 16, "block": 32},
    {"block": 64, "overlap": 8}, {"block": 64, "overlap": 32}, {"block": 64, "overlap": 6,
                                                                 "precision": binding.PREC_FP16},
    {"gamma": 1.0}, {"rhs_restriction": binding.RHS_NAIVE}, {"pre_smooth": 2, "post_smooth": 2},
    {"post_smooth": -1, "pre_smooth": 2}, {"pre_smooth": -1, "post_smooth": 2},
])
def test_options_reach_the_same_solution(kw):
    f = synth.frame_image(180, 140, 1, seed=41)
    m = synth.bernoulli_mask(180, 140, 0.05, seed=42)
    out, st, _ = _solve(f, m, **kw)
    assert st == binding.OK
    _check(out, f, m)


def test_single_level_schedule():
    f = synth.frame_image(64, 48, 1, seed=51)
    m = synth.bernoulli_mask(64, 48, 0.1, seed=52)
    out, st, stats = _solve(f, m, schedule=binding.SCHED_SINGLE)
    assert st == binding.OK
    _check(out, f, m)


def test_rel_res_entry_point_matches_oracle():
    f = synth.frame_image(123, 77, 2, seed=61)
    m = synth.bernoulli_mask(123, 77, 0.05, seed=62)
    rng = np.random.default_rng(63)
    u = np.where(m[None] != 0, f, rng.uniform(0, 255, f.shape)).astype(np.float32)
    got = binding.inpaint_rel_res(u, f, m)
    ref = oracle.rel_res(u.astype(np.float64), f.astype(np.float64), m)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("prec", [binding.PREC_FP16, binding.PREC_BF16])
@pytest.mark.parametrize("W,H,C,dens,seed", [
    (256, 256, 1, 0.05, 1), (301, 157, 3, 0.01, 2), (77, 53, 2, 0.1, 3), (1000, 3, 1, 0.05, 4),
    (31, 29, 1, 0.05, 5),
])
def test_precision_forms_match_oracle(prec, W, H, C, dens, seed):
    """16-bit correction storage with float64 residuals reaches the same tolerance."""
    f = synth.frame_image(W, H, C, seed=seed)
    m = synth.bernoulli_mask(W, H, dens, seed=seed + 7)
    out, st, _ = _solve(f, m, precision=prec)
    assert st == binding.OK
    _check(out, f, m)


def test_precision_forms_are_repeatable_and_channel_independent():
    f = synth.frame_image(160, 96, 3, seed=71)
    m = synth.bernoulli_mask(160, 96, 0.03, seed=72)
    for prec in (binding.PREC_FP16, binding.PREC_BF16):
        a, _, _ = _solve(f, m, precision=prec)
        b, _, _ = _solve(f, m, precision=prec)
        assert np.array_equal(a, b)
        single, _, _ = _solve(np.ascontiguousarray(f[1:2]), m, precision=prec)
        assert np.array_equal(single[0], a[1])


def test_workspace_cache_is_bounded():
    """Idle hierarchies beyond the cache limit are freed (least recently used
    first) and rebuilt when needed again; results do not change."""
    shapes = [(300, 200, 1), (400, 300, 3), (500, 250, 1)]
    probs = [(synth.frame_image(W, H, C, seed=90 + k), synth.bernoulli_mask(W, H, 0.04, seed=95 + k))
             for k, (W, H, C) in enumerate(shapes)]
    ref = [_solve(f, m)[0] for f, m in probs]
    try:
        assert binding.inpaint_cache_limit(1 << 20) <= 1 << 20  # idle hierarchies are freed now
        for _ in range(2):
            for (f, m), r in zip(probs, ref):
                assert np.array_equal(_solve(f, m)[0], r)
                assert binding.inpaint_cache_limit(0) == 0  # nothing idle stays above the limit
        outs, st, _ = binding.inpaint_solve_batched(probs, TOL)
        assert st == binding.OK and all(np.array_equal(o, r) for o, r in zip(outs, ref))
        assert binding.inpaint_cache_limit(0) == 0
        # a limit that holds one of them: the most recent stays
        binding.inpaint_cache_limit(64 << 20)
        for f, m in probs:
            _solve(f, m)
        left = binding.inpaint_cache_limit(0)
        assert 0 < left <= 64 << 20
    finally:
        binding.inpaint_cache_limit(16 << 30)


def _zero_reference_residual_problem():
    """Channel 0: every known pixel next to an unknown one is 0, so
    ||b - A C f|| = 0 and C f is the exact solution, although known pixels
    inside a solid known patch are not 0 (the coarse levels see them).
    Channel 1: an ordinary image on the same mask."""
    W, H = 150, 90
    m = synth.bernoulli_mask(W, H, 0.04, seed=71)
    m[30:50, 40:70] = 1
    f = synth.frame_image(W, H, 2, seed=72)
    f[0][m != 0] = 0.0
    f[0][31:49, 41:69] = 200.0  # the patch's interior: every neighbour is known
    return np.ascontiguousarray(f), m


@pytest.mark.parametrize("sched", ["RFMG", "FMG", "MULTILEVEL", "SINGLE", "CG"])
def test_zero_reference_residual_returns_c_f(sched):
    """The relative residual's denominator is 0 for channel 0: the solve
    returns C f there (the exact solution, rel-res 0) and channel 1 as
    usual; from a warm guess too."""
    f, m = _zero_reference_residual_problem()
    k = m != 0
    exact = np.where(k, f[0], 0.0).astype(np.float32)
    ref1 = oracle.solve_pcg(f[1:2].astype(np.float64), m)
    assert np.array_equal(oracle.solve_pcg(f[0:1].astype(np.float64), m)[0], exact)
    runs = [binding.make_opts(schedule=getattr(binding, "SCHED_" + sched))]
    if sched == "RFMG":
        runs.append(binding.make_opts(schedule=binding.SCHED_WARM))
        runs.append(binding.make_opts(precision=binding.PREC_FP16))
    tol = 1e-5 if sched == "CG" else TOL  # float32 CG stalls near 1e-6
    for opts in runs:
        out = np.random.default_rng(5).uniform(0, 255, f.shape).astype(np.float32)
        _, st, stats = binding.inpaint_solve_ex(f, m, tol, out=out, opts=opts)
        assert st == binding.OK, (sched, st)
        assert np.array_equal(out[0], exact), sched
        assert stats["rel_res"] <= tol
        _check(out[1:2], f[1:2], m, ref=ref1, rr_tol=tol)


@pytest.mark.parametrize("prec", [binding.PREC_FP32, binding.PREC_FP16, binding.PREC_BF16])
def test_single_known_pixel_gives_a_constant(prec):
    """One known pixel: the solution is that value everywhere (the constant is
    discrete-harmonic under reflecting boundaries), a purely global,
    low-frequency error for the coarse levels to remove."""
    W, H = 301, 203
    vals = np.array([137.5, 3.25, 250.0], np.float32)
    f = np.zeros((3, H, W), np.float32)
    m = np.zeros((H, W), np.uint8)
    m[150, 40] = 1
    f[:, 150, 40] = vals
    out, st, stats = _solve(f, m, precision=prec)
    assert st == binding.OK
    for ch in range(3):
        assert np.abs(out[ch].astype(np.float64) - vals[ch]).max() <= 0.5, (ch, prec)
    rr = oracle.rel_res(out.astype(np.float64), f.astype(np.float64), m)
    assert np.all(rr <= TOL), rr


def test_any_nonzero_mask_byte_marks_a_known_pixel():
    """The mask is read as known = (byte != 0): 1, 255 or any other nonzero
    byte give the same result bit for bit, solo and batched."""
    f = synth.frame_image(173, 111, 3, seed=91)
    m = synth.bernoulli_mask(173, 111, 0.05, seed=92)
    rng = np.random.default_rng(93)
    m_any = np.where(m != 0, rng.integers(1, 256, m.shape), 0).astype(np.uint8)
    base, st, _ = _solve(f, m)
    assert st == binding.OK
    for mm in (m * 255, m_any):
        out, st, _ = _solve(f, np.ascontiguousarray(mm))
        assert st == binding.OK and np.array_equal(out, base)
    outs, st, _ = binding.inpaint_solve_batched([(f, m_any), (f, m)], TOL)
    assert st == binding.OK and np.array_equal(outs[0], base) and np.array_equal(outs[1], base)


def test_concurrent_calls_from_threads_match_sequential_ones():
    """The entry points are thread-safe: four host threads solving at once
    (two of them on problems of the same size, so that the cache hands out
    separate workspaces) give the sequential results bit for bit."""
    import threading
    probs = [(synth.frame_image(W, H, C, seed=100 + k), synth.bernoulli_mask(W, H, 0.04, seed=110 + k))
             for k, (W, H, C) in enumerate([(320, 180, 3), (320, 180, 3), (97, 61, 1), (640, 360, 2)])]
    seq = []
    for f, m in probs:
        out, st, _ = _solve(f, m)
        assert st == binding.OK
        seq.append(out)
    got = [[None] * 3 for _ in probs]
    errors = []

    def work(i):
        try:
            for r in range(3):
                out, st, _ = _solve(*probs[i])
                got[i][r] = out if st == binding.OK else None
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(probs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=90)
    assert not any(t.is_alive() for t in threads), "a solving thread did not finish"
    assert not errors, errors
    for i, outs in enumerate(got):
        for out in outs:
            assert out is not None and np.array_equal(out, seq[i]), i


def test_solve_on_a_caller_stream():
    """Work issued on the caller's stream (a torch stream at the default
    priority), with the inputs written on that stream just before the call:
    the results equal those on the null stream, solo, batched and without
    allocation."""
    import torch
    f = synth.frame_image(256, 160, 3, seed=121)
    m = synth.bernoulli_mask(256, 160, 0.05, seed=122)
    base, st, _ = _solve(f, m)
    assert st == binding.OK
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fd = torch.from_numpy(f).cuda(non_blocking=False)
        md = torch.from_numpy(m).cuda(non_blocking=False)
        fd.mul_(1.0)  # pending work on s when the solve is issued
        od = torch.empty_like(fd)
    _, st, _ = binding.inpaint_solve_ex(fd, md, TOL, out=od, stream=s)
    assert st == binding.OK and np.array_equal(od.cpu().numpy(), base)
    with torch.cuda.stream(s):
        od2 = torch.empty_like(fd)
    outs, st, _ = binding.inpaint_solve_batched([(fd, md, od2)], TOL, stream=s)
    assert st == binding.OK and np.array_equal(od2.cpu().numpy(), base)
    with torch.cuda.stream(s):
        od3 = torch.empty_like(fd)
    _, st, _ = binding.inpaint_solve_noalloc(fd, md, TOL, out=od3, stream=s)
    s.synchronize()
    assert st == binding.OK and np.array_equal(od3.cpu().numpy(), base)
