"""Batched solve through the C ABI: every problem's result is bit-identical to
the solve of that problem alone (same options), and meets the parity bar
against the oracle (relative residual <= 1e-6, known pixels bit-exact, max abs
error <= 0.5 grey levels)."""
import time

import numpy as np
import pytest

import oracle
from paper_2401_06744_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _mix(seed=0):
    """Uneven sizes, 1-4 channels, a single-level problem, thin strips."""
    spec = [(77, 53, 1, 0.05), (300, 17, 3, 0.05), (20, 24, 1, 0.2), (129, 257, 4, 0.02),
            (1, 100, 1, 0.1), (511, 383, 3, 0.04), (33, 33, 2, 0.1), (640, 360, 1, 0.01)]
    probs = []
    for k, (W, H, C, d) in enumerate(spec):
        probs.append((synth.frame_image(W, H, C, seed=seed + 10 * k + 1),
                      synth.bernoulli_mask(W, H, d, seed=seed + 10 * k + 2)))
    return probs


def _tol(kw):
    # plain FP32 CG stalls between 1e-6 and 1e-5 on the 1-2 % masks of this mix
    # (rounding of its updates against |u|), so it is held to 1e-5 here
    cg = (binding.SCHED_CG, binding.SCHED_CG_MULTILEVEL, binding.SCHED_CG_MULTIGRID)
    return 1e-5 if kw.get("schedule") in cg else TOL


def _solo(probs, **kw):
    opts = binding.make_opts(**kw) if kw else None
    return [binding.inpaint_solve_ex(f, m, _tol(kw), opts=opts)[0] for f, m in probs]


@pytest.mark.parametrize("kw", [
    {}, {"schedule": binding.SCHED_FMG}, {"schedule": binding.SCHED_MULTILEVEL},
    {"schedule": binding.SCHED_SINGLE}, {"pre_smooth": 2, "post_smooth": -1},
    {"pre_smooth": -1, "post_smooth": 2}, {"block": 16, "overlap": 4}, {"block": 64, "overlap": 8},
    {"precision": binding.PREC_FP16}, {"precision": binding.PREC_BF16}, {"schedule": binding.SCHED_CG},
    {"schedule": binding.SCHED_CG_MULTILEVEL}, {"schedule": binding.SCHED_CG_MULTIGRID},
])
def test_batched_equals_solo_bitwise(kw):
    probs = _mix()
    if kw.get("schedule") == binding.SCHED_SINGLE:
        probs = [probs[0], probs[2], probs[4], probs[6]]
    opts = binding.make_opts(**kw) if kw else None
    outs, st, stats = binding.inpaint_solve_batched(probs, _tol(kw), opts=opts)
    assert st == binding.OK
    solo = _solo(probs, **kw)
    for k, (o, s) in enumerate(zip(outs, solo)):
        assert stats[k]["status"] == binding.OK
        assert np.array_equal(o, s), f"problem {k} differs from its solo solve"


def test_batched_matches_oracle_and_reports_stats():
    probs = _mix(seed=100)
    outs, st, stats = binding.inpaint_solve_batched(probs, TOL)
    assert st == binding.OK
    for k, ((f, m), u) in enumerate(zip(probs, outs)):
        kn = m != 0
        for ch in range(f.shape[0]):
            assert np.array_equal(u[ch][kn], f[ch][kn])
        rr = oracle.rel_res(u.astype(np.float64), f.astype(np.float64), m)
        assert np.all(rr <= TOL), (k, rr)
        assert stats[k]["rel_res"] == pytest.approx(float(rr.max()), rel=1e-6, abs=1e-12)
        ref = oracle.solve_pcg(f.astype(np.float64), m)
        assert np.abs(u.astype(np.float64) - ref).max() <= 0.5
        assert stats[k]["levels"] == binding.inpaint_hierarchy_size(f.shape[2], f.shape[1])[0]
        assert stats[k]["gpu_ms"] > 0


def test_batched_device_pointers_repeat_and_alias():
    import torch
    probs = _mix(seed=200)
    ref, _, _ = binding.inpaint_solve_batched(probs, TOL)
    dev = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in probs]
    for _ in range(2):  # the second call reuses the cached plans and graphs
        outs, st, _ = binding.inpaint_solve_batched(dev, TOL)
        torch.cuda.synchronize()
        assert st == binding.OK
        for o, r in zip(outs, ref):
            assert np.array_equal(o.cpu().numpy(), r)
    alias = [(f.clone(), m, None) for f, m in dev]
    alias = [(f, m, f) for f, m, _ in alias]
    binding.inpaint_solve_batched(alias, TOL)
    torch.cuda.synchronize()
    for (f, _, _), r in zip(alias, ref):
        assert np.array_equal(f.cpu().numpy(), r)


def test_batched_rejected_problems_leave_the_others_alone():
    probs = _mix(seed=300)[:4]
    empty = (probs[1][0], np.zeros_like(probs[1][1]))
    g = probs[2][0].copy()
    k = np.argwhere(probs[2][1])[0]
    g[0, k[0], k[1]] = np.inf
    bad = [probs[0], empty, (g, probs[2][1]), probs[3]]
    outs, st, stats = binding.inpaint_solve_batched(bad, TOL, raise_on_error=False)
    assert st == binding.E_EMPTY_MASK
    assert [s["status"] for s in stats] == [binding.OK, binding.E_EMPTY_MASK, binding.E_INVALID,
                                            binding.OK]
    solo = _solo([probs[0], probs[3]])
    assert np.array_equal(outs[0], solo[0]) and np.array_equal(outs[3], solo[1])
    # the same workspaces with every problem valid again (plans are rebuilt)
    outs2, st2, _ = binding.inpaint_solve_batched(probs, TOL)
    assert st2 == binding.OK
    for o, s in zip(outs2, _solo(probs)):
        assert np.array_equal(o, s)
    # again with the rejected inputs: this call runs ahead without waiting for
    # the input checks, finds them failed and solves again
    outs3, st3, stats3 = binding.inpaint_solve_batched(bad, TOL, raise_on_error=False)
    assert st3 == binding.E_EMPTY_MASK
    assert [s["status"] for s in stats3] == [s["status"] for s in stats]
    assert np.array_equal(outs3[0], solo[0]) and np.array_equal(outs3[3], solo[1])


def _stats_key(stats):
    return [(s["status"], s["cycles"], s["oras_iters"], s["finest_block_solves"], s["rel_res"])
            for s in stats]


def test_batched_repeat_runs_ahead_with_identical_results():
    """A repeated batch issues the V-cycles its context needed last time before
    reading any convergence test back: outputs and statistics must equal those
    of the first call, which tested after every cycle."""
    probs = _mix(seed=700)
    first, st, stats = binding.inpaint_solve_batched(probs, TOL)
    assert st == binding.OK
    assert len({s["cycles"] for s in stats}) > 1  # members stop at different cycles
    for _ in range(2):
        again, st2, stats2 = binding.inpaint_solve_batched(probs, TOL)
        assert st2 == binding.OK
        assert _stats_key(stats2) == _stats_key(stats)
        for a, b in zip(again, first):
            assert np.array_equal(a, b)


def test_batched_running_ahead_too_far_changes_nothing():
    """Same shapes (the same batch context), easier masks after harder ones:
    the cycles issued ahead beyond convergence must leave results as solo."""
    hard = [(synth.frame_image(W, H, 3, seed=800 + k), synth.bernoulli_mask(W, H, 0.01, seed=810 + k))
            for k, (W, H) in enumerate([(301, 203), (160, 96)])]
    easy = [(f, synth.bernoulli_mask(f.shape[2], f.shape[1], 0.4, seed=820 + k))
            for k, (f, _) in enumerate(hard)]
    _, st, sh = binding.inpaint_solve_batched(hard, TOL)
    assert st == binding.OK
    outs, st, se = binding.inpaint_solve_batched(easy, TOL)
    assert st == binding.OK
    assert max(s["cycles"] for s in se) < max(s["cycles"] for s in sh)
    for o, s in zip(outs, _solo(easy)):
        assert np.array_equal(o, s)


def test_batched_running_ahead_too_short_finishes_on_the_host():
    """Same shapes, harder masks after easier ones: the cycles issued ahead
    do not reach convergence, so the output issued with them writes only the
    channels that stopped and the host finishes the rest: results as solo."""
    shapes = [(301, 203), (160, 96)]
    easy = [(synth.frame_image(W, H, 3, seed=830 + k), synth.bernoulli_mask(W, H, 0.4, seed=840 + k))
            for k, (W, H) in enumerate(shapes)]
    hard = [(f, synth.bernoulli_mask(f.shape[2], f.shape[1], 0.01, seed=850 + k))
            for k, (f, _) in enumerate(easy)]
    _, st, se = binding.inpaint_solve_batched(easy, TOL)
    assert st == binding.OK
    outs, st, sh = binding.inpaint_solve_batched(hard, TOL)
    assert st == binding.OK
    assert max(s["cycles"] for s in sh) > max(s["cycles"] for s in se)
    for o, s in zip(outs, _solo(hard)):
        assert np.array_equal(o, s)
    # one problem alone, the same way round (a batch of one reads its own flags)
    f, m = hard[0]
    binding.inpaint_solve_ex(easy[0][0], easy[0][1], TOL)
    u, st, s1 = binding.inpaint_solve_ex(f, m, TOL)
    assert st == binding.OK
    again, _, s2 = binding.inpaint_solve_ex(f, m, TOL)  # now ahead by the right count
    assert np.array_equal(u, again) and s1["cycles"] == s2["cycles"]
    assert np.array_equal(u, outs[0])
    assert np.all(oracle.rel_res(u.astype(np.float64), f.astype(np.float64), m) <= TOL)


def test_batched_in_place_run_ahead_with_a_rejected_problem():
    """Outputs aliasing the inputs in a call that runs ahead and then finds an
    input rejected: the valid problems, written once by the output issued
    ahead and solved again from those buffers, still end as solo (the solve
    reads f at known pixels only, which the output leaves as they were); the
    rejected problem's buffer is untouched."""
    import torch
    probs = _mix(seed=900)[:3]
    ref = _solo(probs)
    dev = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in probs]
    _, st, _ = binding.inpaint_solve_batched(dev, TOL)  # this context now runs ahead
    assert st == binding.OK
    bad = dev[1][0].clone()
    k = torch.nonzero(dev[1][1])[0]
    bad[0, k[0], k[1]] = float("nan")
    bad_before = bad.clone()
    items = [(dev[0][0].clone(), dev[0][1]), (bad, dev[1][1]), (dev[2][0].clone(), dev[2][1])]
    items = [(f, m, f) for f, m in items]
    _, st, stats = binding.inpaint_solve_batched(items, TOL, raise_on_error=False)
    torch.cuda.synchronize()
    assert st == binding.E_INVALID
    assert [s["status"] for s in stats] == [binding.OK, binding.E_INVALID, binding.OK]
    assert np.array_equal(items[0][0].cpu().numpy(), ref[0])
    assert np.array_equal(items[2][0].cpu().numpy(), ref[2])
    assert torch.equal(torch.nan_to_num(bad, nan=7.0), torch.nan_to_num(bad_before, nan=7.0))


def test_batched_argument_errors():
    probs = _mix()[:2]
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_batched([], TOL)
    assert e.value.code == binding.E_INVALID
    f, m = probs[0]
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_batched([probs[0], (np.zeros((5, 8, 8), np.float32),
                                                  np.ones((8, 8), np.uint8))], TOL)
    assert e.value.code == binding.E_INVALID
    shared = np.empty_like(f)
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_batched([(f, m, shared), (f, m, shared)], TOL)
    assert e.value.code == binding.E_INVALID
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_batched(probs, TOL, opts=binding.make_opts(block=24))
    assert e.value.code == binding.E_INVALID


def test_batched_not_converged_is_per_problem():
    probs = _mix(seed=400)[:3]
    outs, st, stats = binding.inpaint_solve_batched(probs, 1e-14,
                                                    opts=binding.make_opts(max_cycles=2),
                                                    raise_on_error=False)
    assert st == binding.NOT_CONVERGED
    for (f, m), u, s in zip(probs, outs, stats):
        assert s["status"] == binding.NOT_CONVERGED and s["cycles"] == 2
        assert np.array_equal(u[:, m != 0], f[:, m != 0])


def test_autotune_picks_a_converging_configuration_and_caches_it(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("INPAINT_AUTOTUNE_CACHE", str(cache))
    probs = _mix(seed=500)[:5]
    t0 = time.perf_counter()
    best, ms = binding.inpaint_autotune(probs, TOL)
    first = time.perf_counter() - t0
    assert best.block in (16, 32, 64) and 2 <= best.overlap <= best.block // 2
    assert best.schedule in (binding.SCHED_RFMG, binding.SCHED_FMG)
    assert ms > 0
    t0 = time.perf_counter()
    again, ms2 = binding.inpaint_autotune(probs, TOL)
    assert time.perf_counter() - t0 < first
    assert (again.block, again.overlap, again.schedule, ms2) == (best.block, best.overlap, best.schedule, ms)
    assert cache.exists() and cache.read_text().count("\n") >= 1
    outs, st, _ = binding.inpaint_solve_batched(probs, TOL, opts=best)
    assert st == binding.OK
    for (f, m), u in zip(probs, outs):
        rr = oracle.rel_res(u.astype(np.float64), f.astype(np.float64), m)
        assert np.all(rr <= TOL)
