"""The solve without device allocation (inpaint_solve_noalloc) against the
allocating solve (inpaint_solve_ex) with the same options, through the C ABI:
two calls in a row on the fixed device array, the second with a smaller
problem, each bit for bit equal to the allocating solve; sizes beyond the
array, host pointers and the CG schedules are rejected before any device work.
"""
import numpy as np
import pytest

import oracle
from paper_2401_06744_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _dev(f, m):
    import torch
    return torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()


def _both(fd, md, opts):
    import torch
    ref, st_ref, _ = binding.inpaint_solve_ex(fd, md, TOL, opts=opts)
    out, st, stats = binding.inpaint_solve_noalloc(fd, md, TOL, opts=opts)
    torch.cuda.synchronize()
    assert st == st_ref == binding.OK
    return ref.cpu().numpy(), out.cpu().numpy(), stats


@pytest.mark.parametrize("prec", [binding.PREC_FP32, binding.PREC_FP16])
def test_two_calls_in_a_row_match_the_allocating_solve(prec):
    opts = binding.make_opts(precision=prec)
    cases = [synth.frame_image(640, 360, 3, seed=61), synth.bernoulli_mask(640, 360, 0.03, seed=62)], \
        list(synth.config_small(W=256, H=256, density=0.05))
    for k, (f, m) in enumerate(cases):
        print(f"no-alloc case {k}: {f.shape} precision {prec}", flush=True)
        fd, md = _dev(f, m)
        ref, out, stats = _both(fd, md, opts)
        assert np.array_equal(out, ref), k
        kn = m != 0
        assert np.array_equal(out[:, kn], f[:, kn])
        rr = oracle.rel_res(out.astype(np.float64), f.astype(np.float64), m)
        assert np.all(rr <= TOL), rr
        assert stats["cycles"] >= 1 and stats["levels"] >= 2
    # the smaller problem's result also matches the oracle within the gate
    f, m = cases[1]
    err = np.abs(out.astype(np.float64) - oracle.solve_pcg(f.astype(np.float64), m)).max()
    assert err <= 0.5, err


def test_single_level_and_schedules():
    """A problem that is its own coarsest grid, and the other ORAS schedules."""
    f, m = synth.config_small(W=30, H=20, density=0.1)
    fd, md = _dev(f, m)
    ref, out, _ = _both(fd, md, None)
    assert np.array_equal(out, ref)
    f, m = synth.config_small(W=200, H=120, density=0.05)
    fd, md = _dev(f, m)
    for sched in (binding.SCHED_FMG, binding.SCHED_MULTILEVEL):
        ref, out, _ = _both(fd, md, binding.make_opts(schedule=sched))
        assert np.array_equal(out, ref), sched


def test_rejections_before_device_work():
    import torch
    # 3840x2160 RGB needs about 0.7 GB: more than the array holds
    f = torch.zeros((3, 2160, 3840), dtype=torch.float32, device="cuda")
    m = torch.zeros((2160, 3840), dtype=torch.uint8, device="cuda")
    m[0, 0] = 1
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_noalloc(f, m, TOL)
    assert e.value.code == binding.E_INVALID and "bytes" in str(e.value)
    fh, mh = synth.config_small(W=64, H=64, density=0.05)
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_noalloc(fh, mh, TOL)
    assert e.value.code == binding.E_INVALID
    fd, md = _dev(fh, mh)
    with pytest.raises(binding.InpaintError) as e:
        binding.inpaint_solve_noalloc(fd, md, TOL, opts=binding.make_opts(schedule=binding.SCHED_CG))
    assert e.value.code == binding.E_INVALID
    # the array still works after the rejections
    ref, out, _ = _both(fd, md, None)
    assert np.array_equal(out, ref)
