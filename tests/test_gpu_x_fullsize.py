"""Full-size parity: every channel of the full-size workloads against the
oracle's solution (float64 Jacobi-PCG to rel-res 1e-12), at the gate of the
method's statement of accuracy: max abs error <= 0.5 grey levels and a float64
relative residual <= 1e-6 per channel (Section 2.2's system; Section 5.2's
relative residual), known pixels bit-exact.

The references come from ``oracle_refs``: worker processes started before the
session touches the GPU compute them while the other tests run (this file is
collected after the other GPU test files for that reason).  Solves run in the
launch configuration the benchmark times: device-resident tensors, the
library's default options unless the form says otherwise.
"""
import numpy as np
import pytest

import oracle
import oracle_refs as refs_mod
from paper_2401_06744_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = 1e-6
GATE = 0.5
PRECS = {"fp32": binding.PREC_FP32, "fp16": binding.PREC_FP16, "bf16": binding.PREC_BF16}


def _check(name, u, f, m, refs, jobs):
    """rel-res, known pixels, maximum principle and max error per channel."""
    k = m != 0
    rr = oracle.rel_res(u.astype(np.float64), f.astype(np.float64), m)
    errs = []
    for ch in range(f.shape[0]):
        assert np.array_equal(u[ch][k], f[ch][k]), f"{name}: known pixels changed in channel {ch}"
        lo, hi = f[ch][k].min(), f[ch][k].max()
        assert u[ch].min() >= lo - 1e-3 and u[ch].max() <= hi + 1e-3, f"{name}: maximum principle"
        ref = refs.get(jobs[ch])
        errs.append(float(np.abs(u[ch].astype(np.float64) - ref).max()))
    print(f"{name}: rel_res {np.array2string(rr, precision=3)} max abs error per channel "
          f"{[f'{e:.3e}' for e in errs]}", flush=True)
    assert np.all(rr <= TOL), (name, rr)
    assert max(errs) <= GATE, (name, errs)
    return errs


@pytest.mark.timeout(1800)
def test_4k_rgb_all_channels_all_precisions(oracle_refs):
    """The headline frame: 3840x2160 RGB, 4 % Bernoulli mask, in every storage
    precision of the correction fields."""
    import torch
    f, m = synth.config_4k()
    fd, md = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
    jobs = [("4k", 0.04, ch) for ch in range(3)]
    for name, prec in PRECS.items():
        out, st, stats = binding.inpaint_solve_ex(fd, md, TOL, opts=binding.make_opts(precision=prec))
        torch.cuda.synchronize()
        assert st == binding.OK and stats["levels"] == 8
        _check(f"4K 4 % {name} ({stats['cycles']} cycles)", out.cpu().numpy(), f, m, oracle_refs, jobs)


@pytest.mark.timeout(1800)
@pytest.mark.parametrize("kind", ["bernoulli", "bluenoise"])
def test_4k_sparse_masks_all_channels_all_precisions(kind, oracle_refs):
    """The precision workload: 4K RGB with a 1 % Bernoulli or blue-noise mask,
    float32, float16 and bfloat16 storage; the error against the oracle is
    stated and gated per variant and channel."""
    import torch
    f, m = synth.config_precision(kind)
    fd, md = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
    jobs = [("prec", kind, ch) for ch in range(3)]
    for name, prec in PRECS.items():
        out, st, stats = binding.inpaint_solve_ex(fd, md, TOL, opts=binding.make_opts(precision=prec))
        torch.cuda.synchronize()
        assert st == binding.OK
        _check(f"4K {kind} 1 % {name} ({stats['cycles']} cycles)", out.cpu().numpy(), f, m,
               oracle_refs, jobs)


@pytest.mark.timeout(1800)
def test_batched_64_uneven_problems(oracle_refs):
    """The 64-problem workload (uneven sizes up to 1920x1080, 1 or 3 channels,
    1-10 % masks) in one batched solve: every problem to 1e-6 with known pixels
    exact; the four largest and every eighth by size against the oracle on
    every channel; a handful bit for bit against their solo solves."""
    import torch
    probs = synth.batched_problems()
    dev = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in probs]
    outs, st, stats = binding.inpaint_solve_batched(dev, TOL)
    torch.cuda.synchronize()
    assert st == binding.OK
    host = [o.cpu().numpy() for o in outs]
    for k, ((f, m), u) in enumerate(zip(probs, host)):
        kn = m != 0
        assert np.array_equal(u[:, kn], f[:, kn]), k
        rr = oracle.rel_res(u.astype(np.float64), f.astype(np.float64), m)
        assert np.all(rr <= TOL), (k, rr)
    sample = refs_mod.batched_sample()
    assert len(sample) >= 10
    for k in sample:
        f, m = probs[k]
        _check(f"batched problem {k} ({f.shape[2]}x{f.shape[1]}x{f.shape[0]})", host[k], f, m,
               oracle_refs, [("batched", k, ch) for ch in range(f.shape[0])])
    order = sorted(range(len(probs)), key=lambda k: probs[k][0].size)
    for k in order[::16]:
        solo, _, _ = binding.inpaint_solve_ex(dev[k][0], dev[k][1], TOL)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), host[k]), k
    print(f"64-problem batch: {stats[0]['gpu_ms']:.2f} ms, cycles "
          f"{sorted(set(s['cycles'] for s in stats))}", flush=True)


@pytest.mark.timeout(1800)
def test_served_4k_and_1080p_requests(oracle_refs):
    """The serving form (float16 storage): a 4K and a 1080p RGB request
    submitted among smaller ones, each against the oracle on every channel and
    bit for bit against its solo solve with the server's options."""
    import torch
    opts = binding.make_opts(precision=binding.PREC_FP16)
    big = {}
    for name, (W, H, C, fs, d, ms) in refs_mod.SERVED.items():
        big[name] = (synth.frame_image(W, H, C, seed=fs), synth.bernoulli_mask(W, H, d, seed=ms))
    small = [(synth.frame_image(W, H, 3, seed=200 + k), synth.bernoulli_mask(W, H, 0.02 + 0.01 * k, seed=210 + k))
             for k, (W, H) in enumerate([(1280, 720), (640, 360), (1280, 720), (320, 180)])]
    srv = binding.inpaint_server_create(opts=opts)
    try:
        dev = {n: (torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for n, (f, m) in big.items()}
        ts = [binding.inpaint_server_submit(srv, *small[0])]
        tb = {"4k": binding.inpaint_server_submit(srv, *dev["4k"])}
        ts += [binding.inpaint_server_submit(srv, *p) for p in small[1:3]]
        tb["1080p"] = binding.inpaint_server_submit(srv, *dev["1080p"])
        ts.append(binding.inpaint_server_submit(srv, *small[3]))
        res = {n: binding.inpaint_server_wait(srv, t) for n, t in tb.items()}
        for t in ts:
            assert binding.inpaint_server_wait(srv, t)[1] == binding.OK
        torch.cuda.synchronize()
    finally:
        binding.inpaint_server_destroy(srv)
    for name, (out, st, stats) in res.items():
        assert st == binding.OK
        f, m = big[name]
        u = out.cpu().numpy()
        W, H, C, fs, d, ms = refs_mod.SERVED[name]
        _check(f"served {name}", u, f, m, oracle_refs, [("frame", W, H, C, fs, d, ms, ch) for ch in range(C)])
        solo, _, _ = binding.inpaint_solve_ex(dev[name][0], dev[name][1], TOL, opts=opts)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), u), name


@pytest.mark.timeout(1800)
@pytest.mark.parametrize("kind", ["pan", "msearch"])
def test_warm_start_4k_sequences(kind, oracle_refs):
    """The warm start at full size: steps 1 and 2 of the panning video (a fresh
    4 % mask each frame) or of the mask search (2 % of the known pixels moved
    per step), each solved in place from the previous step's result (step 0
    solved cold); step 2 against the oracle on every channel, and the warm
    result against the cold solve of the same step (both within the gate)."""
    import torch
    n = refs_mod.WARM_STEP
    if kind == "pan":
        seq = [synth.pan_frame(3840, 2160, t) for t in range(n + 1)]
    else:
        f0, m0 = synth.config_4k()
        seq = [(f0, m) for m in synth.mask_search(m0, n)]
    warm = binding.make_opts(schedule=binding.SCHED_WARM)
    fd, md = torch.from_numpy(seq[0][0]).cuda(), torch.from_numpy(seq[0][1]).cuda()
    buf, st, _ = binding.inpaint_solve_ex(fd, md, TOL)
    assert st == binding.OK
    cycles = []
    for t in range(1, n + 1):
        fd, md = torch.from_numpy(seq[t][0]).cuda(), torch.from_numpy(seq[t][1]).cuda()
        _, st, stats = binding.inpaint_solve_ex(fd, md, TOL, out=buf, opts=warm)
        torch.cuda.synchronize()
        assert st == binding.OK, (t, st)
        cycles.append(stats["cycles"])
    f, m = seq[n]
    jobs = [(kind, n, ch) for ch in range(3)]
    _check(f"warm {kind} step {n} (V-cycles {cycles})", buf.cpu().numpy(), f, m, oracle_refs, jobs)
    cold, st, stats = binding.inpaint_solve_ex(fd, md, TOL)
    torch.cuda.synchronize()
    assert st == binding.OK
    _check(f"cold {kind} step {n} ({stats['cycles']} cycles)", cold.cpu().numpy(), f, m, oracle_refs, jobs)
