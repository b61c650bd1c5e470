"""Benchmark: 4K RGB homogeneous diffusion inpainting on one MI355X.

One step = one full solve of a 3840x2160x3 frame (shared 4 % Bernoulli mask,
seeded synthetic image) to a relative residual of 1e-6 through the C ABI,
with f, mask and out resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                  [--no-forms | --forms precision,solvers,sweeps,batched,serving,warm]
                  [--serve-qps 60,120,240,480] [--serve-requests 2000]

Legs:
  timed      K solves between two device synchronisations -> frames/s, p50/p99
  profiled   K more solves with HIP events around every finest-grid launch ->
             average duration per kernel class, algorithmic bytes and flops per
             launch -> roofline of the dominant kernel
  forms      the same GPU, the same accuracy (rel-res 1e-6 every problem):
             precision  4K RGB with 4 % Bernoulli, 1 % Bernoulli and 1 % blue-noise
                        masks, float32 vs float16 vs bfloat16 correction storage
             batched    64 uneven problems: one at a time (plain float32) vs one
                        autotuned batched solve
             solvers    the 4K frame under reduced full multigrid, full multigrid,
                        multilevel ORAS, plain float32 CG and the multilevel and
                        multigrid CG counterparts, at rel-res 1e-3 and 1e-6
             sweeps     resolution 480x270 ... 4K at 5 % and density 0.5-10 % at 4K,
                        the ORAS solvers vs the CG ones at rel-res 1e-3
             serving    Poisson arrivals of 720p/1080p/4K RGB requests at fixed QPS
                        and a saturating burst: frames/s, p50/p99 latency, vs the
                        same requests solved one at a time
             warm       8-step sequences at 4K (an encoder's mask search, a panning
                        video): the warm start from the previous solution vs
                        the cold reduced full multigrid
  cpu        the CPU oracle (float64 Jacobi-PCG, test infrastructure): its time
             on channel 0 of the 4K frame to rel-res 1e-6 on one core (the
             cpu_baseline), and its reference solutions to rel-res 1e-12 (worker
             processes running beside the GPU legs) against which every form's
             max abs error is reported
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import queue
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X vector FP32, published (packed)
FP32_NONPACKED_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flop x 2.4 GHz (no packed FP32)
CG_FLOPS_PER_PIXEL_ITER = 19   # 5-point apply (9) + 2 dot products (4) + 3 axpys (6)

METRIC = "4K RGB frames/s at max err ≤0.5/255 vs oracle; %HBM roofline; p50/p99 latency"
CSRC = os.path.join(ROOT, "paper_2401_06744_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_4k_rgb.txt")
COPY_BYTES = 1 << 29   # calibration copy: 512 MiB read + 512 MiB written

SERVE_SIZES = [(1280, 720), (1920, 1080), (3840, 2160)]
SERVE_IMAGES, SERVE_MASKS = 2, 8   # per resolution


def kernel_source_sha() -> str:
    """Hash of every source of the library (kernels, launch plans, drivers):
    counter summaries taken before any of them changed no longer apply."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per finest-grid launch of `kernel` from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the factor a plain
    copy of known size gave), or None if the kernels changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    key = f"{kernel}_bytes_per_launch"
    return float(kv[key]) if key in kv else None


def _blocks(n: int, B: int = 32, o: int = 6) -> int:
    """ORAS blocks along an axis of n pixels (stride B - o, the last one clipped)."""
    return max(1, -(-(n - o) // (B - o)))


def algorithmic_bytes(cls: str, W: int, H: int, C: int) -> float:
    """Bytes one finest-grid launch of a kernel class must move (each input read
    once, each output written once; halo and overlap re-reads not counted)."""
    N = float(W * H)
    f4 = 4.0 * C * N
    # level 1's weighted block corrections: its last update of a cycle (and of
    # the cascade) is done by the prolongation to the finest grid
    contrib1 = 4.0 * C * _blocks((W + 1) // 2) * _blocks((H + 1) // 2) * 32 * 32
    return {
        "block_solve": 2 * f4 + N,            # read r, mask; write D_i v_i (once per pixel)
        # read u, corrections, mask; write u and r (16C + 1 B/px: the finest grid
        # holds a solution problem, so b is not read), or, for the update that
        # also restricts (one per V-cycle), write u and the coarse b, u, r instead
        # of r (15C + 1.25 B/px); a launch averages the two
        "update": 0.5 * ((4 * f4 + N) + (3.75 * f4 + 1.25 * N)),
        # read u, mask, coarse e (N/4) and level 1's block corrections; write u, r
        "prolong": 3 * f4 + f4 / 4 + N + contrib1,
        "restrict": f4 + 3 * f4 / 4 + N / 4,  # read r, coarse mask; write coarse b, u, r
        "residual": 2 * f4 + N,               # read u, mask; write r
        "stage": 2 * f4 + 2 * N,              # read f, mask; write b, mask
        "pyramid": N + f4 + 1.25 * N / 4 + f4 / 4,
        "output": 3 * f4 + N,                 # read u, b, mask; write out
        "coarse": 3 * f4 + N,
    }[cls]


def level_sizes(W: int, H: int, coarsest: int = 32):
    """Grid levels: halve with ceil until both sides are at most one block."""
    s = [(W, H)]
    while s[-1][0] > coarsest or s[-1][1] > coarsest:
        w, h = s[-1]
        s.append(((w + 1) // 2, (h + 1) // 2))
    return s


# Bytes per pixel of a level and channel that each pass of the method must move
# at float32 (fused ORAS iteration: read u and b, mask, write u; restriction and
# prolongation about 10; the two pyramids about 7; reading f and writing out 4
# each), the cost model of the method's data movement against which the frame
# is held (halo and overlap re-reads and the blocks' weighted corrections, which
# an ideal fused iteration keeps on chip, are not counted).
MODEL_BPX = {"oras": 13.0, "restrict": 10.0, "prolong": 10.0, "pyramid": 7.0, "io": 4.0}


def frame_model_bytes(W: int, H: int, C: int, cycles: int, schedule: str = "rfmg") -> float:
    """Algorithmic HBM bytes of one frame under the cost model MODEL_BPX for
    the executed schedule: staging and the pyramids, the cascade (reduced full
    multigrid: one ORAS iteration on every coarse level, prolongations to every
    level), `cycles` V-cycles (pre-smoothing and restriction down, the coarsest
    solve, prolongation and post-smoothing up) and the output; the mask (1 B
    per pixel) is read once."""
    lv = level_sizes(W, H)
    N = [w * h for w, h in lv]
    L = len(lv)
    b = MODEL_BPX
    per_ch = b["io"] * N[0] * 2                          # read f, write out
    per_ch += sum(b["pyramid"] * N[l] for l in range(L - 1))
    per_ch += b["oras"] * N[L - 1]                       # cascade: coarsest solve
    for l in range(L - 2, -1, -1):
        per_ch += b["prolong"] * N[l] + (b["oras"] * N[l] if l > 0 else 0.0)
    vcycle = sum((2 * b["oras"] + b["restrict"] + b["prolong"]) * N[l] for l in range(L - 1))
    vcycle += b["oras"] * N[L - 1]
    per_ch += cycles * vcycle
    return C * per_ch + N[0]


# ---------------------------------------------------------------------------
# inputs (seeded; the oracle workers regenerate the same arrays from the seeds)
# ---------------------------------------------------------------------------

def serve_entry(ri: int, j: int, image_cache=None):
    """Request template j of resolution ri: RGB image (SERVE_IMAGES per size),
    Bernoulli mask with density uniform in [0.5 %, 10 %] (seeded)."""
    from paper_2401_06744_amd import synth
    W, H = SERVE_SIZES[ri]
    dens = float(np.random.default_rng(1000 + 10 * ri + j).uniform(0.005, 0.10))
    key = (ri, j % SERVE_IMAGES)
    if image_cache is not None and key in image_cache:
        f = image_cache[key]
    else:
        f = synth.frame_image(W, H, 3, seed=60 + 10 * ri + j % SERVE_IMAGES)
        if image_cache is not None:
            image_cache[key] = f
    return f, synth.bernoulli_mask(W, H, dens, seed=70 + 10 * ri + j), dens


def _inputs(kind, arg):
    from paper_2401_06744_amd import synth
    if kind == "4k":
        return synth.config_4k(density=arg)
    if kind == "prec":
        return synth.config_precision(arg)
    if kind == "4kq":
        return synth.frame_image(3840, 2160, 3, seed=10), synth.bernoulli_mask(3840, 2160, arg, seed=40)
    if kind == "4ke":
        return (synth.frame_image(3840, 2160, 3, seed=10),
                synth.edge_mask(3840, 2160, arg, seed=41, region_seed=10))
    if kind == "small":
        return synth.config_small()
    if kind == "batched":
        return synth.batched_problems()[arg]
    if kind == "serve":
        return serve_entry(*arg)[:2]
    if kind == "warm_enc":
        f, m = synth.config_4k(density=arg[0])
        return f, synth.mask_search(m, arg[1], share=WARM_SHARE)[arg[1]]
    if kind == "warm_vid":
        return synth.pan_frame(3840, 2160, arg)
    raise ValueError(kind)


def oracle_reference(job):
    """CPU leg worker: the oracle's solution of one channel to rel-res 1e-12
    (job = (kind, arg, channel)), with its solve time and iteration count."""
    import oracle
    kind, arg, ch = job
    f, m = _inputs(kind, arg)
    f0 = np.ascontiguousarray(f[ch], dtype=np.float64)
    t = time.perf_counter()
    u, its = oracle.solve_pcg(f0, m, tol=1e-12, return_iters=True)
    return u[0], time.perf_counter() - t, its[0]


def _init_worker():
    # one BLAS/OpenMP thread per oracle process: the pool already uses the cores
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # noqa: BLE001 - only a performance setting
        pass


def host_cpu():
    """Cores this process may use on the host, and the CPU model name."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), model


def oracle_timing(job):
    """CPU leg worker (cpu_baseline): seconds the oracle takes on one channel of
    the benchmark frame to the benchmark's tolerance, and its iteration count
    (input generation is not timed)."""
    import oracle
    from paper_2401_06744_amd import synth
    W, H, density, ch, tol = job
    f, m = synth.config_4k(W, H, density)
    f0 = np.ascontiguousarray(f[ch], dtype=np.float64)
    t = time.perf_counter()
    _, its = oracle.solve_pcg(f0, m, tol=tol, return_iters=True)
    return time.perf_counter() - t, its[0]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms", type=str, default=",".join(FORM_LEGS),
                    help="comma-separated form legs to run (default: all)")
    ap.add_argument("--serve-qps", type=str, default="60,120,240,480")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--width", type=int, default=3840)
    ap.add_argument("--height", type=int, default=2160)
    ap.add_argument("--density", type=float, default=0.04)
    ap.add_argument("--precision", choices=["fp32", "fp16", "bf16"], default="fp32",
                    help="correction storage of the timed and profiled legs (profiling aid; "
                         "the headline value is float32)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 512 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for --gpus {args.gpus}); frames and "
              "requests would shard across GPUs without communication, one process per GPU, "
              "which is not implemented", file=sys.stderr)
        return 2
    full = (args.width, args.height) == (3840, 2160)
    legs = [x for x in args.forms.split(",") if x]
    for x in legs:
        if x not in FORM_LEGS + EXTRA_LEGS:
            print(f"bench.py: unknown form leg {x!r} (known: {', '.join(FORM_LEGS + EXTRA_LEGS)})",
                  file=sys.stderr)
            return 2
    forms = not args.no_forms and full and bool(legs)
    check = not args.no_oracle_check

    # oracle worker processes, started before this process touches the GPU;
    # they stay idle until the GPU legs are over, so that no CPU load perturbs
    # the timings.  A job is one channel of one seeded workload.
    jobs = []
    if check:
        jobs = [("small", None, 0)]
        if full:
            jobs += [("4k", args.density, ch) for ch in range(3)]
        if forms and "precision" in legs:
            jobs += [("prec", k, ch) for k in ("bernoulli", "bluenoise") for ch in range(3)]
        elif forms and "tuning" in legs:
            jobs += [("prec", "bernoulli", ch) for ch in range(3)]
        if forms and "serving" in legs:
            jobs += [("serve", (0, j), ch) for j in (0, 1) for ch in range(3)]
        if forms and "sweeps" in legs:
            jobs += [("4kq", d, 0) for d in QUALITY_DENSITIES] + [("4ke", LEAK_DENSITY, 0)]
        if forms and "warm" in legs:
            jobs += [(k, a, ch) for k, a in (("warm_enc", (args.density, WARM_STEPS)), ("warm_vid", WARM_STEPS))
                     for ch in range(3)]
    host_cores, cpu_model = host_cpu()
    nproc = min(max(len(jobs), 0 if args.no_cpu_baseline else 3), max(3, host_cores - 1))
    pool = mp.get_context("spawn").Pool(nproc, initializer=_init_worker) if nproc else None

    import torch

    from paper_2401_06744_amd import binding, synth

    W, H, C = args.width, args.height, 3
    f, m = synth.config_4k(W, H, args.density)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    fd = torch.from_numpy(f).to(dev)
    md = torch.from_numpy(m).to(dev)
    od = torch.empty_like(fd)
    stream = torch.cuda.current_stream()
    prec = {"fp32": binding.PREC_FP32, "fp16": binding.PREC_FP16, "bf16": binding.PREC_BF16}[args.precision]
    opts = binding.make_opts(precision=prec)

    def step(o, out=od):
        return binding.inpaint_solve_ex(fd, md, args.tol, out=out, opts=o, stream=stream)

    for _ in range(args.warmup):
        step(opts)
    torch.cuda.synchronize()
    log("warm-up done")

    # ---- timed leg
    lat = []
    statuses = []
    cycles = []
    cg_mean = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, st, stats = step(opts)
        lat.append(time.perf_counter() - ts)
        statuses.append(st)
        cycles.append(stats["cycles"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    fps = args.steps / elapsed
    lat_ms = np.array(lat) * 1e3
    out_last = od.clone()

    # ---- profiled leg: per-kernel HIP events on the solve's stream
    popts = binding.make_opts(profile=1, precision=prec)
    kms = np.zeros(len(binding.KERNELS))
    kcalls = np.zeros(len(binding.KERNELS))
    cg_fin = 0.0
    cg_px = 0.0
    fin_solves = 0
    for _ in range(args.steps):
        _, st, stats = step(popts)
        kms += np.array(stats["kernel_ms"])
        kcalls += np.array(stats["kernel_calls"])
        cg_mean.append(stats["local_cg_mean"])
        cg_fin += stats["local_cg_finest"]
        cg_px += stats["finest_cg_pixel_iters"]
        fin_solves += stats["finest_block_solves"]
    torch.cuda.synchronize()
    kernels = {}
    for i, name in enumerate(binding.KERNELS):
        if kcalls[i] == 0:
            continue
        avg_ms = kms[i] / kcalls[i]
        by = algorithmic_bytes(name, W, H, C)
        kernels[name] = {
            "calls_per_frame": kcalls[i] / args.steps,
            "avg_ms": round(avg_ms, 5),
            "share_of_frame": round(kms[i] / args.steps / (1e3 / fps), 4),
            "alg_bytes_per_launch": by,
            "alg_GBps": round(by / (avg_ms * 1e-3) / 1e9, 1),
            "traffic": measured_traffic(name),
        }
    # block solve: algorithmic flops per launch from the measured local iterations
    bs_i = binding.KERNELS.index("block_solve")
    bs_calls = kcalls[bs_i]
    blocks_per_launch = fin_solves / bs_calls if bs_calls else 0
    iters_per_block = cg_fin / fin_solves if fin_solves else 0.0
    bs_flops = CG_FLOPS_PER_PIXEL_ITER * cg_px / bs_calls if bs_calls else 0.0
    dominant = None
    if bs_calls:
        bk = kernels["block_solve"]
        avg = bk["avg_ms"] * 1e-3
        tf = bs_flops / avg / 1e12
        bk["alg_flops_per_launch"] = bs_flops
        bk["alg_TFLOPs"] = round(tf, 3)
        bk["local_iters_per_block"] = round(iters_per_block, 3)
        bk["blocks_per_launch"] = blocks_per_launch
        bk["pixel_iters_per_launch"] = cg_px / bs_calls
        dominant = {"kernel": "block_solve", "bound": "alu", "achieved": round(tf, 3),
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4),
                    "peak_nonpacked_fp32": FP32_NONPACKED_TFLOPS,
                    "frac_nonpacked": round(tf / FP32_NONPACKED_TFLOPS, 4),
                    "avg_us": round(avg * 1e6, 2), "hbm_GBps": bk["alg_GBps"],
                    "hbm_frac": round(bk["alg_GBps"] / HBM_PEAK_GBS, 4), "traffic": bk["traffic"],
                    "flops_per_pixel_iter": CG_FLOPS_PER_PIXEL_ITER}
    # the whole frame against HBM: the cost model's bytes for the executed
    # schedule (every level) over the measured frame time
    k_cyc = int(np.median(cycles))
    frame_bytes = frame_model_bytes(W, H, C, k_cyc)
    frame_gbs = frame_bytes * fps / 1e9
    roof = {"bound": "hbm", "achieved": round(frame_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(frame_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic("frame"),
            "kernel": "whole frame (every launch of one solve, all levels)",
            "alg_bytes_per_frame": frame_bytes, "cycles": k_cyc, "model_bytes_per_px": MODEL_BPX,
            "hbm_floor_ms": round(frame_bytes / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
            "dominant_kernel": dominant}
    log(f"timed and profiled legs done: {fps:.1f} frames/s")

    # achievable bandwidth of a plain device copy (secondary denominator), and
    # the calibration launch for the counter runs
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3 if args.calibrate_copy else 1):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    roof["copy_GBps"] = round(2 * COPY_BYTES * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    roof["frac_of_copy"] = round(frame_gbs / roof["copy_GBps"], 4)
    del src, dst

    # ---- accuracy of the last timed output (device rel-res; oracle error below)
    rr = binding.inpaint_rel_res(out_last, fd, md)
    out_host = out_last.cpu().numpy()
    acc = {"rel_res_max": float(rr.max()), "status": int(max(statuses)),
           "known_exact": bool(np.array_equal(out_host[:, m != 0], f[:, m != 0]))}

    # ---- config 1: the 256x256 grey frame (5 % mask), single solves
    fs, ms_ = synth.config_small()
    fsd, msd = torch.from_numpy(fs).to(dev), torch.from_numpy(ms_).to(dev)
    osd = torch.empty_like(fsd)
    sec_small = _timed(torch, lambda: binding.inpaint_solve_ex(fsd, msd, args.tol, out=osd, stream=stream), 100)
    _, st_s, stats_s = binding.inpaint_solve_ex(fsd, msd, args.tol, out=osd, stream=stream)
    small = {"workload": "256x256 grey (seed 1), Bernoulli 5 % (seed 2), FMG+ORAS to rel-res "
                         f"{args.tol:g}, float32, inputs resident in HBM, one solve at a time",
             "fps": round(1.0 / sec_small, 1), "ms": round(1e3 * sec_small, 4), "status": st_s,
             "cycles": stats_s["cycles"],
             "rel_res_max": float(binding.inpaint_rel_res(osd, fsd, msd).max())}
    pending = {}   # name -> (job, output channel) compared with the oracle below
    pending["config1"] = (("small", None, 0), osd[0].cpu().numpy())

    # ---- forms
    form_res = None
    if forms:
        form_res = {}
        if "precision" in legs:
            form_res["precision"] = precision_leg(binding, torch, synth, args, fd, md, pending)
            log("precision forms done")
        if "solvers" in legs:
            form_res["solvers"] = solvers_leg(binding, torch, args, fd, md, pending)
            log("solver comparison done")
        if "sweeps" in legs:
            form_res["sweeps"] = sweep_leg(binding, torch, synth, args, fd, pending)
            log("resolution and density sweeps done")
        if "tuning" in legs:
            form_res["tuning"] = tuning_leg(binding, torch, synth, args, fd, md, pending)
            log("tuning sweep done")
        if "batched" in legs:
            form_res["batched"] = batched_leg(binding, torch, synth, args)
            log("batched form done")
        if "serving" in legs:
            form_res["serving"] = serving_leg(binding, torch, args, pending)
            log("serving form done")
        if "warm" in legs:
            form_res["warm"] = warm_leg(binding, torch, synth, args, pending)
            log("warm start form done")
    if check and full:
        for ch in range(C):
            pending[f"headline/{ch}"] = (("4k", args.density, ch), out_host[ch])

    # ---- CPU leg: oracle reference solutions (all jobs at once, GPU idle), the
    # max error of every result against them, and the oracle's own time
    cpu = None
    refs = {job: pool.apply_async(oracle_reference, (job,)) for job in jobs} if pool else {}
    if refs:
        log(f"oracle references: {len(refs)} channel solves to rel-res 1e-12 in {nproc} worker processes")
    ref_time = {}
    if check:
        got = {}
        for job, r in refs.items():
            got[job] = r.get()
            ref_time[job] = got[job][1:]
        for name, (job, u0) in pending.items():
            dev_ = u0.astype(np.float64) - got[job][0]
            err = float(np.abs(dev_).max())
            if name.startswith("headline/"):
                acc.setdefault("max_err_vs_oracle", [None] * C)[int(name.split("/")[1])] = err
                continue
            if name == "config1":
                small["max_err_vs_oracle"] = err
                small["gate_0.5_pass"] = err <= 0.5
                continue
            section, key = name.split("/", 1)
            node = form_res[section]
            parts = key.split("/")
            for part in parts[:-1]:
                node = node.setdefault(part, {})
            leaf = parts[-1]
            if leaf.startswith("ch"):  # per-channel errors of a form's result
                node.setdefault("max_err_vs_oracle", {})[leaf] = err
                node["gate_0.5_pass"] = all(v <= 0.5 for v in node["max_err_vs_oracle"].values())
            else:
                node = node[leaf]
                node["max_err_vs_oracle_ch0"] = err
                if job[0] in ("4kq", "4ke"):
                    node["mse_vs_oracle_ch0"] = float(np.mean(dev_ * dev_))
        if "max_err_vs_oracle" in acc:
            acc["gate_0.5_pass"] = max(acc["max_err_vs_oracle"]) <= 0.5
    if refs:
        log("oracle references done")
    if not args.no_cpu_baseline:
        # the oracle as it stands, one process per channel of the same frame
        log("timing the oracle (cpu_baseline)")
        tc = time.perf_counter()
        runs = pool.map(oracle_timing, [(W, H, args.density, ch, args.tol) for ch in range(C)])
        wall = time.perf_counter() - tc
        span = max(t for t, _ in runs)
        cpu = {"value": round(1.0 / span, 5), "unit": "frames/s", "cores": C, "kind": "oracle",
               "host_cores": host_cores, "cpu_model": cpu_model,
               "sample": f"the whole {W}x{H}x{C} frame of the benchmark, float64 Jacobi-PCG to "
                         f"rel-res {args.tol:g}, one process per channel ({C} processes, one thread "
                         f"each, on a host with {host_cores} usable cores: {cpu_model}); "
                         f"per-channel solve times {[round(t, 2) for t, _ in runs]} s, iterations "
                         f"{[int(i) for _, i in runs]}; value = 1 / the slowest channel "
                         f"(wall {wall:.1f} s including input generation)"}
        hl = [ref_time[("4k", args.density, ch)] for ch in range(C) if ("4k", args.density, ch) in ref_time]
        if hl:
            cpu["oracle_tol_1e-12"] = {"frames_per_s": round(1.0 / max(t for t, _ in hl), 5),
                                       "channel_s": [round(t, 2) for t, _ in hl],
                                       "iterations": [int(i) for _, i in hl],
                                       "note": "the reference solutions, timed in the worker pool "
                                               "beside the other references"}
    if pool is not None:
        pool.close()
        pool.join()

    res = {
        "metric": METRIC,
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f32+f16", "bf16": "f32+bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{W}x{H} RGB frame, shared Bernoulli {args.density:.0%} mask, "
                               f"FMG+ORAS to rel-res {args.tol:g}",
                   "W": W, "H": H, "channels": C, "density": args.density, "tol": args.tol,
                   "block": 32, "overlap": 6, "schedule": "reduced FMG",
                   "correction_storage": args.precision},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "cycles": k_cyc,
        "local_cg_mean": round(float(np.mean(cg_mean)), 3),
        "roofline": roof,
        "kernels": kernels,
        "accuracy": acc,
        "config1": small,
        "forms": form_res,
        "cpu_baseline": cpu,
        "paper_context": "14.3 ms (70 fps) per 4K RGB frame at rel-res 1e-3 on a GTX 1080 Ti",
    }
    print(json.dumps(res), flush=True)
    return 0


def log(msg: str) -> None:
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def precision_leg(binding, torch, synth, args, fd4, md4, pending):
    """4K RGB to rel-res 1e-6 with each storage precision of the correction
    fields, on the headline 4 % mask and on the two 1 % masks."""
    names = {binding.PREC_FP32: "fp32", binding.PREC_FP16: "fp16", binding.PREC_BF16: "bf16"}
    out = {"workload": "3840x2160 RGB frame (seed 10) with a 4 % Bernoulli, a 1 % Bernoulli "
                       "(seed 30) and a 1 % blue-noise (seed 31) mask, rel-res 1e-6; max error "
                       "on every channel against the oracle, gated at 0.5 grey levels"}
    cases = [("bernoulli_4pct", None), ("bernoulli_1pct", "bernoulli"), ("bluenoise_1pct", "bluenoise")]
    for name, kind in cases:
        if kind is None:
            fd, md = fd4, md4
            job = ("4k", args.density)
        else:
            f, m = synth.config_precision(kind)
            fd, md = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
            job = ("prec", kind)
        nch = fd.shape[0]
        od = torch.empty_like(fd)
        row = {"density": round(float(md.float().mean().item()), 5)}
        for prec, pn in names.items():
            o = binding.make_opts(precision=prec)
            sec = _timed(torch, lambda: binding.inpaint_solve_ex(fd, md, args.tol, out=od, opts=o),
                         max(5, args.steps // 2))
            _, st, stats = binding.inpaint_solve_ex(fd, md, args.tol, out=od, opts=o)
            rr = binding.inpaint_rel_res(od, fd, md)
            row[pn] = {"fps": round(1.0 / sec, 2), "ms": round(1e3 * sec, 3), "status": st,
                       "cycles": stats["cycles"], "rel_res_max": float(rr.max())}
            host = od.cpu().numpy()
            for ch in range(nch):
                pending[f"precision/{name}/{pn}/ch{ch}"] = ((*job, ch), host[ch])
        row["speedup_fp16"] = round(row["fp16"]["fps"] / row["fp32"]["fps"], 3)
        row["speedup_bf16"] = round(row["bf16"]["fps"] / row["fp32"]["fps"], 3)
        out[name] = row
    return out


def solvers_leg(binding, torch, args, fd, md, pending):
    """The headline frame under each schedule: reduced full multigrid (the
    method), full multigrid, multilevel ORAS (coarse-to-fine start, no
    V-cycles), plain float32 CG on the finest grid and the multilevel and
    multigrid CG counterparts (CG in place of ORAS), at rel-res 1e-3 (the
    stopping rule of the paper's runtime comparison) and at the headline 1e-6
    for the method, CG and multigrid CG (CG's status and rel-res are reported
    as they come: in float32 it can stall near 1e-6)."""
    scheds = [("rfmg", binding.SCHED_RFMG), ("fmg", binding.SCHED_FMG),
              ("multilevel", binding.SCHED_MULTILEVEL), ("cg", binding.SCHED_CG),
              ("cg_multilevel", binding.SCHED_CG_MULTILEVEL),
              ("cg_multigrid", binding.SCHED_CG_MULTIGRID)]
    out = {"workload": "3840x2160 RGB frame (seed 10), 4 % Bernoulli mask; max error on "
                       "channel 0 against the oracle"}
    od = torch.empty_like(fd)
    for tol, names in ((1e-3, [n for n, _ in scheds]), (args.tol, ["rfmg", "cg", "cg_multigrid"])):
        row = {}
        for name, sc in scheds:
            if name not in names:
                continue
            o = binding.make_opts(schedule=sc)
            reps = 3 if name.startswith("cg") else max(5, args.steps // 2)
            sec = _timed(torch, lambda: binding.inpaint_solve_ex(fd, md, tol, out=od, opts=o), reps)
            _, st, stats = binding.inpaint_solve_ex(fd, md, tol, out=od, opts=o)
            rr = binding.inpaint_rel_res(od, fd, md)
            row[name] = {"fps": round(1.0 / sec, 2), "ms": round(1e3 * sec, 3), "status": st,
                         "cycles": stats["cycles"], "rel_res_max": float(rr.max())}
            if name.startswith("cg"):
                row[name]["cg_iterations"] = stats["oras_iters"] // fd.shape[0]
            pending[f"solvers/tol_{tol:g}/{name}"] = (("4k", args.density, 0), od[0].cpu().numpy())
        # the paper's pairs: each ORAS solver against its CG counterpart
        row["rfmg_over_cg"] = round(row["rfmg"]["fps"] / row["cg"]["fps"], 2)
        row["rfmg_over_cg_multigrid"] = round(row["rfmg"]["fps"] / row["cg_multigrid"]["fps"], 2)
        if "multilevel" in row:
            row["multilevel_over_cg_multilevel"] = round(
                row["multilevel"]["fps"] / row["cg_multilevel"]["fps"], 2)
        out[f"tol_{tol:g}"] = row
    return out


def tuning_leg(binding, torch, synth, args, fd4, md4, pending):
    """The block solve's work trade (Section 3.1 block and overlap, the local
    stop): overlap {4, 6} x tau {0.002, 0.005, 0.01} x local cap {8, 16} on the
    headline 4 % frame and the 1 % Bernoulli frame at rel-res 1e-6: frames/s,
    V-cycles, finest-grid local CG pixel-iterations per frame, max error of
    every channel against the oracle."""
    out = {"workload": "3840x2160 RGB, 4 % and 1 % Bernoulli masks, rel-res 1e-6, float32, "
                       "block 32, gamma 0.5; each setting timed over 8 solves"}
    f1, m1 = synth.config_precision("bernoulli")
    frames = [("bernoulli_4pct", fd4, md4, ("4k", args.density)),
              ("bernoulli_1pct", torch.from_numpy(f1).cuda(), torch.from_numpy(m1).cuda(),
               ("prec", "bernoulli"))]
    for name, fd, md, job in frames:
        od = torch.empty_like(fd)
        row = {}
        for o in (4, 6):
            for tau in (0.002, 0.005, 0.01):
                for cap in (8, 16):
                    opts = binding.make_opts(overlap=o, tau=tau, max_local_iters=cap)
                    sec = _timed(torch, lambda: binding.inpaint_solve_ex(fd, md, args.tol, out=od,
                                                                         opts=opts), 8)
                    _, st, stats = binding.inpaint_solve_ex(
                        fd, md, args.tol, out=od,
                        opts=binding.make_opts(overlap=o, tau=tau, max_local_iters=cap, profile=1))
                    key = f"o{o}_tau{tau:g}_cap{cap}"
                    row[key] = {"fps": round(1.0 / sec, 2), "ms": round(1e3 * sec, 3), "status": st,
                                "cycles": stats["cycles"],
                                "finest_pixel_iters": stats["finest_cg_pixel_iters"]}
                    host = od.cpu().numpy()
                    for ch in range(host.shape[0]):
                        pending[f"tuning/{name}/{key}/ch{ch}"] = ((*job, ch), host[ch])
        out[name] = row
    return out


QUALITY_DENSITIES = (0.005, 0.01, 0.02, 0.05, 0.10)
LEAK_DENSITY = 0.02
FORM_LEGS = ("precision", "solvers", "sweeps", "batched", "serving", "warm")
WARM_STEPS = 8       # solves per warm-start sequence
WARM_SHARE = 0.02    # share of the known pixels moved per mask-search step
EXTRA_LEGS = ("tuning",)   # run only when --forms names them


def sweep_leg(binding, torch, synth, args, fd4, pending):
    """The paper's two runtime sweeps on synthetic stand-ins, at its stopping
    rule (rel-res 1e-3) and at 1e-6: RGB frames of 480x270 to 3840x2160 with a
    5 % Bernoulli mask (resolution scaling), and the 4K frame with 0.5-10 %
    Bernoulli masks (density scaling), under the method, multilevel ORAS,
    float32 CG and the multilevel and multigrid CG counterparts.  On the
    density sweep every result's channel 0 is also compared with the oracle's
    converged solution (mean squared and max error: the approximation quality
    that rel-res 1e-3 buys), and the method runs with the naive known-value
    restriction beside the modified one (cycles and time saved by the
    modification)."""
    out = {"workload": "RGB frames (seed 10) 480x270 ... 3840x2160 with a 5 % Bernoulli mask "
                       "(seed 20), and the 4K frame with 0.5/1/2/5/10 % Bernoulli masks (seed 40); "
                       "rel-res 1e-3 unless named; errors on channel 0 against the oracle at 1e-12"}

    def run(fd, md, tol, sc, job=None, name=None, **kw):
        o = binding.make_opts(schedule=sc, **kw)
        od = torch.empty_like(fd)
        reps = 2 if sc in (binding.SCHED_CG, binding.SCHED_CG_MULTILEVEL) else 4
        sec = _timed(torch, lambda: binding.inpaint_solve_ex(fd, md, tol, out=od, opts=o), reps)
        _, st, stats = binding.inpaint_solve_ex(fd, md, tol, out=od, opts=o)
        if job is not None:
            pending[name] = (job, od[0].cpu().numpy())
        res = {"ms": round(1e3 * sec, 3), "fps": round(1.0 / sec, 1), "status": st,
               "cycles": stats["cycles"]}
        if tol >= 0.5:
            res["rel_res_max"] = float(binding.inpaint_rel_res(od, fd, md).max())
        return res

    res = {}
    for W, H in ((480, 270), (960, 540), (1920, 1080), (3840, 2160)):
        fd = fd4 if tuple(fd4.shape[1:]) == (H, W) else torch.from_numpy(synth.frame_image(W, H, 3, seed=10)).cuda()
        md = torch.from_numpy(synth.bernoulli_mask(W, H, 0.05, seed=20)).cuda()
        res[f"{W}x{H}"] = {"rfmg": run(fd, md, 1e-3, binding.SCHED_RFMG),
                           "rfmg_1e-6": run(fd, md, args.tol, binding.SCHED_RFMG),
                           "multilevel": run(fd, md, 1e-3, binding.SCHED_MULTILEVEL),
                           "cg": run(fd, md, 1e-3, binding.SCHED_CG),
                           "cg_multilevel": run(fd, md, 1e-3, binding.SCHED_CG_MULTILEVEL),
                           "cg_multigrid": run(fd, md, 1e-3, binding.SCHED_CG_MULTIGRID)}
    out["resolution_5pct"] = res
    res = {}
    quality = tuple(fd4.shape[1:]) == (2160, 3840) and not args.no_oracle_check
    for d in QUALITY_DENSITIES:
        md = torch.from_numpy(synth.bernoulli_mask(fd4.shape[2], fd4.shape[1], d, seed=40)).cuda()
        key = f"{d:g}"
        job = ("4kq", d, 0) if quality else None
        runs = [("rfmg", 1e-3, binding.SCHED_RFMG, {}), ("rfmg_1e-6", args.tol, binding.SCHED_RFMG, {}),
                ("rfmg_naive", 1e-3, binding.SCHED_RFMG, {"rhs_restriction": binding.RHS_NAIVE}),
                ("rfmg_naive_1e-6", args.tol, binding.SCHED_RFMG, {"rhs_restriction": binding.RHS_NAIVE}),
                # the cascade alone (a tolerance of 0.99 stops at its first test)
                ("cascade", 0.99, binding.SCHED_RFMG, {}),
                ("cascade_naive", 0.99, binding.SCHED_RFMG, {"rhs_restriction": binding.RHS_NAIVE}),
                ("multilevel", 1e-3, binding.SCHED_MULTILEVEL, {}), ("cg", 1e-3, binding.SCHED_CG, {}),
                ("cg_multilevel", 1e-3, binding.SCHED_CG_MULTILEVEL, {}),
                ("cg_multigrid", 1e-3, binding.SCHED_CG_MULTIGRID, {})]
        res[key] = {}
        for name, tol, sc, kw in runs:
            res[key][name] = run(fd4, md, tol, sc, job, f"sweeps/density_4k/{key}/{name}", **kw)
    out["density_4k"] = res
    # Section 4.3's leakage case: a 2 % mask concentrated on the region borders
    # of the frame (as masks optimised for such images are), where many coarse
    # cells hold several known children on both sides of an edge; the cascade
    # alone (the one-way coarse-to-fine start) and the method, with the naive
    # and the modified known-value restriction
    me = torch.from_numpy(synth.edge_mask(fd4.shape[2], fd4.shape[1], LEAK_DENSITY, seed=41,
                                          region_seed=10)).cuda()
    job = ("4ke", LEAK_DENSITY, 0) if quality else None
    leak = {"density": round(float(me.float().mean().item()), 5)}
    for name, tol, kw in (("cascade", 0.99, {}), ("cascade_naive", 0.99, {"rhs_restriction": binding.RHS_NAIVE}),
                          ("rfmg", 1e-3, {}), ("rfmg_naive", 1e-3, {"rhs_restriction": binding.RHS_NAIVE}),
                          ("rfmg_1e-6", args.tol, {}),
                          ("rfmg_naive_1e-6", args.tol, {"rhs_restriction": binding.RHS_NAIVE})):
        leak[name] = run(fd4, me, tol, binding.SCHED_RFMG, job, f"sweeps/leakage_edge_2pct/{name}", **kw)
    out["leakage_edge_2pct"] = leak
    out["workload"] += ("; leakage case: the 4K frame with a 2 % mask, 80 % of its known pixels on the "
                        "region borders (seed 41)")
    return out


def batched_leg(binding, torch, synth, args):
    """64 uneven problems: solved one at a time with the plain float32 solver,
    and in one batched solve with autotuned options."""
    probs = synth.batched_problems()
    dev = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in probs]
    outs = [torch.empty_like(f) for f, _ in dev]
    items = [(f, m, o) for (f, m), o in zip(dev, outs)]
    px = sum(f.numel() for f, _ in dev)
    reps = 5

    def plain():
        for f, m, o in items:
            binding.inpaint_solve_ex(f, m, args.tol, out=o)

    t_plain = _timed(torch, plain, reps)
    t0 = time.perf_counter()
    tuned, tuned_ms = binding.inpaint_autotune(items, args.tol)
    t_tune = time.perf_counter() - t0
    default = binding.make_opts()
    t_default = _timed(torch, lambda: binding.inpaint_solve_batched(items, args.tol, opts=default), reps)
    t_tuned = _timed(torch, lambda: binding.inpaint_solve_batched(items, args.tol, opts=tuned), reps)
    _, st, stats = binding.inpaint_solve_batched(items, args.tol, opts=tuned)
    torch.cuda.synchronize()
    rr = max(float(binding.inpaint_rel_res(o, f, m).max()) for f, m, o in items)
    known = all(bool(torch.equal(o[:, m != 0], f[:, m != 0])) for f, m, o in items)
    n = len(items)
    sizes = [f.numel() for f, _, _ in items]
    # V-cycles per pixel-channel: the 1-10 % masks of the mix need more
    # cycles than the headline frame's 4 % mask (a third for the sparser ones)
    px_cycles = sum(z * s["cycles"] for z, s in zip(sizes, stats)) / px
    # the same 64 shapes, channels and images with every mask at the headline
    # frame's density: the batch's pixel rate at the headline's cycle count
    same = synth.batched_problems(density=args.density)
    dev_s = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in same]
    items_s = [(f, m, o) for (f, m), o in zip(dev_s, outs)]
    t_same = _timed(torch, lambda: binding.inpaint_solve_batched(items_s, args.tol, opts=default), reps)
    _, st_s, stats_s = binding.inpaint_solve_batched(items_s, args.tol, opts=default)
    torch.cuda.synchronize()
    rr_s = max(float(binding.inpaint_rel_res(o, f, m).max()) for f, m, o in items_s)
    del dev_s, items_s
    return {
        "workload": f"{n} problems (seed 40): W uniform 128..1920, H 128..1080, 1 or 3 channels, "
                    f"Bernoulli 1-10 %, rel-res {args.tol:g}, float32",
        "problems": n, "pixel_channels": px, "equiv_4k_rgb_frames": round(px / (3840 * 2160 * 3), 3),
        "plain": {"ms": round(1e3 * t_plain, 3), "problems_per_s": round(n / t_plain, 2)},
        "batched_default": {"ms": round(1e3 * t_default, 3), "problems_per_s": round(n / t_default, 2)},
        "batched_autotuned": {"ms": round(1e3 * t_tuned, 3), "problems_per_s": round(n / t_tuned, 2),
                              "opts": {"block": tuned.block, "overlap": tuned.overlap,
                                       "gamma": round(tuned.gamma, 3), "tau": round(tuned.tau, 4),
                                       "schedule": tuned.schedule},
                              "autotune_s": round(t_tune, 2)},
        "speedup_vs_plain": round(t_plain / t_tuned, 3),
        # the batch's pixel rate in 4K RGB frames per second, to set beside
        # the single-frame headline (the same pixels, channel count and tol)
        "equiv_4k_rgb_fps": {"plain": round(px / (3840 * 2160 * 3) / t_plain, 1),
                             "batched_default": round(px / (3840 * 2160 * 3) / t_default, 1),
                             "batched_autotuned": round(px / (3840 * 2160 * 3) / t_tuned, 1)},
        "status": st, "rel_res_max": rr, "known_exact": known,
        "cycles": sorted({s["cycles"] for s in stats}),
        "cycles_per_pixel": round(px_cycles, 3),
        f"same_shapes_{args.density:.0%}_masks": {
            "ms": round(1e3 * t_same, 3), "opts": "default",
            "equiv_4k_rgb_fps": round(px / (3840 * 2160 * 3) / t_same, 1),
            "cycles_per_pixel": round(sum(z * s["cycles"] for z, s in zip(sizes, stats_s)) / px, 3),
            "status": st_s, "rel_res_max": rr_s},
        "batched_equals_solo": "bitwise (tests/test_gpu_batched.py)",
    }


def warm_leg(binding, torch, synth, args, pending):
    """Warm start (schedule WARM: V-cycles from the previous solution) against
    the cold reduced FMG, on two 4K RGB sequences at the benchmark tolerance:
    an encoder's mask search (each step moves 2 % of the known pixels of the
    4 % mask) and a panning video (one pixel per frame, a fresh 4 % mask per
    frame).  Each sequence is timed as WARM_STEPS solves in a row, every warm
    solve reading its guess from the buffer the previous one wrote."""
    warm = binding.make_opts(schedule=binding.SCHED_WARM)
    out = {"workload": f"3840x2160 RGB, rel-res {args.tol:g}, float32; mask search: the 4 % frame "
                       f"(seeds 10, 20), {WARM_STEPS} steps each moving {WARM_SHARE:.0%} of the known "
                       f"pixels (seeds 42...); video: the frame panned one pixel per frame, a fresh 4 % "
                       f"mask per frame (seeds 60...); max error of the last solve against the oracle"}
    f, m = synth.config_4k(density=args.density)
    masks = synth.mask_search(m, WARM_STEPS, share=WARM_SHARE)
    fd = torch.from_numpy(f).cuda()
    seqs = {"mask_search": ([fd] * (WARM_STEPS + 1), [torch.from_numpy(x).cuda() for x in masks],
                            ("warm_enc", (args.density, WARM_STEPS)))}
    # synth.pan_frame(3840, 2160, t), with the roll done on the device
    v0, _ = synth.pan_frame(3840, 2160, 0)
    v0 = torch.from_numpy(v0).cuda()
    seqs["video"] = ([torch.roll(v0, t, dims=2).contiguous() for t in range(WARM_STEPS + 1)],
                     [torch.from_numpy(synth.pan_frame_mask(3840, 2160, t)).cuda() for t in range(WARM_STEPS + 1)],
                     ("warm_vid", WARM_STEPS))
    for name, (fs, ms, job) in seqs.items():
        buf = torch.empty_like(fd)
        cold_out = torch.empty_like(fd)
        res = {}
        for mode in ("cold", "warm"):
            for rep in range(2):  # the first pass builds workspaces and plans
                # the guess for step 1: the solution of step 0
                binding.inpaint_solve_ex(fs[0], ms[0], args.tol, out=buf)
                torch.cuda.synchronize()
                cycles = []
                t = time.perf_counter()
                for k in range(1, WARM_STEPS + 1):
                    if mode == "warm":
                        _, _, st = binding.inpaint_solve_ex(fs[k], ms[k], args.tol, out=buf, opts=warm)
                    else:
                        _, _, st = binding.inpaint_solve_ex(fs[k], ms[k], args.tol, out=cold_out)
                    cycles.append(st["cycles"])
                torch.cuda.synchronize()
                sec = (time.perf_counter() - t) / WARM_STEPS
            last = (buf if mode == "warm" else cold_out).cpu().numpy()
            res[mode] = {"ms": round(1e3 * sec, 3), "fps": round(1.0 / sec, 1), "cycles": cycles,
                         "rel_res_max": float(binding.inpaint_rel_res(last, fs[-1].cpu().numpy(),
                                                                      ms[-1].cpu().numpy()).max())}
            for ch in range(last.shape[0]):
                pending[f"warm/{name}/{mode}/ch{ch}"] = ((*job, ch), last[ch])
        res["speedup"] = round(res["cold"]["ms"] / res["warm"]["ms"], 3)
        out[name] = res
    return out


def serving_leg(binding, torch, args, pending):
    """Poisson arrivals (seed 50) of RGB requests, resolution uniform over 720p,
    1080p and 4K, mask density uniform in 0.5-10 %, float16 correction storage,
    device-resident inputs; plus a burst that saturates the server."""
    from paper_2401_06744_amd import synth
    images = {}
    tmpl = {}
    for ri in range(len(SERVE_SIZES)):
        for j in range(SERVE_MASKS):
            f, m, d = serve_entry(ri, j, images)
            tmpl[(ri, j)] = (torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), d)
    dens = {ri: np.array([tmpl[(ri, j)][2] for j in range(SERVE_MASKS)]) for ri in range(3)}
    opts = binding.make_opts(precision=binding.PREC_FP16)

    def requests(qps, n, seed=50):
        reqs = []
        for t, W, H, d in synth.poisson_trace(qps, n, seed=seed):
            ri = SERVE_SIZES.index((W, H))
            j = int(np.argmin(np.abs(dens[ri] - d)))
            reqs.append((t, ri, j))
        return reqs

    def run(srv, reqs, burst=False):
        tq = queue.Queue()

        def submitter():
            start = time.perf_counter()
            for k, (t, ri, j) in enumerate(reqs):
                if not burst:
                    dt = t - (time.perf_counter() - start)
                    if dt > 0:
                        time.sleep(dt)
                f, m, _ = tmpl[(ri, j)]
                tq.put((k, ri, j, binding.inpaint_server_submit(srv, f, m, tol=args.tol)))
            tq.put(None)

        th = threading.Thread(target=submitter)
        th.start()
        rows = []
        keep = {}
        while True:
            item = tq.get()
            if item is None:
                break
            k, ri, j, ticket = item
            out, st, s = binding.inpaint_server_wait(srv, ticket, raise_on_error=False)
            rows.append((s["t_submit_ms"], s["t_start_ms"], s["t_done_ms"], st, s["rel_res"], ri))
            if ri == 0 and j in (0, 1) and j not in keep:
                keep[j] = out.cpu().numpy()
        th.join()
        a = np.array(rows)
        lat = a[:, 2] - a[:, 0]
        span = (a[:, 2].max() - a[:, 0].min()) / 1e3
        return {"requests": len(rows), "fps": round(len(rows) / span, 2),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "queue_p50_ms": round(float(np.percentile(a[:, 1] - a[:, 0], 50)), 3),
                "all_ok": bool(np.all(a[:, 3] == binding.OK)),
                "rel_res_max": float(a[:, 4].max())}, keep

    srv = binding.inpaint_server_create(max_batch=64, opts=opts)
    try:
        run(srv, requests(1000.0, 3 * SERVE_MASKS, seed=49), burst=True)  # warm-up: every template
        points = {}
        keep = {}
        for q in [float(x) for x in args.serve_qps.split(",") if x]:
            # each point: --serve-requests arrivals, at most 8 s of them
            r, kp = run(srv, requests(q, max(50, min(args.serve_requests, int(8 * q)))))
            points[f"{q:g}"] = r
            keep.update({j: v for j, v in kp.items() if j not in keep})
        burst_reqs = requests(1000.0, min(args.serve_requests, 600), seed=51)
        points["burst"], _ = run(srv, burst_reqs, burst=True)
    finally:
        binding.inpaint_server_destroy(srv)
    # the same requests, one at a time, plain float32 solver
    plain_reqs = burst_reqs[:150]
    outs = {ri: torch.empty_like(tmpl[(ri, 0)][0]) for ri in range(3)}

    def plain():
        for _, ri, j in plain_reqs:
            f, m, _ = tmpl[(ri, j)]
            binding.inpaint_solve_ex(f, m, args.tol, out=outs[ri])

    t_plain = _timed(torch, plain, 1)
    for j, u in keep.items():
        for ch in range(u.shape[0]):
            pending[f"serving/sample_720p_{j}/ch{ch}"] = (("serve", (0, j), ch), u[ch])
    res = {"workload": "Poisson arrivals (seed 50), RGB 1280x720 / 1920x1080 / 3840x2160 uniform, "
                       "Bernoulli 0.5-10 % (2 images x 8 masks per size), float16 correction "
                       f"storage, rel-res {args.tol:g}, inputs resident in HBM, max_batch 64",
           "points": points,
           "plain_fps": round(len(plain_reqs) / t_plain, 2)}
    res["speedup_burst_vs_plain"] = round(points["burst"]["fps"] / res["plain_fps"], 3)
    for j in keep:
        res[f"sample_720p_{j}"] = {}
    return res


if __name__ == "__main__":
    sys.exit(main())
