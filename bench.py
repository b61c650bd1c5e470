"""Benchmark: 4K RGB homogeneous diffusion inpainting on one MI355X.

One step = one full solve of a 3840x2160x3 frame (shared 4 % Bernoulli mask,
seeded synthetic image) to a relative residual of 1e-6 through the C ABI,
with f, mask and out resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Legs:
  timed      K solves between two device synchronisations -> frames/s, p50/p99
  profiled   K more solves with HIP events around every finest-grid launch ->
             average duration per kernel class, algorithmic bytes and flops per
             launch -> roofline of the dominant kernel
  accuracy   relative residual of the output (float64, on the device) and, on
             channel 0, max abs error against the CPU oracle solved to 1e-12
  cpu        the CPU oracle (Jacobi-PCG, float64, one core) on channel 0 to
             rel-res 1e-6, scaled to frames/s of the 3-channel frame
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
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
KERNEL_SRC = os.path.join(ROOT, "paper_2401_06744_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_4k_rgb.txt")
COPY_BYTES = 1 << 29   # calibration copy: 512 MiB read + 512 MiB written


def kernel_source_sha() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


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


def algorithmic_bytes(cls: str, W: int, H: int, C: int) -> float:
    """Bytes one finest-grid launch of a kernel class must move (each input read
    once, each output written once; halo and overlap re-reads not counted)."""
    N = float(W * H)
    f4 = 4.0 * C * N
    return {
        "block_solve": 2 * f4 + N,            # read r, mask; write D_i v_i (once per pixel)
        # read u, corrections, b, mask; write u and r (20C + 1 B/px), or, for the
        # update that also restricts (one per V-cycle level visit), write u and the
        # coarse b, u, r instead of r (19C + 1.25 B/px); the finest grid sees one
        # of each per V-cycle, so a launch averages the two
        "update": 0.5 * ((5 * f4 + N) + (4.75 * f4 + 1.25 * N)),
        "prolong": 4 * f4 + f4 / 4 + N,       # read u, b, mask, coarse e (N/4); write u, r
        "restrict": f4 + 3 * f4 / 4 + N / 4,  # read r, coarse mask; write coarse b, u, r
        "residual": 3 * f4 + N,               # read u, b, mask; write r
        "stage": 3 * f4 + 2 * N,              # read f, mask; write b, u, mask (per stage launch)
        "pyramid": N + f4 + 1.25 * N / 4 + f4 / 4,
        "output": 3 * f4 + N,                 # read u, b, mask; write out
        "coarse": 3 * f4 + N,
    }[cls]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--width", type=int, default=3840)
    ap.add_argument("--height", type=int, default=2160)
    ap.add_argument("--density", type=float, default=0.04)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 512 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "frames and requests shard across GPUs without communication, see DESIGN.md",
              file=sys.stderr)
        return 2

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
    opts = binding.make_opts()

    def step(o):
        return binding.inpaint_solve_ex(fd, md, args.tol, out=od, opts=o, stream=stream)

    for _ in range(args.warmup):
        step(opts)
    torch.cuda.synchronize()

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

    # ---- profiled leg: per-kernel HIP events on the solve's stream
    popts = binding.make_opts(profile=1)
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
        }
    # block solve: algorithmic flops per launch from the measured local iterations
    bs_i = binding.KERNELS.index("block_solve")
    bs_calls = kcalls[bs_i]
    blocks_per_launch = fin_solves / bs_calls if bs_calls else 0
    iters_per_block = cg_fin / fin_solves if fin_solves else 0.0
    bs_flops = CG_FLOPS_PER_PIXEL_ITER * cg_px / bs_calls if bs_calls else 0.0
    if bs_calls:
        avg = kernels["block_solve"]["avg_ms"] * 1e-3
        kernels["block_solve"]["alg_flops_per_launch"] = bs_flops
        kernels["block_solve"]["alg_TFLOPs"] = round(bs_flops / avg / 1e12, 3)
        kernels["block_solve"]["local_iters_per_block"] = round(iters_per_block, 3)
        kernels["block_solve"]["blocks_per_launch"] = blocks_per_launch
    dom = max(kernels, key=lambda k: kms[binding.KERNELS.index(k)])
    dk = kernels[dom]
    hbm_frac = dk["alg_GBps"] / HBM_PEAK_GBS
    if dom == "block_solve":
        alu_frac = dk["alg_TFLOPs"] / FP32_VECTOR_PEAK_TFLOPS
        roof = {"bound": "alu", "achieved": dk["alg_TFLOPs"], "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": None,
                "kernel": dom, "hbm_GBps": dk["alg_GBps"], "hbm_frac": round(hbm_frac, 4),
                "peak_nonpacked_fp32": FP32_NONPACKED_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": dk["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4), "traffic": None, "kernel": dom}
    roof["traffic"] = measured_traffic(dom)

    if args.calibrate_copy:
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- accuracy of the last output
    rr = binding.inpaint_rel_res(od, fd, md)
    out0 = od[0].float().cpu().numpy()
    acc = {"rel_res_max": float(rr.max()), "status": int(max(statuses)),
           "known_exact": bool(np.array_equal(out0[m != 0], f[0][m != 0]))}

    # ---- CPU oracle legs
    cpu = None
    if not args.no_cpu_baseline or not args.no_oracle_check:
        import oracle
        f0 = f[0].astype(np.float64)
        if not args.no_cpu_baseline:
            tc = time.perf_counter()
            _, its = oracle.solve_pcg(f0, m, tol=args.tol, return_iters=True)
            tcpu = time.perf_counter() - tc
            cpu = {"value": round(1.0 / (C * tcpu), 5), "unit": "frames/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"channel 0 of the same 4K frame, float64 Jacobi-PCG to rel-res "
                             f"{args.tol:g} ({its[0]} iterations, {tcpu:.1f} s), scaled to 3 channels"}
        if not args.no_oracle_check:
            ref = oracle.solve_pcg(f0, m, tol=1e-12)[0]
            acc["max_err_vs_oracle_ch0"] = float(np.abs(out0.astype(np.float64) - ref).max())

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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{W}x{H} RGB frame, shared Bernoulli {args.density:.0%} mask, "
                               f"FMG+ORAS to rel-res {args.tol:g}",
                   "W": W, "H": H, "channels": C, "density": args.density, "tol": args.tol,
                   "block": 32, "overlap": 6, "schedule": "reduced FMG"},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "cycles": int(np.median(cycles)),
        "local_cg_mean": round(float(np.mean(cg_mean)), 3),
        "roofline": roof,
        "kernels": kernels,
        "accuracy": acc,
        "cpu_baseline": cpu,
        "paper_context": "14.3 ms (70 fps) per 4K RGB frame at rel-res 1e-3 on a GTX 1080 Ti",
    }
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
