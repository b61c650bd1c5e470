"""Oracle reference solutions of the full-size workloads (test infrastructure).

The oracle (float64 Jacobi-PCG to a relative residual of 1e-12) takes about a
minute per 4K channel, so the references of the full-size parity tests are
computed in worker processes that start before the test session touches the
GPU (``conftest.pytest_configure``) and run while the other tests do.  Each
job names one channel of one seeded workload; a worker regenerates the inputs
from the seeds in ``paper_2401_06744_amd.synth`` and returns the oracle's
solution of that channel.  Results are cached per session, keyed by the job.

Jobs:
  ("4k", density, ch)                       the 4K RGB frame, shared Bernoulli mask
  ("prec", kind, ch)                        the 4K frame with a 1 % Bernoulli / blue-noise mask
  ("batched", i, ch)                        problem i of the 64-problem batch
  ("frame", W, H, C, img_seed, density, mask_seed, ch)
                                            synth.frame_image + synth.bernoulli_mask
  ("pan", t, ch)                            frame t of the 4K panning video (synth.pan_frame)
  ("msearch", k, ch)                        the 4K frame with step k of the mask search
                                            (synth.mask_search of its 4 % mask)
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

TOL = 1e-12

# the workloads of the full-size parity tests (tests/test_gpu_x_fullsize.py)
BATCHED_SAMPLE_STRIDE = 8
SERVED = {"4k": (3840, 2160, 3, 90, 0.03, 91), "1080p": (1920, 1080, 3, 92, 0.05, 93)}
WARM_STEP = 2  # the warm-start sequences are checked at their second step


def job_inputs(job):
    """(f [C][H][W] float32, mask [H][W] uint8) of the workload a job names."""
    from paper_2401_06744_amd import synth
    kind = job[0]
    if kind == "4k":
        return synth.config_4k(density=job[1])
    if kind == "prec":
        return synth.config_precision(job[1])
    if kind == "batched":
        return synth.batched_problem(job[1])
    if kind == "frame":
        W, H, C, fs, d, ms = job[1:7]
        return synth.frame_image(W, H, C, seed=fs), synth.bernoulli_mask(W, H, d, seed=ms)
    if kind == "pan":
        return synth.pan_frame(3840, 2160, job[1])
    if kind == "msearch":
        f, m = synth.config_4k()
        return f, synth.mask_search(m, job[1])[job[1]]
    raise ValueError(f"unknown job {job!r}")


def solve_job(job):
    """The oracle's float64 solution of the job's channel."""
    import oracle
    f, m = job_inputs(job)
    ch = job[-1]
    return oracle.solve_pcg(np.ascontiguousarray(f[ch], dtype=np.float64), m, tol=TOL)[0]


def _init_worker():
    # one BLAS/OpenMP thread per worker: the pool already uses the cores
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # noqa: BLE001 - only a performance setting
        pass


def batched_sample():
    """Indices of the batched problems checked against the oracle: the four
    largest and every eighth by size (a stratified sample)."""
    from paper_2401_06744_amd import synth
    specs = synth.batched_specs()
    order = sorted(range(len(specs)), key=lambda k: specs[k][0] * specs[k][1] * specs[k][2])
    return sorted(set(order[-4:]) | set(order[::BATCHED_SAMPLE_STRIDE]))


def full_size_jobs():
    """Every job of the full-size parity tests, the longest first."""
    from paper_2401_06744_amd import synth
    jobs = [("prec", k, ch) for k in ("bernoulli", "bluenoise") for ch in range(3)]
    jobs += [("4k", 0.04, ch) for ch in range(3)]
    jobs += [("frame", *SERVED["4k"], ch) for ch in range(SERVED["4k"][2])]
    jobs += [(kind, WARM_STEP, ch) for kind in ("pan", "msearch") for ch in range(3)]
    specs = synth.batched_specs()
    bj = [("batched", i, ch) for i in batched_sample() for ch in range(specs[i][2])]
    bj.sort(key=lambda j: -specs[j[1]][0] * specs[j[1]][1])
    jobs += bj
    jobs += [("frame", *SERVED["1080p"], ch) for ch in range(SERVED["1080p"][2])]
    return jobs


class RefPool:
    """Worker processes computing oracle references; ``get`` waits for one."""

    def __init__(self, jobs, workers=None):
        workers = workers or min(len(jobs), 14, max(1, (os.cpu_count() or 2) - 2))
        self._pool = mp.get_context("spawn").Pool(workers, initializer=_init_worker)
        self._res = {job: self._pool.apply_async(solve_job, (job,)) for job in jobs}
        self._cache = {}
        self.report = lambda msg: print(msg, flush=True)

    def get(self, job, timeout=1800.0):
        if job not in self._cache:
            if job not in self._res:
                self._res[job] = self._pool.apply_async(solve_job, (job,))
            t = time.perf_counter()
            res = self._res[job]
            # wait in slices with a progress line, so that a long wait is
            # visibly a wait and not a hang
            while not res.ready():
                waited = time.perf_counter() - t
                if waited > timeout:
                    raise TimeoutError(f"oracle reference {job}: no result after {waited:.0f} s")
                res.wait(min(30.0, timeout - waited))
                if not res.ready():
                    done = sum(r.ready() for r in self._res.values())
                    self.report(f"oracle reference {job}: waiting {time.perf_counter() - t:.0f} s "
                                f"({done}/{len(self._res)} references done)")
            self._cache[job] = res.get(0)
            waited = time.perf_counter() - t
            if waited > 1.0:
                print(f"oracle reference {job}: waited {waited:.1f} s", flush=True)
        return self._cache[job]

    def close(self):
        self._pool.terminate()
        self._pool.join()
