"""The serving core on the CPU: the library's request loop (admission in
arrival order by free slot and HBM footprint, continuous batching, completion,
latency stamps, error isolation) run against a fake executor whose results
come from the oracle.  The fake (tests/fake_serve/fake_executor.cpp) and the
core's sources (paper_2401_06744_amd/csrc/serve_core.cpp, errors.cpp) are built
here with g++; nothing touches a GPU."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2401_06744_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2401_06744_amd", "csrc")
FAKE = os.path.join(ROOT, "tests", "fake_serve", "fake_executor.cpp")

CHECK = ct.CFUNCTYPE(ct.c_int, ct.POINTER(binding.InpaintProblem), ct.POINTER(ct.c_int))
SOLVE = ct.CFUNCTYPE(ct.c_int, ct.POINTER(binding.InpaintProblem), ct.c_double)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("fake_serve") / "libfakeserve.so")
    cmd = ["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "serve_core.cpp"), os.path.join(CSRC, "errors.cpp"), FAKE, "-o", so]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    L = ct.CDLL(so)
    vp = ct.c_void_p
    L.fake_server_create.argtypes = [ct.c_int, ct.c_size_t, ct.c_int, CHECK, SOLVE, ct.POINTER(vp)]
    L.fake_server_release.argtypes = [vp]
    L.fake_server_release.restype = None
    L.fake_server_submit.argtypes = [vp, ct.POINTER(binding.InpaintProblem), ct.c_double,
                                     ct.POINTER(ct.c_uint64)]
    L.fake_server_collect.argtypes = [vp, ct.c_uint64, ct.POINTER(binding.InpaintStats), ct.c_int]
    L.fake_server_last_error.restype = ct.c_char_p
    L.fake_server_log.argtypes = [vp, ct.c_char_p, ct.c_size_t]
    L.fake_server_log.restype = ct.c_size_t
    L.fake_server_peak_bytes.argtypes = [vp]
    L.fake_server_peak_bytes.restype = ct.c_size_t
    L.fake_server_destroy.argtypes = [vp]
    L.fake_server_destroy.restype = None
    return L


def _arrays(p):
    C, H, W = p.channels, p.H, p.W
    f = np.ctypeslib.as_array(ct.cast(p.f, ct.POINTER(ct.c_float)), shape=(C, H, W))
    m = np.ctypeslib.as_array(ct.cast(p.mask, ct.POINTER(ct.c_uint8)), shape=(H, W))
    out = np.ctypeslib.as_array(ct.cast(p.out, ct.POINTER(ct.c_float)), shape=(C, H, W))
    return f, m, out


class Fake:
    """A fake server: requests are registered with the V-cycles they need and
    whether their solve fails; the check rejects what the library's staging
    rejects (no known pixel, non-finite f at a known pixel); the solve writes
    the oracle's solution."""

    def __init__(self, lib, max_batch=4, budget=1 << 30, max_cycles=30):
        self.lib = lib
        self.spec = {}   # address of f -> (cycles, fail)
        self.keep = []   # arrays and problem structs alive while the server runs
        self.pending = set()
        self._check = CHECK(self.check)
        self._solve = SOLVE(self.solve)
        h = ct.c_void_p()
        assert lib.fake_server_create(max_batch, budget, max_cycles, self._check, self._solve,
                                      ct.byref(h)) == 0
        self.h = h

    def check(self, pp, cycles):
        try:
            p = pp.contents
            f, m, _ = _arrays(p)
            if not m.any():
                return binding.E_EMPTY_MASK
            if not np.all(np.isfinite(f[:, m != 0])):
                return binding.E_INVALID
            cycles[0] = self.spec[p.f][0]
            return 0
        except Exception:  # noqa: BLE001 - a callback must not raise into C
            return binding.E_DEVICE

    def solve(self, pp, tol):
        try:
            p = pp.contents
            if self.spec[p.f][1]:
                return binding.E_DEVICE
            f, m, out = _arrays(p)
            out[:] = oracle.solve_pcg(f.astype(np.float64), m).astype(np.float32)
            return 0
        except Exception:  # noqa: BLE001
            return binding.E_DEVICE

    def submit(self, f, m, cycles=1, fail=False, tol=1e-6):
        out = np.zeros_like(f)
        arr, _ = binding._problems([(f, m, out)])
        self.keep.append((f, m, out, arr))
        self.spec[arr[0].f] = (cycles, fail)
        t = ct.c_uint64()
        code = self.lib.fake_server_submit(self.h, arr, tol, ct.byref(t))
        if code < 0:
            raise binding.InpaintError(code, self.lib.fake_server_last_error().decode())
        self.pending.add(t.value)
        return t.value, out

    def collect(self, t, block=True):
        st = binding.InpaintStats()
        code = self.lib.fake_server_collect(self.h, t, ct.byref(st), 1 if block else 0)
        if code != binding.PENDING:
            self.pending.discard(t)
        if code == binding.E_INVALID and not st.t_done_ms and b"ticket" in self.lib.fake_server_last_error():
            raise binding.InpaintError(code, self.lib.fake_server_last_error().decode())
        return code, st.as_dict()

    def release(self):
        self.lib.fake_server_release(self.h)

    def log(self):
        if not self.h:
            return self._log  # kept by destroy
        n = self.lib.fake_server_log(self.h, None, 0)
        buf = ct.create_string_buffer(n + 1)
        self.lib.fake_server_log(self.h, buf, n + 1)
        return buf.value.decode().splitlines()

    def steps(self):
        out = []
        for line in self.log():
            mt = re.match(r"step cas(.*) going(.*)$", line)
            if mt:
                out.append(([int(x) for x in mt.group(1).split()], [int(x) for x in mt.group(2).split()]))
        return out

    def destroy(self):
        if self.h:
            self.lib.fake_server_release(self.h)
            for t in list(self.pending):
                self.collect(t)  # the destructor would finish them anyway
            self._log = self.log()
            self.lib.fake_server_destroy(self.h)
            self.h = None


def _req(W, H, C, seed, dens=0.05):
    return synth.frame_image(W, H, C, seed=seed), synth.bernoulli_mask(W, H, dens, seed=seed + 1)


def test_arrival_order_continuous_batching_and_oracle_results(lib):
    fk = Fake(lib, max_batch=3)
    try:
        reqs = [_req(40 + 7 * k, 30 + 5 * k, 1 + 2 * (k % 2), seed=10 * k) for k in range(7)]
        cyc = [2, 0, 3, 1, 2, 1, 4]
        sub = [fk.submit(f, m, cycles=c) for (f, m), c in zip(reqs, cyc)]
        fk.release()
        res = [fk.collect(t) for t, _ in sub]
    finally:
        fk.destroy()
    for (f, m), (t, out), (code, st), c in zip(reqs, sub, res, cyc):
        assert code == binding.OK and st["status"] == binding.OK
        assert st["cycles"] == c
        assert 0 <= st["t_submit_ms"] <= st["t_start_ms"] <= st["t_done_ms"]
        assert np.abs(out.astype(np.float64) - oracle.solve_pcg(f.astype(np.float64), m)).max() <= 1e-3
    log = fk.log()
    prepared = [int(x.split()[1]) for x in log if x.startswith("prepare")]
    assert prepared == sorted(prepared) == [t for t, _ in sub]  # arrival order
    steps = fk.steps()
    assert all(len(c) + len(g) <= 3 for c, g in steps)  # at most max_batch in flight
    # continuous batching: requests admitted while others run share a step with them
    assert any(c and g for c, g in steps)
    # each request is cascaded once and then cycles until it leaves
    for t, _ in sub:
        assert sum(t in c for c, _ in steps) == 1


def test_budget_admission_reuse_and_eviction(lib):
    small = _req(32, 32, 1, seed=1)
    big = _req(96, 64, 3, seed=2)
    b_small = 4096 + 32 * 32 * 16
    b_big = 4096 + 96 * 64 * 3 * 16
    budget = b_big + b_small  # one big and one small at a time
    fk = Fake(lib, max_batch=8, budget=budget)
    try:
        with pytest.raises(binding.InpaintError) as e:
            fk.submit(*_req(200, 200, 3, seed=3))  # larger than the whole budget
        assert e.value.code == binding.E_NOMEM
        order = [small, big, small, big, big, small, small]
        sub = [fk.submit(*r, cycles=2) for r in order]
        fk.release()
        res = [fk.collect(t) for t, _ in sub]
        peak = lib.fake_server_peak_bytes(fk.h)
    finally:
        fk.destroy()
    assert all(code == binding.OK for code, _ in res)
    assert peak <= budget
    creates = [x for x in fk.log() if x.startswith("create")]
    # idle hierarchies of the same shape are reused: fewer creations than requests
    assert len(creates) < len(order)
    # at most one big request runs at a time: their runs do not overlap
    bigs = [st for (code, st), r in zip(res, order) if r is big]
    for a, b in zip(bigs, bigs[1:]):
        assert b["t_start_ms"] >= a["t_done_ms"] - 1e-6 or a["t_start_ms"] >= b["t_done_ms"] - 1e-6


def test_errors_are_isolated(lib):
    fk = Fake(lib, max_batch=4)
    try:
        good = [_req(50, 40, 3, seed=20 + k) for k in range(3)]
        f_bad, m_bad = _req(50, 40, 1, seed=30)
        f_inf = f_bad.copy()
        k = np.argwhere(m_bad)[0]
        f_inf[0, k[0], k[1]] = np.inf
        t0, o0 = fk.submit(*good[0], cycles=2)
        t_empty, _ = fk.submit(f_bad, np.zeros_like(m_bad))
        t1, o1 = fk.submit(*good[1], cycles=1)
        t_inf, _ = fk.submit(f_inf, m_bad)
        t_fail, _ = fk.submit(*good[2], cycles=1, fail=True)
        t2, o2 = fk.submit(*good[0], cycles=3)
        fk.release()
        codes = {t: fk.collect(t)[0] for t in (t0, t_empty, t1, t_inf, t_fail, t2)}
    finally:
        fk.destroy()
    assert codes[t_empty] == binding.E_EMPTY_MASK
    assert codes[t_inf] == binding.E_INVALID
    assert codes[t_fail] == binding.E_DEVICE
    assert codes[t0] == codes[t1] == codes[t2] == binding.OK
    for (f, m), o in ((good[0], o0), (good[1], o1), (good[0], o2)):
        assert np.abs(o.astype(np.float64) - oracle.solve_pcg(f.astype(np.float64), m)).max() <= 1e-3


def test_cycle_cap_and_argument_errors(lib):
    fk = Fake(lib, max_batch=2, max_cycles=2)
    try:
        t_slow, _ = fk.submit(*_req(30, 20, 1, seed=40), cycles=5)
        t_ok, _ = fk.submit(*_req(30, 20, 1, seed=41), cycles=2)
        with pytest.raises(binding.InpaintError) as e:
            fk.submit(*_req(30, 20, 1, seed=42), tol=2.0)
        assert e.value.code == binding.E_INVALID
        assert fk.collect(t_ok, block=False)[0] == binding.PENDING  # the loop is held
        fk.release()
        code, st = fk.collect(t_slow)
        assert code == binding.NOT_CONVERGED and st["cycles"] == 2
        assert fk.collect(t_ok)[0] == binding.OK
        with pytest.raises(binding.InpaintError) as e:
            fk.collect(t_ok)
        assert e.value.code == binding.E_INVALID
    finally:
        fk.destroy()


def test_destroy_finishes_submitted_requests(lib):
    fk = Fake(lib, max_batch=2)
    reqs = [_req(40, 30, 3, seed=50 + k) for k in range(4)]
    outs = [fk.submit(f, m, cycles=k % 3)[1] for k, (f, m) in enumerate(reqs)]
    # the destructor itself releases the held loop and finishes every request first
    lib.fake_server_destroy(fk.h)
    fk.h = None
    for (f, m), o in zip(reqs, outs):
        assert np.abs(o.astype(np.float64) - oracle.solve_pcg(f.astype(np.float64), m)).max() <= 1e-3
