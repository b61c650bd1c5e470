"""The C ABI library loads and exports every function include/*.h declares (CPU only)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2401_06744_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(inpaint_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_entry_points():
    d = _declared()
    assert {"inpaint_solve", "inpaint_solve_ex", "inpaint_last_error"} <= d


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    for name in sorted(_declared()):
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)
    assert set(binding.EXPORTED) == _declared()


def test_host_only_calls_without_gpu():
    assert binding.inpaint_version().startswith("inpaint-mi355x")
    assert binding.inpaint_hierarchy_size(3840, 2160, 32) == (8, 3840 * 2160 + 1920 * 1080 + 960 * 540
                                                             + 480 * 270 + 240 * 135 + 120 * 68
                                                             + 60 * 34 + 30 * 17)
    assert binding.inpaint_hierarchy_size(256, 256, 32)[0] == 4
    try:
        binding.inpaint_hierarchy_size(0, 5, 32)
    except binding.InpaintError as e:
        assert e.code == binding.E_INVALID
    else:
        raise AssertionError("expected E_INVALID")


def test_opts_struct_layout_matches_header():
    # 15 fields of 4 bytes each
    assert ctypes.sizeof(binding.InpaintOpts) == 15 * 4
    # ... + status, padding, three serving times
    assert ctypes.sizeof(binding.InpaintStats) == (8 + 3 * 4 + 4 + 8 + 4 + 4 + 8 + 8 + 8 + 9 * 4 + 9 * 4
                                                   + 4 + 4 + 3 * 8)
    assert ctypes.sizeof(binding.InpaintProblem) == 8 + 8 + 3 * 4 + 4 + 8
    assert ctypes.sizeof(binding.InpaintServerCfg) == 4 + 4 + 8 + 15 * 4 + 4


def test_binding_constants_match_the_header():
    """Every status, schedule, restriction and precision value of the header
    has the same value under the binding's name for it."""
    src = ""
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src += re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
    consts = {m.group(1): int(m.group(2)) for m in re.finditer(r"\bINPAINT_(\w+)\s*=\s*(-?\d+)", src)}
    checked = 0
    for name, value in consts.items():
        if name.startswith(("K_", "NUM_")):
            continue
        assert getattr(binding, name) == value, name
        checked += 1
    assert checked >= 20
    assert len(binding.KERNELS) == consts["NUM_KERNELS"]
    for i, k in enumerate(binding.KERNELS):
        assert consts["K_" + k.upper()] == i, k


def _fake_solve(W, H, C=1, **opts):
    """inpaint_solve_ex on fake, never dereferenced addresses: the size checks
    run before any pointer is used and before any device call."""
    lib = binding.lib()
    o = binding.make_opts(**opts) if opts else None
    code = lib.inpaint_solve_ex(ctypes.c_void_p(1 << 44), ctypes.c_void_p(2 << 44), W, H, C, 1e-6,
                                ctypes.c_void_p(3 << 44), ctypes.byref(o) if o is not None else None,
                                None, None)
    return code, binding.inpaint_last_error()


def test_sizes_beyond_32_bit_offsets_are_rejected_before_any_work():
    """The kernels address one channel's fields and block corrections with
    32-bit offsets and split pixel indices exactly only below 2^24: larger
    problems are rejected as invalid, before any allocation or device call."""
    # 1.6 Gpx: the plane fits, the weighted block corrections (about 1.5 planes
    # at block 32, overlap 6) do not
    code, msg = _fake_solve(40000, 40000)
    assert code == binding.E_INVALID and "32-bit" in msg, (code, msg)
    # 0.54 Gpx at block 16, overlap 8: four planes of corrections
    code, msg = _fake_solve(23200, 23200, block=16, overlap=8)
    assert code == binding.E_INVALID and "32-bit" in msg, (code, msg)
    # one side of 2^24 pixels
    code, msg = _fake_solve(1 << 24, 2)
    assert code == binding.E_INVALID and "2^24" in msg, (code, msg)
    code, msg = _fake_solve(3, 1 << 24)
    assert code == binding.E_INVALID and "2^24" in msg, (code, msg)


def test_odd_overlaps_are_rejected_before_any_work():
    """The overlap is twice the per-side halo of a block (even): an odd one is
    an invalid option, rejected before any pointer is used."""
    for o in (3, 5, 7):
        code, msg = _fake_solve(64, 64, overlap=o)
        assert code == binding.E_INVALID and "even" in msg, (o, code, msg)


def test_noalloc_entry_point_checks_before_device_work():
    """inpaint_solve_noalloc rejects bad options and the comparison CG
    schedules before it looks at the pointers or the device."""
    lib = binding.lib()
    for opts in (binding.make_opts(overlap=5), binding.make_opts(schedule=binding.SCHED_CG)):
        code = lib.inpaint_solve_noalloc(ctypes.c_void_p(1 << 44), ctypes.c_void_p(2 << 44), 64, 64, 1,
                                         1e-6, ctypes.c_void_p(3 << 44), ctypes.byref(opts), None, None)
        assert code == binding.E_INVALID, (code, binding.inpaint_last_error())
    assert binding.NOALLOC_SCRATCH_BYTES == 256 << 20


def test_batched_stats_view_reads_the_struct():
    """The batched binding returns one read-only mapping per problem over the
    C statistics struct: same keys and values as the dict of a single solve."""
    s = binding.InpaintStats()
    s.rel_res, s.cycles, s.status = 3.5e-7, 2, binding.NOT_CONVERGED
    s.kernel_calls[2] = 4
    v = binding.StatsView(s)
    assert dict(v) == s.as_dict()
    assert v["cycles"] == 2 and v["rel_res"] == 3.5e-7 and v["status"] == binding.NOT_CONVERGED
    assert v["kernel_calls"][2] == 4 and len(v) == len(binding.InpaintStats._fields_)
    with pytest.raises(KeyError):
        v["no_such_field"]


def test_schedules_are_validated_and_the_server_refuses_a_warm_start():
    """Schedules 0..7 are accepted (7 = warm start from the guess in out), any
    other value is invalid before any work; the request loop solves from the
    cascade and rejects a warm start before it touches the device."""
    code, msg = _fake_solve(64, 64, schedule=8)
    assert code == binding.E_INVALID and "schedule" in msg, (code, msg)
    assert binding.SCHED_WARM == 7
    # an accepted schedule gets past option checks to the size checks
    code, msg = _fake_solve(1 << 24, 2, schedule=binding.SCHED_WARM)
    assert code == binding.E_INVALID and "2^24" in msg, (code, msg)
    cfg = binding.InpaintServerCfg()
    cfg.struct_size = ctypes.sizeof(binding.InpaintServerCfg)
    cfg.opts = binding.make_opts(schedule=binding.SCHED_WARM)
    h = ctypes.c_void_p()
    code = binding.lib().inpaint_server_create(ctypes.byref(cfg), ctypes.byref(h))
    assert code == binding.E_INVALID and "cascade" in binding.inpaint_last_error()
