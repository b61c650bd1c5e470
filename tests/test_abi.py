"""The C ABI library loads and exports every function include/*.h declares (CPU only)."""
import ctypes
import glob
import os
import re

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
