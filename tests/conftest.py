import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)

FULLSIZE = "test_gpu_x_fullsize.py"
_refs = None


def _selects_fullsize(config) -> bool:
    """Whether this session may run the full-size GPU parity tests: a GPU
    device node exists, the marker expression keeps GPU tests, and the
    arguments name the tests directory or the full-size file."""
    if not os.path.exists("/dev/kfd"):
        return False
    expr = (config.option.markexpr or "").replace(" ", "")
    if "notgpu" in expr:
        return False
    for a in config.args or [os.getcwd()]:
        p = os.path.abspath(a.split("::")[0])
        if p in (TESTS, ROOT) or os.path.basename(p) == FULLSIZE:
            return True
    return False


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")
    global _refs
    # the oracle's full-size references start here, before anything touches
    # the GPU, and are computed while the other tests run
    if _refs is None and _selects_fullsize(config):
        import oracle_refs
        _refs = oracle_refs.RefPool(oracle_refs.full_size_jobs())
        _refs.report = _live_printer(config)


def _live_printer(config):
    """A print that reaches the terminal while pytest captures output (the
    progress of long waits for oracle references)."""
    capman = config.pluginmanager.getplugin("capturemanager")

    def report(msg):
        if capman is None:
            print(msg, flush=True)
            return
        with capman.global_and_fixture_disabled():
            print(msg, flush=True)
    return report


def pytest_unconfigure(config):
    global _refs
    if _refs is not None:
        _refs.close()
        _refs = None


@pytest.fixture(scope="session")
def oracle_refs(pytestconfig):
    """The session's pool of oracle reference solutions (started on demand
    when the session did not start it up front)."""
    global _refs
    if _refs is None:
        import oracle_refs as mod
        _refs = mod.RefPool(mod.full_size_jobs())
        _refs.report = _live_printer(pytestconfig)
    return _refs


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
