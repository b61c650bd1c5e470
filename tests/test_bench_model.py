"""The benchmark's cost model (CPU only): the grid levels and block counts it
prices agree with the oracle's geometry and the paper's figures, and the frame
bytes it reports are those the committed profile summary quotes."""
import os
import re

import pytest

import bench
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("W,H", [(3840, 2160), (256, 256), (1920, 1080), (97, 33), (33, 2)])
def test_level_sizes_follow_the_oracle(W, H):
    assert bench.level_sizes(W, H) == oracle.level_sizes(W, H, 32)


def test_4k_geometry_matches_the_paper():
    """Section 3.1: 36852 local problems for a 4K RGB image (32x32 blocks,
    overlap 6); Section 4.4: 8 levels at 4K."""
    assert 3 * bench._blocks(3840) * bench._blocks(2160) == 36852
    assert len(bench.level_sizes(3840, 2160)) == 8


def test_frame_model_is_additive_in_cycles_and_channels():
    """Each V-cycle adds the same bytes; every term but the mask scales with
    the channel count."""
    W, H = 3840, 2160
    b = {k: bench.frame_model_bytes(W, H, 3, k) for k in (1, 2, 3)}
    assert b[3] - b[2] == pytest.approx(b[2] - b[1], rel=1e-12)
    one, three = bench.frame_model_bytes(W, H, 1, 2), bench.frame_model_bytes(W, H, 3, 2)
    assert three - W * H == pytest.approx(3 * (one - W * H), rel=1e-12)
    # a V-cycle moves at least one full ORAS iteration pair of the finest grid
    assert b[2] - b[1] > 3 * 2 * bench.MODEL_BPX["oras"] * W * H


def test_profile_summary_quotes_the_model():
    """The kernel-time summary states the algorithmic bytes of one frame that
    the benchmark's roofline uses (2 V-cycles at 4K RGB)."""
    text = open(os.path.join(ROOT, "profiles", "kernel_stats_4k_rgb.md")).read()
    m = re.search(r"executed schedule \((\d+) V-cycles\) = ([\d.]+) GB", text)
    assert m, "summary does not state the frame's algorithmic bytes"
    cycles, gb = int(m.group(1)), float(m.group(2))
    assert bench.frame_model_bytes(3840, 2160, 3, cycles) / 1e9 == pytest.approx(gb, abs=5e-4)


def test_algorithmic_bytes_cover_every_kernel_class():
    for cls in ("block_solve", "update", "prolong", "restrict", "residual", "stage", "pyramid", "output",
                "coarse"):
        assert bench.algorithmic_bytes(cls, 3840, 2160, 3) > 3840 * 2160


def test_more_than_one_gpu_is_refused_before_any_work():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
