"""Readers for the hand-worked text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(lines, i, n):
    return np.array([[float(t) for t in lines[i + k].split()] for k in range(n)]), i + n


def small_systems():
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "small_systems.txt"))
             if ln.strip() and not ln.lstrip().startswith("#")]
    cases, i = [], 0
    while i < len(lines):
        _, name, H, W = lines[i].split()
        H, W = int(H), int(W)
        assert lines[i + 1] == "mask"
        mask, i = _rows(lines, i + 2, H)
        assert lines[i] == "f"
        f, i = _rows(lines, i + 1, H)
        assert lines[i] == "u"
        u, i = _rows(lines, i + 1, H)
        assert lines[i] == "end"
        i += 1
        cases.append((name, mask.astype(np.uint8), f, u))
    return cases


def pyramid_cases():
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "pyramid_4x4.txt"))
             if ln.strip() and not ln.lstrip().startswith("#")]
    cases, i, cur, key, buf = [], 0, {}, None, []
    for ln in lines:
        if ln in ("fine_mask", "fine_b", "coarse_mask", "naive", "modified", "end"):
            if key is not None:
                cur[key] = np.array(buf)
            key, buf = ln, []
            if ln == "end":
                cases.append(cur)
                cur, key = {}, None
            continue
        buf.append([float(t) for t in ln.split()])
    return cases
