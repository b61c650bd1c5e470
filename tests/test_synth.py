"""Seeded input generators: the workload recipes hold what they promise."""
import numpy as np
from scipy.spatial import cKDTree

from paper_2401_06744_amd import synth


def test_blue_noise_mask_density_and_spacing():
    m, d = synth.blue_noise_mask(300, 200, 0.02, seed=3)
    assert abs(d - 0.02) < 0.2 * 0.02
    pts = np.argwhere(m).astype(np.float64)
    nn = cKDTree(pts).query(pts, k=2)[0][:, 1]
    # Poisson-disk: no two samples closer than a fixed fraction of the mean spacing
    assert nn.min() >= 0.6 / np.sqrt(0.02)
    m2, _ = synth.blue_noise_mask(300, 200, 0.02, seed=3)
    assert np.array_equal(m, m2)


def test_bernoulli_and_images_are_seeded_and_in_range():
    m = synth.bernoulli_mask(400, 300, 0.04, seed=20)
    assert abs(m.mean() - 0.04) < 0.004
    assert np.array_equal(m, synth.bernoulli_mask(400, 300, 0.04, seed=20))
    f = synth.frame_image(64, 48, 3, seed=10)
    assert f.shape == (3, 48, 64) and f.dtype == np.float32
    assert f.min() >= 0.0 and f.max() <= 255.0


def test_batched_and_trace_recipes():
    probs = synth.batched_problems(n=6, seed=40, wmax=300, hmax=200)
    for f, m in probs:
        C, H, W = f.shape
        assert 128 <= W <= 300 and 128 <= H <= 200 and C in (1, 3)
        assert 0.005 < m.mean() < 0.12
    tr = synth.poisson_trace(100.0, 2000, seed=50)
    t = np.array([a[0] for a in tr])
    assert np.all(np.diff(t) > 0)
    assert abs(np.diff(t).mean() - 0.01) < 0.001
    assert {(w, h) for _, w, h, _ in tr} == {(1280, 720), (1920, 1080), (3840, 2160)}
    assert all(0.005 <= d <= 0.10 for *_, d in tr)


def test_edge_mask_concentrates_on_region_borders():
    W, H = 480, 270
    e = synth.region_edges(W, H, region_seed=10)
    f = synth.frame_image(W, H, 1, seed=10)
    # region borders are where the piecewise-constant part of the image jumps
    jump = np.zeros((H, W), bool)
    d = np.abs(np.diff(f[0], axis=1)) > 8.0
    jump[:, 1:] |= d
    jump[:, :-1] |= d
    assert (jump & e).sum() > 0.5 * jump.sum()
    m = synth.edge_mask(W, H, 0.02, seed=5, region_seed=10)
    assert abs(m.mean() - 0.02) < 0.004
    share = (m.astype(bool) & e).sum() / m.sum()
    assert 0.7 < share < 0.9
    assert np.array_equal(m, synth.edge_mask(W, H, 0.02, seed=5, region_seed=10))


def test_warm_start_sequences():
    m = synth.bernoulli_mask(300, 200, 0.05, seed=3)
    seq = synth.mask_search(m, 3, share=0.02, seed=42)
    k = int(m.sum())
    moved = int(round(0.02 * k))
    for a, b in zip(seq, seq[1:]):
        assert int(b.sum()) == k                      # the same number of known pixels
        assert int((a & ~b).sum()) == moved           # moved away ...
        assert int((b & ~a).sum()) == moved           # ... to pixels unknown before
    assert np.array_equal(synth.mask_search(m, 3, share=0.02, seed=42)[3], seq[3])  # seeded
    f0, m0 = synth.pan_frame(64, 32, 0)
    f2, m2 = synth.pan_frame(64, 32, 2)
    assert np.array_equal(f2[:, :, 2:], f0[:, :, :-2]) and not np.array_equal(m0, m2)
