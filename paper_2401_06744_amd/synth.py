"""Seeded synthetic inputs: images, masks, batches and arrival traces.

This module draws random images and inpainting masks and nothing else: it
holds none of the solver's arithmetic, so both the GPU path and the CPU
checker can take their inputs from it without sharing any method code.

The paper evaluates on twelve 4K photographs with optimised (Delaunay
densified) masks that are not available here.  The generators below stand in
for them with the same shapes (4K, FullHD, 720p, RGB or grey), the same
density range (0.5 % to 10 %, Section 5.2) and a mix of smooth regions and
edges.  Bernoulli masks leave larger voids than optimised masks do, which is
the harder case for the solver; blue-noise masks imitate the even spacing of
optimised masks in flat regions.

All images are planar float32 ``[C][H][W]`` in [0, 255]; masks are uint8
``[H][W]`` with 1 = known pixel.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "smooth_field", "voronoi_field", "plain_image", "frame_image",
    "bernoulli_mask", "blue_noise_mask", "region_edges", "edge_mask", "config_small", "config_4k",
    "config_precision", "batched_specs", "batched_problem", "batched_problems", "poisson_trace",
]


def _scale01(a: np.ndarray) -> np.ndarray:
    lo, hi = float(a.min()), float(a.max())
    if hi <= lo:
        return np.zeros_like(a)
    return (a - lo) / (hi - lo)


def smooth_field(rng: np.random.Generator, W: int, H: int, n_gauss: int = 8) -> np.ndarray:
    """Sum of ``n_gauss`` random 2-D Gaussians plus a linear ramp, in [0, 1].

    Centres are uniform over the frame, widths uniform in [n/16, n/4] with
    n = min(W, H), amplitudes uniform in [-1, 1]; the ramp is a*x/W + b*y/H
    with a, b uniform in [-1, 1].
    """
    n = float(min(W, H))
    x = np.arange(W, dtype=np.float64)[None, :]
    y = np.arange(H, dtype=np.float64)[:, None]
    img = np.zeros((H, W), dtype=np.float64)
    for _ in range(n_gauss):
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        sig = rng.uniform(n / 16.0, n / 4.0)
        amp = rng.uniform(-1.0, 1.0)
        gx = np.exp(-((x - cx) ** 2) / (2 * sig * sig))
        gy = np.exp(-((y - cy) ** 2) / (2 * sig * sig))
        img += amp * (gy * gx)
    a, b = rng.uniform(-1, 1, size=2)
    img += a * x / W + b * y / H
    return _scale01(img)


def voronoi_field(rng: np.random.Generator, W: int, H: int, n_seeds: int = 64) -> np.ndarray:
    """Nearest-seed region labels in ``[0, n_seeds)`` (piecewise-constant regions)."""
    from scipy.spatial import cKDTree

    pts = np.stack([rng.uniform(0, W, n_seeds), rng.uniform(0, H, n_seeds)], axis=1)
    tree = cKDTree(pts)
    labels = np.empty((H, W), dtype=np.int32)
    xs = np.arange(W, dtype=np.float64)
    step = max(1, (1 << 20) // max(W, 1))
    for y0 in range(0, H, step):
        y1 = min(H, y0 + step)
        yy, xx = np.meshgrid(np.arange(y0, y1, dtype=np.float64), xs, indexing="ij")
        q = np.stack([xx.ravel() + 0.5, yy.ravel() + 0.5], axis=1)
        labels[y0:y1] = tree.query(q)[1].reshape(y1 - y0, W)
    return labels


def plain_image(W: int, H: int, seed: int) -> np.ndarray:
    """Grey image ``[1][H][W]``: smooth field scaled to [0, 255]."""
    rng = np.random.default_rng(seed)
    return (255.0 * smooth_field(rng, W, H)).astype(np.float32)[None]


def frame_image(W: int, H: int, channels: int, seed: int, region_seed: int | None = None) -> np.ndarray:
    """Image ``[C][H][W]``: 0.6 * smooth field + 0.4 * piecewise-constant regions.

    The 64 Voronoi regions are shared by all channels (drawn from
    ``region_seed``); each channel has its own smooth field (seed + ch) and its
    own per-region levels, so edges line up across channels as in a photo.
    """
    rs = seed if region_seed is None else region_seed
    labels = voronoi_field(np.random.default_rng(rs + 1_000_003), W, H)
    out = np.empty((channels, H, W), dtype=np.float32)
    for ch in range(channels):
        rng = np.random.default_rng(seed + ch)
        sm = smooth_field(rng, W, H)
        levels = rng.uniform(0.0, 1.0, size=int(labels.max()) + 1)
        img = 0.6 * sm + 0.4 * levels[labels]
        out[ch] = (255.0 * _scale01(img)).astype(np.float32)
    return out


def bernoulli_mask(W: int, H: int, density: float, seed: int) -> np.ndarray:
    """Each pixel known with probability ``density``; never empty (pixel (0,0) forced)."""
    rng = np.random.default_rng(seed)
    m = (rng.random((H, W)) < density).astype(np.uint8)
    if not m.any():
        m[0, 0] = 1
    return m


def _poisson_disk(rng: np.random.Generator, W: int, H: int, radius: float, rounds: int = 24) -> np.ndarray:
    """Poisson-disk sampling by phased dart throwing on a background grid of
    cells of side radius/sqrt(2) (each holds at most one point); returns an
    (n, 2) array of (x, y).

    Every round visits the 9 cell phases (x mod 3, y mod 3) in random order and
    throws one dart into each empty cell of the phase; a dart is kept when no
    point of the 5x5 cell neighbourhood lies closer than the radius.  Cells of
    one phase are at least two cells (1.41 radii) apart, so their darts never
    conflict and a whole phase is processed at once."""
    cell = radius / np.sqrt(2.0)
    gw, gh = int(np.ceil(W / cell)), int(np.ceil(H / cell))
    px = np.full((gh + 4, gw + 4), np.nan)
    py = np.full((gh + 4, gw + 4), np.nan)
    gy, gx = np.mgrid[0:gh, 0:gw]
    phase_of = (gy % 3) * 3 + (gx % 3)
    r2 = radius * radius
    for _ in range(rounds):
        for phase in rng.permutation(9):
            sel = (phase_of == phase) & np.isnan(px[2:-2, 2:-2])
            cy, cx = gy[sel], gx[sel]
            if cy.size == 0:
                continue
            x = (cx + rng.random(cx.size)) * cell
            y = (cy + rng.random(cy.size)) * cell
            ok = (x < W) & (y < H)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    qx = px[cy + 2 + dy, cx + 2 + dx]
                    qy = py[cy + 2 + dy, cx + 2 + dx]
                    ok &= ~((qx - x) ** 2 + (qy - y) ** 2 < r2)
            px[cy[ok] + 2, cx[ok] + 2] = x[ok]
            py[cy[ok] + 2, cx[ok] + 2] = y[ok]
    inner_x, inner_y = px[2:-2, 2:-2], py[2:-2, 2:-2]
    keep = ~np.isnan(inner_x)
    return np.stack([inner_x[keep], inner_y[keep]], axis=1)


def blue_noise_mask(W: int, H: int, density: float, seed: int, iters: int = 12) -> tuple[np.ndarray, float]:
    """Poisson-disk mask whose density is calibrated to ``density`` by bisection on the radius.

    Returns ``(mask, achieved_density)``.  Bisection runs on a crop (at most
    512x512) and the calibrated radius is then used for the full frame.
    """
    cw, chh = min(W, 512), min(H, 512)
    lo, hi = 0.5, 4.0 / np.sqrt(max(density, 1e-6))
    for i in range(iters):
        mid = 0.5 * (lo + hi)
        n = len(_poisson_disk(np.random.default_rng(seed + 7919 * i), cw, chh, mid))
        if n / (cw * chh) > density:
            lo = mid
        else:
            hi = mid
    pts = _poisson_disk(np.random.default_rng(seed), W, H, 0.5 * (lo + hi))
    m = np.zeros((H, W), dtype=np.uint8)
    xi = np.clip(pts[:, 0].astype(np.int64), 0, W - 1)
    yi = np.clip(pts[:, 1].astype(np.int64), 0, H - 1)
    m[yi, xi] = 1
    if not m.any():
        m[0, 0] = 1
    return m, float(m.mean())


def region_edges(W: int, H: int, region_seed: int) -> np.ndarray:
    """Pixels on the border of the piecewise-constant regions of
    ``frame_image(..., seed=region_seed)``: a 4-neighbour has another label."""
    labels = voronoi_field(np.random.default_rng(region_seed + 1_000_003), W, H)
    e = np.zeros((H, W), dtype=bool)
    dx = labels[:, 1:] != labels[:, :-1]
    dy = labels[1:, :] != labels[:-1, :]
    e[:, 1:] |= dx
    e[:, :-1] |= dx
    e[1:, :] |= dy
    e[:-1, :] |= dy
    return e


def edge_mask(W: int, H: int, density: float, seed: int, region_seed: int,
              edge_share: float = 0.8) -> np.ndarray:
    """Mask concentrated on the region borders of a ``frame_image``: about
    ``edge_share`` of its ``density * W * H`` known pixels lie on border pixels
    (each border pixel known with one probability, every other pixel with
    another), as masks optimised for such images place their points along
    edges.  Never empty."""
    e = region_edges(W, H, region_seed)
    n = density * W * H
    ne = max(int(e.sum()), 1)
    p_e = min(1.0, edge_share * n / ne)
    p_f = max(0.0, (n - p_e * ne) / max(W * H - ne, 1))
    r = np.random.default_rng(seed).random((H, W))
    m = np.where(e, r < p_e, r < p_f).astype(np.uint8)
    if not m.any():
        m[0, 0] = 1
    return m


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def perturbed_mask(mask: np.ndarray, share: float, seed: int) -> np.ndarray:
    """``mask`` with ``share`` of its known pixels moved to unknown pixels
    drawn at random (the same count known): one step of an encoder's mask
    search."""
    rng = np.random.default_rng(seed)
    m = mask.ravel().copy()
    known = np.flatnonzero(m)
    unknown = np.flatnonzero(m == 0)
    k = int(round(share * known.size))
    m[rng.choice(known, size=k, replace=False)] = 0
    m[rng.choice(unknown, size=k, replace=False)] = 1
    return m.reshape(mask.shape)


def mask_search(mask: np.ndarray, steps: int, share: float = 0.02, seed: int = 42) -> list:
    """``mask`` and ``steps`` successive perturbations of it (seeds seed, seed + 1, ...)."""
    seq = [mask]
    for j in range(steps):
        seq.append(perturbed_mask(seq[-1], share, seed + j))
    return seq


def pan_frame_mask(W: int, H: int, t: int, density: float = 0.04, mask_seed: int = 60) -> np.ndarray:
    """The mask of frame t of the panning video: a fresh Bernoulli mask."""
    return bernoulli_mask(W, H, density, seed=mask_seed + t)


def pan_frame(W: int, H: int, t: int, seed: int = 10, density: float = 0.04, mask_seed: int = 60):
    """Frame t of a panning video: the RGB frame of ``seed`` moved t pixels to
    the right (wrapping), with a fresh Bernoulli mask (seed mask_seed + t)."""
    f = np.ascontiguousarray(np.roll(frame_image(W, H, 3, seed=seed), t, axis=2))
    return f, pan_frame_mask(W, H, t, density, mask_seed)


def config_small(W: int = 256, H: int = 256, density: float = 0.05):
    """256x256 grey, smooth field (seed 1), Bernoulli mask (seed 2)."""
    return plain_image(W, H, seed=1), bernoulli_mask(W, H, density, seed=2)


def config_4k(W: int = 3840, H: int = 2160, density: float = 0.04, channels: int = 3):
    """4K RGB frame (seeds 10+ch, regions seed 10), shared Bernoulli mask (seed 20)."""
    return frame_image(W, H, channels, seed=10), bernoulli_mask(W, H, density, seed=20)


def config_precision(kind: str = "bernoulli", W: int = 3840, H: int = 2160):
    """4K RGB frame with a 1 % mask: Bernoulli (seed 30) or blue noise (seed 31)."""
    img = frame_image(W, H, 3, seed=10)
    if kind == "bernoulli":
        return img, bernoulli_mask(W, H, 0.01, seed=30)
    m, _ = blue_noise_mask(W, H, 0.01, seed=31)
    return img, m


def batched_specs(n: int = 64, seed: int = 40, wmax: int = 1920, hmax: int = 1080,
                  density: float | None = None):
    """Shapes of ``batched_problems``: ``(W, H, C, density, image_seed)`` per problem.

    ``density`` set: every problem gets that mask density, with the same sizes,
    channels and seeds as the default draw."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n):
        W = int(rng.integers(128, wmax + 1))
        H = int(rng.integers(128, hmax + 1))
        C = 1 if rng.random() < 0.5 else 3
        dens = float(rng.uniform(0.01, 0.10))
        s = int(rng.integers(1 << 30))
        specs.append((W, H, C, dens if density is None else density, s))
    return specs


def batched_problem(i: int, n: int = 64, seed: int = 40, wmax: int = 1920, hmax: int = 1080):
    """Problem ``i`` of ``batched_problems(n, seed, wmax, hmax)`` alone."""
    W, H, C, dens, s = batched_specs(n, seed, wmax, hmax)[i]
    return frame_image(W, H, C, seed=s), bernoulli_mask(W, H, dens, seed=s + 1)


def batched_problems(n: int = 64, seed: int = 40, wmax: int = 1920, hmax: int = 1080,
                     density: float | None = None):
    """``n`` problems of uneven size: W in [128, wmax], H in [128, hmax], C in {1, 3}, 1-10 % masks
    (or all at ``density``)."""
    return [(frame_image(W, H, C, seed=s), bernoulli_mask(W, H, dens, seed=s + 1))
            for W, H, C, dens, s in batched_specs(n, seed, wmax, hmax, density)]


def poisson_trace(qps: float, n: int, seed: int = 50):
    """Arrival times (s) of ``n`` requests with exponential gaps, plus their (W, H, density)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=n))
    sizes = [(1280, 720), (1920, 1080), (3840, 2160)]
    pick = rng.integers(0, 3, size=n)
    dens = rng.uniform(0.005, 0.10, size=n)
    return [(float(t[i]), sizes[pick[i]][0], sizes[pick[i]][1], float(dens[i])) for i in range(n)]
