"""Plain, slow, float64 reference for homogeneous diffusion inpainting.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg, never by the
product path.

What is here, and the passage each part follows:

* The discrete system ``A u = b`` with ``A = C + (I - C) L`` and ``b = C f``
  (Section 2.2: the entries of ``L`` and the discrete linear system): ``L`` is the
  5-point negated Laplacian with reflecting boundaries, diagonal
  ``|N(i)| / h^2`` and ``-1 / h^2`` for each direct neighbour.  ``h = 1``
  here; it cancels in ``A u = b`` on the finest grid.
* ``solve_pcg``: the unique solution, through the symmetric positive definite
  system on the unknown pixels (Section 2.2, "Practical Considerations"),
  solved by Jacobi-preconditioned CG to a relative residual of 1e-12.
* ``solve_dense``: the same system solved by a dense LU factorisation of the
  full N x N matrix ``A`` (small images only).
* ``rel_res``: the stopping measure of Section 5.2 ("relative decay of the
  Euclidean norm of the residual").  The paper does not name the reference
  residual; the reading used here is the residual of the zero-filled start
  ``C f``:  ``||b - A u|| / ||b - A C f||``.
* Geometry of the method (Sections 3.1 and 4.4): level sizes by halving with
  ceil until one 32x32 block remains; overlapping blocks of side B with
  overlap o placed at stride B - o, the last one clipped at the image edge;
  separable linear partition-of-unity weights, 0 at the outermost overlap
  pixel and 1 at the innermost.
* Coarse problems (Section 4.3): mask max-pooling, the naive masked mean of
  the known values, and the modified, neighbour-weighted mean.
* Grid transfers (Sections 4.1 and 4.4): residual restriction by 2x2
  averaging away from coarse mask pixels, bilinear (cell-centred)
  prolongation.
* ``oras_step``: one iteration of discrete ORAS (Algorithm 2, Section 3) with
  every local problem solved exactly by a sparse direct solver.

Functions whose only check is their own definition are marked
"parity unpinned" in their docstrings; everything else is pinned by
``tests/test_oracle_*.py`` against closed forms, worked examples from the
paper, invariants and brute force.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "neighbour_count", "apply_L", "apply_A", "rhs", "residual", "rel_res",
    "solve_pcg", "solve_dense", "dense_matrix",
    "level_sizes", "block_starts", "num_blocks", "pou_weights_1d", "block_weight_2d",
    "mask_down", "rhs_down_naive", "rhs_down_modified", "restrict_residual",
    "prolong_bilinear", "oras_local_matrix", "oras_step",
]


# ---------------------------------------------------------------------------
# Section 2.2: the discrete system
# ---------------------------------------------------------------------------

def neighbour_count(H: int, W: int) -> np.ndarray:
    """``|N(i)|``: number of direct (4-) neighbours of each pixel inside the image.

    Reflecting boundaries drop the missing neighbours from both the diagonal
    and the off-diagonal of ``L`` (Section 2.2, entries of ``L``).
    """
    n = np.full((H, W), 4, dtype=np.float64)
    n[:, 0] -= 1
    n[:, W - 1] -= 1
    n[0, :] -= 1
    n[H - 1, :] -= 1
    return n


def apply_L(v: np.ndarray, h: float = 1.0) -> np.ndarray:
    """``L v`` for the 5-point negated Laplacian with reflecting boundaries.

    Row i: ``(|N(i)| v_i - sum_{j in N(i)} v_j) / h^2`` (Section 2.2).
    """
    v = np.asarray(v, dtype=np.float64)
    H, W = v.shape
    out = neighbour_count(H, W) * v
    out[:, 1:] -= v[:, :-1]
    out[:, :-1] -= v[:, 1:]
    out[1:, :] -= v[:-1, :]
    out[:-1, :] -= v[1:, :]
    return out / (h * h)


def apply_A(u: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """``A u = C u + (I - C) L u`` (Section 2.2, the discrete system), one channel."""
    c = (np.asarray(mask) != 0).astype(np.float64)
    u = np.asarray(u, dtype=np.float64)
    return c * u + (1.0 - c) * apply_L(u)


def rhs(f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """``b = C f`` (Section 2.2, the discrete system), one channel.  ``f`` at unknown pixels is never read."""
    c = np.asarray(mask) != 0
    return np.where(c, np.asarray(f, dtype=np.float64), 0.0)


def residual(u: np.ndarray, f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """``b - A u`` in float64, one channel."""
    return rhs(f, mask) - apply_A(u, mask)


def rel_res(u: np.ndarray, f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Relative residual ``||b - A u||_2 / ||b - A C f||_2`` per channel (Section 5.2).

    ``u`` and ``f`` are ``[C][H][W]`` (or ``[H][W]``); returns one value per
    channel.  The reference residual is that of the zero-filled start ``C f``
    (the paper names a relative decay but not its start).
    """
    u = np.asarray(u)
    f = np.asarray(f)
    if u.ndim == 2:
        u, f = u[None], f[None]
    out = np.empty(u.shape[0])
    for ch in range(u.shape[0]):
        b = rhs(f[ch], mask)
        num = np.linalg.norm(residual(u[ch], f[ch], mask))
        den = np.linalg.norm(b - apply_A(b, mask))
        out[ch] = num / den if den > 0 else (0.0 if num == 0 else np.inf)
    return out


def _pcg_channel(f: np.ndarray, mask: np.ndarray, tol: float, maxiter: int):
    """Jacobi-preconditioned CG on the unknown pixels (Section 2.2).

    With ``K`` the known pixels and ``U`` the unknown ones, the rows of
    ``A u = b`` at ``U`` read ``L_UU u_U = -L_UK f_K``; ``L_UU`` is symmetric
    positive definite when ``K`` is not empty.  CG runs on full-size arrays
    that are kept at zero on ``K``.  Stops when ``||r_U|| <= tol * ||g||`` with
    ``g = -L_UK f_K`` (the residual of the zero-filled start, so the result
    has ``rel_res <= tol``).
    """
    c = np.asarray(mask) != 0
    unk = (~c).astype(np.float64)
    H, W = c.shape
    fk = np.where(c, np.asarray(f, dtype=np.float64), 0.0)
    g = -apply_L(fk) * unk
    diag = neighbour_count(H, W)
    gnorm = np.linalg.norm(g)
    x = np.zeros((H, W))
    if gnorm == 0.0:
        return fk, 0
    r = g.copy()
    z = r / diag
    p = z.copy()
    rz = float(np.vdot(r, z))
    it = 0
    while it < maxiter and np.linalg.norm(r) > tol * gnorm:
        q = apply_L(p) * unk
        alpha = rz / float(np.vdot(p, q))
        x += alpha * p
        r -= alpha * q
        z = r / diag
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return np.where(c, fk, x), it


def solve_pcg(f: np.ndarray, mask: np.ndarray, tol: float = 1e-12, maxiter: int = 200000,
              return_iters: bool = False):
    """Unique solution of ``A u = b`` per channel, float64, ``[C][H][W]``.

    Raises ``ValueError`` for an empty mask: with reflecting boundaries and no
    known pixel any constant solves the system (Section 2.2).
    """
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    if not np.any(np.asarray(mask) != 0):
        raise ValueError("empty mask: the inpainting system is singular")
    out = np.empty(f.shape, dtype=np.float64)
    iters = []
    for ch in range(f.shape[0]):
        out[ch], it = _pcg_channel(f[ch], mask, tol, maxiter)
        iters.append(it)
    return (out, iters) if return_iters else out


def dense_matrix(mask: np.ndarray) -> np.ndarray:
    """The full ``N x N`` matrix ``A = C + (I - C) L`` (h = 1), row-major pixel order."""
    c = np.asarray(mask) != 0
    H, W = c.shape
    N = H * W
    A = np.zeros((N, N))
    for y in range(H):
        for x in range(W):
            i = y * W + x
            if c[y, x]:
                A[i, i] = 1.0
                continue
            for dy, dx in ((0, -1), (0, 1), (-1, 0), (1, 0)):
                yy, xx = y + dy, x + dx
                if 0 <= yy < H and 0 <= xx < W:
                    A[i, i] += 1.0
                    A[i, yy * W + xx] -= 1.0
    return A


def solve_dense(f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Dense LU solve of ``A u = C f`` on the full pixel grid (small images only)."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    c = np.asarray(mask) != 0
    if not c.any():
        raise ValueError("empty mask: the inpainting system is singular")
    H, W = c.shape
    if H * W > 4096:
        raise ValueError("solve_dense is for images of at most 4096 pixels")
    A = dense_matrix(mask)
    out = np.empty_like(f)
    for ch in range(f.shape[0]):
        b = np.where(c, f[ch], 0.0).ravel()
        out[ch] = np.linalg.solve(A, b).reshape(H, W)
    return out


# ---------------------------------------------------------------------------
# Sections 3.1 and 4.4: geometry
# ---------------------------------------------------------------------------

def level_sizes(W: int, H: int, coarsest: int = 32) -> list[tuple[int, int]]:
    """Grid sizes finest to coarsest.

    Each level halves both sides (``ceil``, so a partial 2x2 cell keeps its
    existing children); the hierarchy stops at the first level whose sides are
    both at most ``coarsest``, i.e. a single ORAS block (Section 4.4).
    """
    sizes = [(W, H)]
    while sizes[-1][0] > coarsest or sizes[-1][1] > coarsest:
        w, h = sizes[-1]
        sizes.append(((w + 1) // 2, (h + 1) // 2))
    return sizes


def num_blocks(n: int, B: int, o: int) -> int:
    """Blocks along one axis of length ``n``: 1 if ``n <= B`` else ``ceil((n - o) / (B - o))``."""
    if n <= B:
        return 1
    s = B - o
    return -(-(n - o) // s)


def block_starts(n: int, B: int, o: int) -> list[tuple[int, int]]:
    """``(start, width)`` of the blocks along one axis.

    Blocks sit at stride ``B - o``, so neighbours share ``o`` pixels; the last
    block is clipped at the image edge (Section 3.1 gives 32x32 blocks with a
    6-pixel overlap).
    """
    nb = num_blocks(n, B, o)
    s = B - o
    return [(k * s, min(B, n - k * s)) for k in range(nb)]


def pou_weights_1d(n: int, B: int, o: int) -> list[np.ndarray]:
    """1-D partition-of-unity weights of every block along an axis of length ``n``.

    Inside an overlap of ``o`` pixels the weight falls linearly from 1 at the
    innermost pixel to 0 at the outermost one (Section 3.1 and its figure of
    the overlap weights); away
    from overlaps (and toward the image edge) it is 1.  Needs ``o >= 2``.
    """
    blocks = block_starts(n, B, o)
    nb = len(blocks)
    out = []
    for k, (s0, w) in enumerate(blocks):
        wt = np.ones(w)
        if nb > 1:
            j = np.arange(w, dtype=np.float64)
            if k > 0:
                left = j < o
                wt[left] = j[left] / (o - 1)
            if k < nb - 1:
                right = j >= w - o
                wt[right] = (w - 1 - j[right]) / (o - 1)
        out.append(wt)
    return out


def block_weight_2d(W: int, H: int, B: int, o: int, bx: int, by: int) -> np.ndarray:
    """Separable weight ``D_i`` of block (bx, by) as an array over that block."""
    return np.outer(pou_weights_1d(H, B, o)[by], pou_weights_1d(W, B, o)[bx])


# ---------------------------------------------------------------------------
# Section 4.3: coarse problems
# ---------------------------------------------------------------------------

def _children(Hf: int, Wf: int, Y: int, X: int):
    return [(y, x) for y in (2 * Y, 2 * Y + 1) for x in (2 * X, 2 * X + 1) if y < Hf and x < Wf]


def mask_down(c: np.ndarray) -> np.ndarray:
    """Coarse mask: a coarse pixel is known if any of its existing children is (max pooling)."""
    c = np.asarray(c) != 0
    Hf, Wf = c.shape
    Hc, Wc = (Hf + 1) // 2, (Wf + 1) // 2
    out = np.zeros((Hc, Wc), dtype=np.uint8)
    for Y in range(Hc):
        for X in range(Wc):
            out[Y, X] = 1 if any(c[y, x] for (y, x) in _children(Hf, Wf, Y, X)) else 0
    return out


def rhs_down_naive(c: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Naive coarse known values: mean of the known children, 0 if none (Section 4.3)."""
    c = np.asarray(c) != 0
    b = np.asarray(b, dtype=np.float64)
    Hf, Wf = c.shape
    Hc, Wc = (Hf + 1) // 2, (Wf + 1) // 2
    out = np.zeros((Hc, Wc))
    for Y in range(Hc):
        for X in range(Wc):
            ch = _children(Hf, Wf, Y, X)
            num = sum(b[y, x] for (y, x) in ch if c[y, x])
            den = sum(1 for (y, x) in ch if c[y, x])
            out[Y, X] = num / max(1, den)
    return out


def rhs_down_modified(c: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Modified coarse known values (Section 4.3, "Modified Mask Values Downsampling").

    Each known child ``j`` is weighted by the number of its direct neighbours
    that are not known.  A neighbour inside the same coarse cell is judged by
    the fine mask; a neighbour in an adjacent coarse cell is judged by that
    cell's coarse mask.  Neighbours outside the image are not counted.  The
    printed weights for three of the four children carry index typos; this
    follows the prose rule, which the one correct printed weight agrees
    with.  When every weight is 0 but some child is known, the naive mean is
    used so that a known coarse pixel never gets the value 0 by accident.
    """
    cf = np.asarray(c) != 0
    b = np.asarray(b, dtype=np.float64)
    Hf, Wf = cf.shape
    cc = mask_down(cf) != 0
    Hc, Wc = cc.shape
    naive = rhs_down_naive(cf, b)
    out = np.zeros((Hc, Wc))
    for Y in range(Hc):
        for X in range(Wc):
            num = 0.0
            den = 0.0
            for (y, x) in _children(Hf, Wf, Y, X):
                if not cf[y, x]:
                    continue
                free = 0
                for dy, dx in ((0, -1), (0, 1), (-1, 0), (1, 0)):
                    yy, xx = y + dy, x + dx
                    if not (0 <= yy < Hf and 0 <= xx < Wf):
                        continue
                    if yy // 2 == Y and xx // 2 == X:
                        known = cf[yy, xx]
                    else:
                        known = cc[yy // 2, xx // 2]
                    free += 0 if known else 1
                num += free * b[y, x]
                den += free
            if den > 0:
                out[Y, X] = num / den
            else:
                out[Y, X] = naive[Y, X]
    return out


def restrict_residual(r: np.ndarray, c_coarse: np.ndarray) -> np.ndarray:
    """Coarse right-hand side of the correction problem from a fine residual.

    The paper restricts by simple averaging away from mask pixels (Sections
    4.1 and 4.4) and keeps ``L`` scaled by ``1/h^2`` with ``H = 2h``.  Written
    with the integer stencil ``h^2 L`` on every level, the coarse right-hand
    side is ``H^2/h^2 = 4`` times the mean of the existing children.  It is 0
    at coarse mask pixels, where the coarse error is 0.  The factor is pinned
    by two-grid consistency: for a quadratic error the restricted fine
    residual equals the coarse residual of the same function.
    """
    r = np.asarray(r, dtype=np.float64)
    cc = np.asarray(c_coarse) != 0
    Hf, Wf = r.shape
    Hc, Wc = cc.shape
    out = np.zeros((Hc, Wc))
    for Y in range(Hc):
        for X in range(Wc):
            if cc[Y, X]:
                continue
            ch = _children(Hf, Wf, Y, X)
            out[Y, X] = 4.0 * sum(r[y, x] for (y, x) in ch) / len(ch)
    return out


def prolong_bilinear(uc: np.ndarray, Wf: int, Hf: int) -> np.ndarray:
    """Bilinear, cell-centred prolongation to a ``Hf x Wf`` grid (Section 4.4).

    Fine pixel i has its centre at coarse coordinate ``i/2 - 1/4``; it mixes the
    two nearest coarse cells per axis with weights 3/4 and 1/4, and a coarse
    index beyond the edge is clamped (reflecting boundary).
    """
    uc = np.asarray(uc, dtype=np.float64)
    Hc, Wc = uc.shape

    def axis(n_f: int, n_c: int):
        i = np.arange(n_f)
        near = i // 2
        far = np.where(i % 2 == 0, near - 1, near + 1)
        far = np.clip(far, 0, n_c - 1)
        return near, far

    ny, fy = axis(Hf, Hc)
    nx, fx = axis(Wf, Wc)
    out = (0.5625 * uc[ny][:, nx] + 0.1875 * uc[ny][:, fx]
           + 0.1875 * uc[fy][:, nx] + 0.0625 * uc[fy][:, fx])
    return out


# ---------------------------------------------------------------------------
# Section 3, Algorithm 2: one ORAS iteration with exact local solves
# ---------------------------------------------------------------------------

def oras_local_matrix(mask: np.ndarray, x0: int, y0: int, w: int, h: int, gamma: float):
    """Local matrix ``A_i`` of the block ``[y0, y0+h) x [x0, x0+w)``.

    Rows of known pixels are identity rows.  A row of an unknown pixel keeps
    ``-1`` for each neighbour inside the block; each neighbour inside the image
    adds 1 to the diagonal, except that a neighbour outside the block (an
    inner subdomain boundary) adds ``gamma`` instead: the Robin condition
    ``d_n v + alpha v = 0`` there, with ``gamma = 1`` the Dirichlet (RAS) case
    and ``gamma -> 0`` the Neumann one (Section 3, the mixed transmission
    condition of ORAS).  Neighbours outside
    the image add nothing (reflecting boundary).
    """
    c = np.asarray(mask) != 0
    H, W = c.shape
    n = w * h
    rows, cols, vals = [], [], []
    for ly in range(h):
        for lx in range(w):
            i = ly * w + lx
            y, x = y0 + ly, x0 + lx
            if c[y, x]:
                rows.append(i); cols.append(i); vals.append(1.0)
                continue
            d = 0.0
            for dy, dx in ((0, -1), (0, 1), (-1, 0), (1, 0)):
                yy, xx = y + dy, x + dx
                if not (0 <= yy < H and 0 <= xx < W):
                    continue
                lyy, lxx = ly + dy, lx + dx
                if 0 <= lyy < h and 0 <= lxx < w:
                    d += 1.0
                    rows.append(i); cols.append(lyy * w + lxx); vals.append(-1.0)
                else:
                    d += gamma
            rows.append(i); cols.append(i); vals.append(d)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def oras_step(u: np.ndarray, f: np.ndarray, mask: np.ndarray, B: int = 32, o: int = 6,
              gamma: float = 0.5) -> np.ndarray:
    """One discrete ORAS iteration (Algorithm 2) on the finest grid, one channel.

    1. ``r = b - A u``;  2. ``A_i v_i = R_i r`` for every block, solved
    exactly;  3. ``u + sum_i R_i^T D_i v_i``.  ``u`` must equal ``f`` at known
    pixels (the interpolation condition), so ``r`` and every ``v_i`` vanish
    there.
    """
    u = np.asarray(u, dtype=np.float64)
    H, W = u.shape
    r = residual(u, f, mask)
    xs, ys = block_starts(W, B, o), block_starts(H, B, o)
    wx, wy = pou_weights_1d(W, B, o), pou_weights_1d(H, B, o)
    out = u.copy()
    for by, (y0, h) in enumerate(ys):
        for bx, (x0, w) in enumerate(xs):
            Ai = oras_local_matrix(mask, x0, y0, w, h, gamma)
            ri = r[y0:y0 + h, x0:x0 + w].ravel()
            vi = spla.spsolve(Ai.tocsc(), ri).reshape(h, w)
            out[y0:y0 + h, x0:x0 + w] += np.outer(wy[by], wx[bx]) * vi
    return out
