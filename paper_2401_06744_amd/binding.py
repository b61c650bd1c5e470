"""ctypes binding of ``libinpaint.so`` (argument marshalling only).

Every function here has the name of the C entry point it calls (see
``include/inpaint.h``) and does no arithmetic of its own.  Arrays may be
numpy arrays (host memory) or torch CUDA tensors (device memory); the library
stages host buffers itself.  If the library has not been built the first
call raises ``RuntimeError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
from collections.abc import Mapping
import os
import threading

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libinpaint.so")
_lib = None
_lock = threading.Lock()

OK, NOT_CONVERGED, PENDING = 0, 1, 2
E_INVALID, E_EMPTY_MASK, E_NOMEM, E_DEVICE, E_DIVERGED = -1, -2, -3, -4, -5
KERNELS = ["stage", "pyramid", "block_solve", "update", "prolong", "restrict", "coarse",
           "residual", "output"]
SCHED_RFMG, SCHED_FMG, SCHED_MULTILEVEL, SCHED_SINGLE, SCHED_CG = 0, 1, 2, 3, 4
SCHED_CG_MULTILEVEL, SCHED_CG_MULTIGRID, SCHED_WARM = 5, 6, 7
RHS_MODIFIED, RHS_NAIVE = 0, 1
PREC_FP32, PREC_FP16, PREC_BF16 = 0, 1, 2

EXPORTED = [
    "inpaint_solve", "inpaint_solve_ex", "inpaint_rel_res", "inpaint_last_error",
    "inpaint_version", "inpaint_hierarchy_size", "inpaint_debug_pyramid",
    "inpaint_debug_oras_step", "inpaint_debug_restrict", "inpaint_debug_prolong",
    "inpaint_solve_batched", "inpaint_server_create", "inpaint_server_submit",
    "inpaint_server_poll", "inpaint_server_wait", "inpaint_server_destroy", "inpaint_autotune",
    "inpaint_cache_limit", "inpaint_solve_noalloc",
]
# device bytes of the fixed array behind inpaint_solve_noalloc (INPAINT_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 256 << 20


class InpaintOpts(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_int), ("block", ct.c_int), ("overlap", ct.c_int),
        ("gamma", ct.c_float), ("tau", ct.c_float), ("max_local_iters", ct.c_int),
        ("schedule", ct.c_int), ("max_cycles", ct.c_int), ("pre_smooth", ct.c_int),
        ("post_smooth", ct.c_int), ("rhs_restriction", ct.c_int), ("coarse_tau", ct.c_float),
        ("coarse_max_iters", ct.c_int), ("profile", ct.c_int), ("precision", ct.c_int),
    ]


class InpaintStats(ct.Structure):
    _fields_ = [
        ("rel_res", ct.c_double), ("cycles", ct.c_int), ("levels", ct.c_int),
        ("oras_iters", ct.c_int), ("local_cg_mean", ct.c_double), ("local_cg_max", ct.c_int),
        ("gpu_ms", ct.c_float), ("local_cg_finest", ct.c_double),
        ("finest_block_solves", ct.c_longlong), ("finest_cg_pixel_iters", ct.c_double),
        ("kernel_ms", ct.c_float * 9), ("kernel_calls", ct.c_int * 9),
        ("status", ct.c_int), ("t_submit_ms", ct.c_double), ("t_start_ms", ct.c_double),
        ("t_done_ms", ct.c_double),
    ]

    def as_dict(self) -> dict:
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k in ("kernel_ms", "kernel_calls") else v
        return d


class StatsView(Mapping):
    """Read-only mapping over one InpaintStats of a batch: fields are read from
    the C struct when asked for (a batch's statistics are not copied into 64
    dicts on every call)."""
    __slots__ = ("_s",)
    _names = tuple(k for k, _ in InpaintStats._fields_)

    def __init__(self, s: InpaintStats):
        self._s = s

    def __getitem__(self, k):
        if k not in self._names:
            raise KeyError(k)
        v = getattr(self._s, k)
        return list(v) if k in ("kernel_ms", "kernel_calls") else v

    def __iter__(self):
        return iter(self._names)

    def __len__(self):
        return len(self._names)


class InpaintProblem(ct.Structure):
    _fields_ = [("f", ct.c_void_p), ("mask", ct.c_void_p), ("W", ct.c_int), ("H", ct.c_int),
                ("channels", ct.c_int), ("out", ct.c_void_p)]


class InpaintServerCfg(ct.Structure):
    _fields_ = [("struct_size", ct.c_int), ("max_batch", ct.c_int), ("hbm_budget", ct.c_size_t),
                ("opts", InpaintOpts)]


class InpaintError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"inpaint error {code}: {msg}")
        self.code = code


def lib_path() -> str:
    return _LIB_PATH


def lib() -> ct.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"HIP library missing: {_LIB_PATH} (run __graft_entry__.build())")
        L = ct.CDLL(_LIB_PATH)
        vp, i, d, f32p = ct.c_void_p, ct.c_int, ct.c_double, ct.c_void_p
        L.inpaint_solve.argtypes = [vp, vp, i, i, i, d, vp]
        L.inpaint_solve_ex.argtypes = [vp, vp, i, i, i, d, vp, ct.POINTER(InpaintOpts), vp,
                                       ct.POINTER(InpaintStats)]
        L.inpaint_solve_noalloc.argtypes = [vp, vp, i, i, i, d, vp, ct.POINTER(InpaintOpts), vp,
                                             ct.POINTER(InpaintStats)]
        L.inpaint_rel_res.argtypes = [vp, vp, vp, i, i, i, vp]
        L.inpaint_last_error.restype = ct.c_char_p
        L.inpaint_version.restype = ct.c_char_p
        L.inpaint_hierarchy_size.argtypes = [i, i, i, ct.POINTER(ct.c_int), ct.POINTER(ct.c_size_t)]
        L.inpaint_debug_pyramid.argtypes = [vp, vp, i, i, i, i, i, ct.POINTER(ct.c_int), vp, vp, vp]
        L.inpaint_debug_oras_step.argtypes = [vp, vp, vp, i, i, i, ct.POINTER(InpaintOpts), vp]
        L.inpaint_debug_restrict.argtypes = [vp, vp, i, i, vp]
        L.inpaint_debug_prolong.argtypes = [vp, i, i, vp, vp, vp, i, vp]
        L.inpaint_solve_batched.argtypes = [ct.POINTER(InpaintProblem), i, d,
                                            ct.POINTER(InpaintOpts), vp, ct.POINTER(InpaintStats)]
        L.inpaint_autotune.argtypes = [ct.POINTER(InpaintProblem), i, d, ct.POINTER(InpaintOpts),
                                       vp, ct.POINTER(InpaintOpts), ct.POINTER(ct.c_double)]
        L.inpaint_server_create.argtypes = [ct.POINTER(InpaintServerCfg), ct.POINTER(vp)]
        L.inpaint_server_submit.argtypes = [vp, ct.POINTER(InpaintProblem), d,
                                            ct.POINTER(ct.c_uint64)]
        L.inpaint_server_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(InpaintStats)]
        L.inpaint_server_wait.argtypes = [vp, ct.c_uint64, ct.POINTER(InpaintStats)]
        L.inpaint_server_destroy.argtypes = [vp]
        L.inpaint_server_destroy.restype = None
        L.inpaint_cache_limit.argtypes = [ct.c_size_t, ct.POINTER(ct.c_size_t)]
        for name in EXPORTED:
            fn = getattr(L, name)
            if name != "inpaint_server_destroy" and (fn.restype is ct.c_int or fn.restype is None):
                fn.restype = ct.c_int
        L.inpaint_last_error.restype = ct.c_char_p
        L.inpaint_version.restype = ct.c_char_p
        _lib = L
        return L


# --------------------------------------------------------------------------- helpers

def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ct.c_void_p(x.data_ptr())
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return ct.c_void_p(x.ctypes.data)


def _shape(f):
    shp = tuple(f.shape)
    if len(shp) == 2:
        return 1, shp[0], shp[1]
    if len(shp) == 3:
        return shp
    raise ValueError("f must be [H][W] or [C][H][W]")


def _check(code: int) -> int:
    if code < 0:
        raise InpaintError(code, lib().inpaint_last_error().decode())
    return code


def make_opts(**kw) -> InpaintOpts:
    o = InpaintOpts()
    o.struct_size = ct.sizeof(InpaintOpts)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ct.c_void_p(stream)
    return ct.c_void_p(stream.cuda_stream)


def _empty_like(f):
    if _is_torch(f):
        import torch
        return torch.empty_like(f)
    return np.empty_like(f)


# --------------------------------------------------------------------------- entry points

def inpaint_solve(f, mask, tol: float = 1e-6, out=None):
    """Synchronous solve with default options; returns (out, status)."""
    C, H, W = _shape(f)
    out = _empty_like(f) if out is None else out
    st = _check(lib().inpaint_solve(_ptr(f), _ptr(mask), W, H, C, tol, _ptr(out)))
    return out, st


def inpaint_solve_ex(f, mask, tol: float = 1e-6, out=None, opts: InpaintOpts | None = None,
                     stream=None):
    """Solve with options on a stream; returns (out, status, stats dict)."""
    C, H, W = _shape(f)
    out = _empty_like(f) if out is None else out
    stats = InpaintStats()
    st = _check(lib().inpaint_solve_ex(_ptr(f), _ptr(mask), W, H, C, tol, _ptr(out),
                                       ct.byref(opts) if opts is not None else None,
                                       _stream_handle(stream), ct.byref(stats)))
    return out, st, stats.as_dict()


def inpaint_solve_noalloc(f, mask, tol: float = 1e-6, out=None, opts: InpaintOpts | None = None,
                          stream=None):
    """As inpaint_solve_ex, without device allocation in the library (device
    tensors only); returns (out, status, stats dict)."""
    C, H, W = _shape(f)
    out = _empty_like(f) if out is None else out
    stats = InpaintStats()
    st = _check(lib().inpaint_solve_noalloc(_ptr(f), _ptr(mask), W, H, C, tol, _ptr(out),
                                            ct.byref(opts) if opts is not None else None,
                                            _stream_handle(stream), ct.byref(stats)))
    return out, st, stats.as_dict()


def _problems(items):
    arr = (InpaintProblem * len(items))()
    outs = []
    for k, it in enumerate(items):
        f, mask = it[0], it[1]
        out = it[2] if len(it) > 2 and it[2] is not None else _empty_like(f)
        C, H, W = _shape(f)
        arr[k].f = _ptr(f)
        arr[k].mask = _ptr(mask)
        arr[k].W, arr[k].H, arr[k].channels = W, H, C
        arr[k].out = _ptr(out)
        outs.append(out)
    return arr, outs


def inpaint_solve_batched(problems, tol: float = 1e-6, opts: InpaintOpts | None = None,
                          stream=None, raise_on_error: bool = True):
    """Solve a list of (f, mask) or (f, mask, out) problems in one batch.

    Returns (outs, status, per-problem stats dicts).  With raise_on_error a
    negative status raises InpaintError; otherwise it is returned and each
    problem's own status is in its stats."""
    arr, outs = _problems(problems)
    stats = (InpaintStats * max(1, len(problems)))()
    st = lib().inpaint_solve_batched(arr, len(problems), tol,
                                     ct.byref(opts) if opts is not None else None,
                                     _stream_handle(stream), stats)
    if raise_on_error:
        _check(st)
    return outs, st, [StatsView(stats[k]) for k in range(len(problems))]


def inpaint_autotune(problems, tol: float = 1e-6, base: InpaintOpts | None = None, stream=None):
    """Tune the batched solve's options on these problems; returns (opts, ms per batch)."""
    arr, _ = _problems(problems)
    best = InpaintOpts()
    ms = ct.c_double(0.0)
    _check(lib().inpaint_autotune(arr, len(problems), tol, ct.byref(base) if base is not None else None,
                                  _stream_handle(stream), ct.byref(best), ct.byref(ms)))
    return best, ms.value


class ServerHandle:
    """A running server: the C handle plus references to the buffers of every
    uncollected ticket, so that they stay alive while the device uses them."""

    def __init__(self, handle):
        self.handle = handle
        self.buffers = {}


def inpaint_server_create(max_batch: int = 0, hbm_budget: int = 0,
                          opts: InpaintOpts | None = None) -> ServerHandle:
    cfg = InpaintServerCfg()
    cfg.struct_size = ct.sizeof(InpaintServerCfg)
    cfg.max_batch = max_batch
    cfg.hbm_budget = hbm_budget
    if opts is not None:
        cfg.opts = opts
    h = ct.c_void_p()
    _check(lib().inpaint_server_create(ct.byref(cfg), ct.byref(h)))
    return ServerHandle(h)


def inpaint_server_submit(srv: ServerHandle, f, mask, out=None, tol: float = 1e-6) -> int:
    """Queue (f, mask); returns the ticket.  The output buffer is returned by
    inpaint_server_wait / inpaint_server_poll."""
    arr, outs = _problems([(f, mask, out)])
    t = ct.c_uint64(0)
    _check(lib().inpaint_server_submit(srv.handle, arr, tol, ct.byref(t)))
    srv.buffers[t.value] = (f, mask, outs[0])
    return t.value


def _collect(srv: ServerHandle, ticket: int, fn, raise_on_error: bool):
    st = InpaintStats()
    code = fn(srv.handle, ticket, ct.byref(st))
    if code == PENDING:
        return None
    bufs = srv.buffers.pop(ticket, (None, None, None))
    if raise_on_error:
        _check(code)
    return bufs[2], code, st.as_dict()


def inpaint_server_poll(srv: ServerHandle, ticket: int, raise_on_error: bool = True):
    """None while the request runs, else (out, status, stats dict)."""
    return _collect(srv, ticket, lib().inpaint_server_poll, raise_on_error)


def inpaint_server_wait(srv: ServerHandle, ticket: int, raise_on_error: bool = True):
    """Block until the request has finished; returns (out, status, stats dict)."""
    return _collect(srv, ticket, lib().inpaint_server_wait, raise_on_error)


def inpaint_server_destroy(srv: ServerHandle) -> None:
    if srv.handle:
        lib().inpaint_server_destroy(srv.handle)
        srv.handle = None
        srv.buffers.clear()


def inpaint_rel_res(u, f, mask) -> np.ndarray:
    C, H, W = _shape(f)
    res = np.zeros(C, dtype=np.float64)
    _check(lib().inpaint_rel_res(_ptr(u), _ptr(f), _ptr(mask), W, H, C, _ptr(res)))
    return res


def inpaint_cache_limit(limit_bytes: int = 0) -> int:
    """Set the byte limit of the solves' workspace cache (0: keep it) and
    return the bytes still cached after trimming."""
    n = ct.c_size_t(0)
    _check(lib().inpaint_cache_limit(limit_bytes, ct.byref(n)))
    return n.value


def inpaint_last_error() -> str:
    return lib().inpaint_last_error().decode()


def inpaint_version() -> str:
    return lib().inpaint_version().decode()


def inpaint_hierarchy_size(W: int, H: int, block: int = 32):
    L = ct.c_int(0)
    n = ct.c_size_t(0)
    _check(lib().inpaint_hierarchy_size(W, H, block, ct.byref(L), ct.byref(n)))
    return L.value, n.value


def inpaint_debug_pyramid(f: np.ndarray, mask: np.ndarray, block: int = 32,
                          rhs_restriction: int = RHS_MODIFIED):
    """Returns a list of (mask_l [H_l][W_l] uint8, b_l [C][H_l][W_l] float32)."""
    C, H, W = _shape(f)
    f = np.ascontiguousarray(f, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nlev, npx = inpaint_hierarchy_size(W, H, block)
    masks = np.zeros(npx, dtype=np.uint8)
    rhs = np.zeros(npx * C, dtype=np.float32)
    sizes = np.zeros(2 * 24, dtype=np.int32)
    L = ct.c_int(0)
    _check(lib().inpaint_debug_pyramid(_ptr(f), _ptr(mask), W, H, C, block, rhs_restriction,
                                       ct.byref(L), _ptr(sizes), _ptr(masks), _ptr(rhs)))
    out, mo, ro = [], 0, 0
    for lvl in range(L.value):
        w, h = int(sizes[2 * lvl]), int(sizes[2 * lvl + 1])
        out.append((masks[mo:mo + w * h].reshape(h, w), rhs[ro:ro + C * w * h].reshape(C, h, w)))
        mo += w * h
        ro += C * w * h
    return out


def inpaint_debug_oras_step(u_in: np.ndarray, f: np.ndarray, mask: np.ndarray,
                            opts: InpaintOpts | None = None) -> np.ndarray:
    C, H, W = _shape(f)
    u_in = np.ascontiguousarray(u_in, dtype=np.float32)
    f = np.ascontiguousarray(f, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros_like(u_in)
    _check(lib().inpaint_debug_oras_step(_ptr(u_in), _ptr(f), _ptr(mask), W, H, C,
                                         ct.byref(opts) if opts is not None else None, _ptr(out)))
    return out


def inpaint_debug_restrict(r_f: np.ndarray, mask_c: np.ndarray) -> np.ndarray:
    Hf, Wf = r_f.shape
    r_f = np.ascontiguousarray(r_f, dtype=np.float32)
    mask_c = np.ascontiguousarray(mask_c, dtype=np.uint8)
    out = np.zeros(((Hf + 1) // 2, (Wf + 1) // 2), dtype=np.float32)
    _check(lib().inpaint_debug_restrict(_ptr(r_f), _ptr(mask_c), Wf, Hf, _ptr(out)))
    return out


def inpaint_debug_prolong(u_c: np.ndarray, mask_f: np.ndarray, b_f: np.ndarray,
                          u_in: np.ndarray | None = None, mode: int = 0) -> np.ndarray:
    Hf, Wf = mask_f.shape
    u_c = np.ascontiguousarray(u_c, dtype=np.float32)
    mask_f = np.ascontiguousarray(mask_f, dtype=np.uint8)
    b_f = np.ascontiguousarray(b_f, dtype=np.float32)
    u_in = None if u_in is None else np.ascontiguousarray(u_in, dtype=np.float32)
    out = np.zeros((Hf, Wf), dtype=np.float32)
    _check(lib().inpaint_debug_prolong(_ptr(u_c), Wf, Hf, _ptr(mask_f), _ptr(b_f), _ptr(u_in),
                                       mode, _ptr(out)))
    return out
