"""ctypes binding of libms (include/ms.h) with the same entry-point names.

Argument marshalling only: every step of a solve runs in the HIP library.
Vectors are torch tensors on the GPU (float64, contiguous, 16-byte aligned);
PyTorch supplies device memory and the current HIP stream.  The library must
be built (``python -m paper_2009_12638_amd.build``); loading fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libms.so")

MS_OK, MS_ERR_ARG, MS_ERR_HIP, MS_ERR_NOMEM = 0, 1, 2, 3
MS_ERR_NOT_CONVERGED, MS_ERR_NONFINITE, MS_ERR_DIVERGED, MS_ERR_UNSUPPORTED = 4, 5, 6, 7
MS_SYNC, MS_ASYNC = 0, 1
MS_FP64, MS_MIXED = 0, 1
MS_INNER_CG, MS_INNER_GMRES = 0, 1
MS_ENGINE_AUTO, MS_ENGINE_PHASE, MS_ENGINE_TEAM = 0, 1, 2
ENGINES = {"auto": MS_ENGINE_AUTO, "phase": MS_ENGINE_PHASE, "team": MS_ENGINE_TEAM}
KERNEL_CLASSES = ["resid", "stencil", "update", "final", "check", "other", "orth", "hess"]


class MsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status
        self.msg = msg


class ms_grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64)]


class ms_blocks(C.Structure):
    _fields_ = [("gx", C.c_int32), ("gy", C.c_int32), ("gz", C.c_int32),
                ("cuts_x", C.POINTER(C.c_int32)), ("cuts_y", C.POINTER(C.c_int32)),
                ("cuts_z", C.POINTER(C.c_int32))]


class ms_bc(C.Structure):
    _fields_ = [("face", C.c_void_p * 6)]


class ms_opts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int32), ("inner_tol", C.c_double),
                ("staleness", C.c_int32), ("precision", C.c_int32),
                ("stream", C.c_void_p), ("check_every", C.c_int32),
                ("group_blocks", C.c_int32), ("x_chunk", C.c_int32),
                ("profile", C.c_int32), ("use_graph", C.c_int32), ("rows", C.c_int32),
                ("workers", C.c_int32), ("inner_solver", C.c_int32), ("z_vector", C.c_int32),
                ("slow_block", C.c_int32), ("slow_sleep", C.c_int32),
                ("trace", C.c_void_p), ("trace_cap", C.c_int32), ("engine", C.c_int32),
                ("team_spin", C.c_int32)]


class ms_stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("inner_iters", C.c_int64),
                ("rel_residual", C.c_double), ("seconds", C.c_double),
                ("max_staleness_seen", C.c_int32), ("relaunches", C.c_int32),
                ("history_len", C.c_int32), ("history", C.POINTER(C.c_double)),
                ("history_cap", C.c_int32), ("kernel_ms", C.c_double * 8),
                ("kernel_launches", C.c_int64 * 8), ("trace_len", C.c_int32),
                ("block_sweeps", C.POINTER(C.c_int32)), ("block_sweeps_cap", C.c_int32),
                ("engine_used", C.c_int32)]


_L = None


def lib() -> C.CDLL:
    """Open libms.so (raises if it has not been built)."""
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2009_12638_amd.build`")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        L.ms_default_opts.argtypes = [C.POINTER(ms_opts)]
        L.ms_default_opts.restype = None
        L.ms_create.argtypes = [C.POINTER(ms_grid), C.POINTER(ms_blocks), C.POINTER(ms_bc),
                                C.POINTER(H)]
        L.ms_create.restype = C.c_int
        L.ms_set_bc.argtypes = [H, C.POINTER(ms_bc)]
        L.ms_set_bc.restype = C.c_int
        L.ms_set_overlap.argtypes = [H, C.c_int32]
        L.ms_set_overlap.restype = C.c_int
        L.ms_reserve_krylov.argtypes = [H, C.c_int32]
        L.ms_reserve_krylov.restype = C.c_int
        L.ms_solve.argtypes = [H, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int,
                               C.POINTER(ms_opts), C.POINTER(ms_stats)]
        L.ms_solve.restype = C.c_int
        L.ms_residual.argtypes = [H, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.c_void_p]
        L.ms_residual.restype = C.c_int
        L.ms_residual_noalloc.argtypes = [H, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.c_void_p]
        L.ms_residual_noalloc.restype = C.c_int
        L.ms_lift.argtypes = [H, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.ms_lift.restype = C.c_int
        L.ms_lift_adjoint.argtypes = [H, C.c_void_p, C.c_double, C.c_void_p,
                                      C.POINTER(C.c_void_p), C.c_void_p]
        L.ms_lift_adjoint.restype = C.c_int
        L.ms_apply.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ms_apply.restype = C.c_int
        L.ms_cg.argtypes = [H, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                            C.POINTER(ms_opts), C.POINTER(ms_stats)]
        L.ms_cg.restype = C.c_int
        L.ms_reserve.argtypes = [H, C.c_int32]
        L.ms_reserve.restype = C.c_int
        L.ms_solve_batch.argtypes = [H, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                     C.c_int, C.POINTER(ms_opts), C.POINTER(ms_stats)]
        L.ms_solve_batch.restype = C.c_int
        L.ms_destroy.argtypes = [H]
        L.ms_destroy.restype = None
        L.ms_status_string.argtypes = [C.c_int]
        L.ms_status_string.restype = C.c_char_p
        L.ms_last_error.argtypes = [H]
        L.ms_last_error.restype = C.c_char_p
        L.ms_version.argtypes = []
        L.ms_version.restype = C.c_char_p
        _L = L
    return _L


def _status_name(s: int) -> str:
    try:
        return lib().ms_status_string(s).decode()
    except Exception:
        return f"status {s}"


def _ptr(t) -> int:
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return int(t)


def _vec(h, t, name):
    """Device pointer of a solver vector.  Torch tensors are checked here
    (dtype, device, contiguity, size): a caching allocator hands out pieces
    of larger allocations, which the library's own range check cannot tell
    apart from a whole buffer."""
    if t is None:
        raise MsError(MS_ERR_ARG, f"{name} is None")
    if hasattr(t, "data_ptr"):
        n = h.shape[0] * h.shape[1] * h.shape[2]
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() \
                or t.numel() != n:
            raise MsError(MS_ERR_ARG, f"{name} must be a contiguous float64 GPU tensor "
                                      f"of {n} elements")
        return t.data_ptr()
    return int(t)


def _stream(stream):
    if stream is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:
            return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return stream


class Handle:
    """Owns one ms_handle (plus the host cut arrays it was made from)."""

    def __init__(self, raw: C.c_void_p, shape, cuts, nblocks: int):
        self.raw = raw
        self.shape = tuple(shape)
        self.cuts = cuts
        self.nblocks = nblocks

    def __del__(self):
        try:
            ms_destroy(self)
        except Exception:
            pass


def _check(h, status: int):
    if status != MS_OK:
        msg = lib().ms_last_error(h.raw if isinstance(h, Handle) else h)
        raise MsError(status, (msg or b"").decode())


# ---------------------------------------------------------------------------
# entry points (same names as include/ms.h)
# ---------------------------------------------------------------------------

def ms_default_opts() -> ms_opts:
    o = ms_opts()
    lib().ms_default_opts(C.byref(o))
    return o


def ms_create(shape, blocks=None, cuts=None, faces=None) -> Handle:
    """shape = (nx, ny, nz); blocks = (gx, gy, gz) for a uniform split, or
    cuts = three integer sequences of block boundaries; faces = six device
    tensors (or None) in the order -x, +x, -y, +y, -z, +z."""
    nx, ny, nz = (int(v) for v in shape)
    g = ms_grid(nx, ny, nz)
    keep = []
    nblocks = 1
    if cuts is not None:
        arrs = []
        for c in cuts:
            a = (C.c_int32 * len(c))(*[int(v) for v in c])
            arrs.append(a)
        keep = arrs
        nblocks = (len(cuts[0]) - 1) * (len(cuts[1]) - 1) * (len(cuts[2]) - 1)
        bl = ms_blocks(len(cuts[0]) - 1, len(cuts[1]) - 1, len(cuts[2]) - 1,
                       C.cast(arrs[0], C.POINTER(C.c_int32)),
                       C.cast(arrs[1], C.POINTER(C.c_int32)),
                       C.cast(arrs[2], C.POINTER(C.c_int32)))
    else:
        gx, gy, gz = blocks
        nblocks = int(gx) * int(gy) * int(gz)
        bl = ms_blocks(gx, gy, gz, None, None, None)
    bc = ms_bc()
    for t, f in enumerate(faces or [None] * 6):
        bc.face[t] = _ptr(f)
    raw = C.c_void_p()
    st = lib().ms_create(C.byref(g), C.byref(bl), C.byref(bc), C.byref(raw))
    if st != MS_OK:
        raise MsError(st, (lib().ms_last_error(None) or b"").decode())
    return Handle(raw, (nx, ny, nz), keep, nblocks)


def ms_set_bc(h: Handle, faces) -> None:
    bc = ms_bc()
    for t, f in enumerate(faces or [None] * 6):
        bc.face[t] = _ptr(f)
    _check(h, lib().ms_set_bc(h.raw, C.byref(bc)))


def ms_set_overlap(h: Handle, overlap: int) -> None:
    """Overlap depth of the blocks' inner-solve regions (0: plain blocks)."""
    _check(h, lib().ms_set_overlap(h.raw, int(overlap)))


def ms_reserve_krylov(h: Handle, max_inner: int) -> None:
    """Allocate the GMRES basis for inner_iters up to max_inner (call again
    after ms_reserve / ms_set_overlap enlarge the handle)."""
    _check(h, lib().ms_reserve_krylov(h.raw, int(max_inner)))


@dataclass
class Stats:
    status: int
    sweeps: int
    inner_iters: int
    rel_residual: float
    seconds: float
    max_staleness_seen: int
    relaunches: int
    history: list = field(default_factory=list)
    kernel_ms: dict = field(default_factory=dict)
    kernel_launches: dict = field(default_factory=dict)
    trace_len: int = 0
    block_sweeps: list = field(default_factory=list)
    engine: str = ""


def _opts(precision="fp64", max_sweeps=100000, inner_tol=0.0, staleness=2, stream=None,
          check_every=0, group_blocks=0, x_chunk=0, profile=False, use_graph=True,
          rows=0, workers=0, inner="cg", z_vector=0, slow_block=-1, slow_sleep=0,
          trace=None, engine="auto", team_spin=0) -> ms_opts:
    o = ms_default_opts()
    o.max_sweeps = int(max_sweeps)
    o.inner_tol = float(inner_tol)
    o.staleness = int(staleness)
    o.precision = {"fp64": MS_FP64, "mixed": MS_MIXED}[precision] \
        if isinstance(precision, str) else int(precision)
    o.stream = _stream(stream)
    o.check_every = int(check_every)
    o.group_blocks = int(group_blocks)
    o.x_chunk = int(x_chunk)
    o.profile = 1 if profile else 0
    o.use_graph = 1 if use_graph else 0
    o.rows = int(rows)
    o.workers = int(workers)
    o.inner_solver = {"cg": MS_INNER_CG, "gmres": MS_INNER_GMRES}[inner] \
        if isinstance(inner, str) else int(inner)
    o.z_vector = int(z_vector)
    o.engine = ENGINES[engine] if isinstance(engine, str) else int(engine)
    o.team_spin = int(team_spin)
    o.slow_block = int(slow_block)
    o.slow_sleep = int(slow_sleep)
    if trace is not None:
        # an int32 device tensor of shape [cap, 8]
        o.trace = _ptr(trace)
        o.trace_cap = int(trace.shape[0]) if hasattr(trace, "shape") else 0
    return o


def _stats_of(st: int, s: ms_stats, hist, bsw=None) -> Stats:
    return Stats(status=st, sweeps=s.sweeps, inner_iters=s.inner_iters,
                 rel_residual=s.rel_residual, seconds=s.seconds,
                 max_staleness_seen=s.max_staleness_seen, relaunches=s.relaunches,
                 history=list(hist[: s.history_len]) if hist is not None else [],
                 kernel_ms={KERNEL_CLASSES[i]: s.kernel_ms[i] for i in range(8)},
                 kernel_launches={KERNEL_CLASSES[i]: s.kernel_launches[i] for i in range(8)},
                 trace_len=s.trace_len,
                 block_sweeps=list(bsw) if bsw is not None else [],
                 engine={1: "phase", 2: "team"}.get(s.engine_used, ""))


def _nblocks(h) -> int:
    return h.nblocks


def ms_solve(h: Handle, b, x, tol: float, inner_iters: int, mode="sync", history=0,
             raise_on_error=True, **opts) -> Stats:
    """Solve in place into x (see ms.h).  mode: "sync" | "async".  history:
    number of residual-history entries to return.  Other keywords fill
    ms_opts (precision="fp64"|"mixed", max_sweeps, inner_tol, staleness,
    stream, check_every, group_blocks, x_chunk, profile, use_graph)."""
    o = _opts(**opts)
    s = ms_stats()
    hist = None
    if history:
        hist = (C.c_double * int(history))()
        s.history = C.cast(hist, C.POINTER(C.c_double))
        s.history_cap = int(history)
    nb = _nblocks(h)
    bsw = (C.c_int32 * nb)()
    s.block_sweeps = C.cast(bsw, C.POINTER(C.c_int32))
    s.block_sweeps_cap = nb
    md = {"sync": MS_SYNC, "async": MS_ASYNC}[mode] if isinstance(mode, str) else int(mode)
    st = lib().ms_solve(h.raw, _vec(h, b, "b"), _vec(h, x, "x"), float(tol), int(inner_iters), md,
                        C.byref(o), C.byref(s))
    out = _stats_of(st, s, hist, bsw)
    if raise_on_error and st != MS_OK:
        _check(h, st)
    return out


def ms_reserve(h: Handle, nrhs: int) -> None:
    """Room for ms_solve_batch with up to nrhs right-hand sides."""
    _check(h, lib().ms_reserve(h.raw, int(nrhs)))


def _vecs(h, t, name, nrhs):
    if hasattr(t, "data_ptr"):
        import torch
        n = h.shape[0] * h.shape[1] * h.shape[2] * nrhs
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() \
                or t.numel() != n:
            raise MsError(MS_ERR_ARG, f"{name} must be a contiguous float64 GPU tensor "
                                      f"of {n} elements")
        return t.data_ptr()
    return int(t)


def ms_solve_batch(h: Handle, b, x, tol: float, inner_iters: int, history=0,
                   raise_on_error=True, **opts):
    """Solve every right-hand side of b ([nrhs, nx, ny, nz]) into x in the same
    launches (synchronous sweeps).  Returns a list of Stats."""
    nrhs = int(b.shape[0]) if hasattr(b, "shape") else int(opts.pop("nrhs"))
    o = _opts(**opts)
    arr = (ms_stats * nrhs)()
    hists = []
    for k in range(nrhs):
        if history:
            hk = (C.c_double * int(history))()
            arr[k].history = C.cast(hk, C.POINTER(C.c_double))
            arr[k].history_cap = int(history)
            hists.append(hk)
        else:
            hists.append(None)
    st = lib().ms_solve_batch(h.raw, nrhs, _vecs(h, b, "b", nrhs), _vecs(h, x, "x", nrhs),
                              float(tol), int(inner_iters), MS_SYNC, C.byref(o), arr)
    out = [_stats_of(st, arr[k], hists[k]) for k in range(nrhs)]
    if raise_on_error and st != MS_OK:
        _check(h, st)
    return out


def ms_residual(h: Handle, b, x, stream=None):
    """(relative, absolute) FP64 residual of x."""
    rel = C.c_double()
    ab = C.c_double()
    _check(h, lib().ms_residual(h.raw, _vec(h, b, "b"), _vec(h, x, "x"), C.byref(rel), C.byref(ab),
                                _stream(stream)))
    return rel.value, ab.value


def ms_residual_noalloc(h: Handle, b, x, stream=None):
    """(relative, absolute) FP64 residual of x, computed in the library's
    static scratch (no allocation, no handle work buffers)."""
    rel = C.c_double()
    ab = C.c_double()
    _check(h, lib().ms_residual_noalloc(h.raw, _vec(h, b, "b"), _vec(h, x, "x"), C.byref(rel),
                                        C.byref(ab), _stream(stream)))
    return rel.value, ab.value


def ms_lift(h: Handle, f, s: float, b_eff, stream=None) -> None:
    """b_eff = s * f + the handle's boundary values next to each cell."""
    _check(h, lib().ms_lift(h.raw, _vec(h, f, "f"), float(s), _vec(h, b_eff, "b_eff"),
                            _stream(stream)))


def _face_ptr(h, t, g):
    if g is None:
        return None
    if hasattr(g, "data_ptr"):
        import torch
        nx, ny, nz = h.shape
        want = [(ny, nz), (ny, nz), (nx, nz), (nx, nz), (nx, ny), (nx, ny)][t]
        if g.dtype != torch.float64 or not g.is_cuda or not g.is_contiguous() \
                or tuple(g.shape) != want:
            raise MsError(MS_ERR_ARG, f"face {t} must be a contiguous float64 GPU tensor "
                                      f"of shape {want}")
        return g.data_ptr()
    return int(g)


def ms_lift_adjoint(h: Handle, lam, s: float, grad_f=None, grad_faces=None, stream=None) -> None:
    """grad_f = s * lam; grad_faces[t] = lam at the cells next to face t
    (entries None are skipped)."""
    arr = None
    if grad_faces is not None:
        arr = (C.c_void_p * 6)(*[_face_ptr(h, t, g) for t, g in enumerate(grad_faces)])
    _check(h, lib().ms_lift_adjoint(h.raw, _vec(h, lam, "lambda"), float(s),
                                    None if grad_f is None else _vec(h, grad_f, "grad_f"),
                                    arr, _stream(stream)))


def ms_apply(h: Handle, u, y, stream=None) -> None:
    _check(h, lib().ms_apply(h.raw, _vec(h, u, "u"), _vec(h, y, "y"), _stream(stream)))


def ms_cg(h: Handle, b, x, tol: float, max_iters: int, history=0, raise_on_error=True,
          **opts) -> Stats:
    o = _opts(**opts)
    s = ms_stats()
    hist = None
    if history:
        hist = (C.c_double * int(history))()
        s.history = C.cast(hist, C.POINTER(C.c_double))
        s.history_cap = int(history)
    st = lib().ms_cg(h.raw, _vec(h, b, "b"), _vec(h, x, "x"), float(tol), int(max_iters), C.byref(o),
                     C.byref(s))
    out = _stats_of(st, s, hist)
    if raise_on_error and st != MS_OK:
        _check(h, st)
    return out


def ms_destroy(h: Handle) -> None:
    if h is not None and getattr(h, "raw", None):
        if _L is not None:
            _L.ms_destroy(h.raw)
        h.raw = None


def ms_status_string(s: int) -> str:
    return lib().ms_status_string(int(s)).decode()


def ms_last_error(h: Handle | None) -> str:
    return (lib().ms_last_error(h.raw if h is not None else None) or b"").decode()


def ms_version() -> str:
    return lib().ms_version().decode()
