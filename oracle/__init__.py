"""Plain FP64 CPU oracle for two-stage multisplitting (block Jacobi + inner CG).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares nothing with
the GPU library: the C source beside this file is compiled on its own by gcc
(``-O2 -fopenmp -ffp-contract=off``) and loaded with ctypes.

What each function follows in Brown, Bull and Bethune, "A highly scalable
approach to solving linear systems using two-stage multisplitting":

* ``apply`` / ``lift_bc`` / ``residual``: the 7-point Laplace stencil of
  Section 2.1 (diagonal 6, off-diagonal -1) with Dirichlet data moved into the
  right-hand side; the stopping quantity ``||Ax - b||_2`` of Section 2.1.
* ``block_jacobi``: Section 3's block formula
  ``X_i^(k) = A_ii^{-1}(B_i - sum_{j != i} A_ij X_j^(k-1))`` with the inverse
  replaced by at most m CG iterations (the two-stage inner solve of Section 2.3
  and the maximum inner iterations of Section 3.2), looped as in Listing 1
  (global residual test, inner solves, halo exchange).  The global residual is
  the root-sum-square of the block residuals (Section 3).
* ``block_sweep_some``: one synchronous sweep of the same method restricted to a
  list of blocks (per-block check at sizes too large for a whole-grid run).
* ``block_jacobi_async``: a bounded-delay model of the asynchronous outer
  iteration (Sections 2.1 and 2.3: blocks use the latest received, possibly
  old, neighbour values); deterministic for a given delay table.
* ``async_replay``: the asynchronous outer iteration replayed from a schedule
  of block sweeps, each naming the version of every neighbour block it reads
  (Section 2.3: the latest values received, of any age); reproduces a
  recorded asynchronous run exactly when the recorded reads are whole.
* ``cg``: the conventional global Krylov solver the paper compares against
  (Section 4), here CG.
* ``block_jacobi_ovl`` / ``ovl_sweep_some`` / ``overlap_cells``: overlapping
  blocks (the block overlap of Section 3.2 and the multisplitting weights of
  Section 2.3).  A block's region is its own cells plus slabs of depth o
  across each face that has a neighbour (the cells a face halo of depth o
  carries, giving the paper's o(2xy+2yz+2zx) extra unknowns); each block
  solves on its region and every cell takes its owner's new value.
* ``multisplit`` / ``multisplit_sweep_some``: the same synchronous method with
  any overlap and either inner solver: CG, or one GMRES(m) cycle (Sections
  3.1 and 4: the experiments' inner solver was GMRES), Arnoldi with classical
  Gram-Schmidt and Givens rotations, minimising the block residual over the
  Krylov space.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ms_oracle.c")

OK, ARG, NOT_CONVERGED, NONFINITE, DIVERGED = 0, 1, 4, 5, 6

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)


def lib_path(mutant: int = 0) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_mut{mutant}.so"
    return os.path.join(HERE, name)


SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]


def build(mutant: int = 0, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (mutant > 0 plants a known mistake;
    sanitize: AddressSanitizer + UndefinedBehaviorSanitizer build, loaded only
    by a process that preloads their runtimes)."""
    out = out or lib_path(mutant)
    tmp = out + f".tmp{os.getpid()}"
    opt = SANITIZE if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-std=c99", f"-DORACLE_MUTANT={int(mutant)}", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str):
        self.path = path
        L = C.CDLL(path)
        L.or_apply.argtypes = [C.c_long] * 3 + [_dp, _dp]
        L.or_apply.restype = None
        L.or_lift_bc.argtypes = [C.c_long] * 3 + [_dp] * 8
        L.or_lift_bc.restype = None
        L.or_residual.argtypes = [C.c_long] * 3 + [_dp, _dp, _dp]
        L.or_residual.restype = C.c_double
        L.or_block_jacobi.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                      [_dp, _dp, C.c_double, C.c_int, C.c_double,
                                       C.c_int, C.c_int, _dp, _ip, _lp])
        L.or_block_jacobi.restype = C.c_int
        L.or_block_sweep_some.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                          [_dp, _dp, C.c_int, _ip, C.c_int, C.c_double, _dp])
        L.or_block_sweep_some.restype = C.c_int
        L.or_block_jacobi_async.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                            [_dp, _dp, C.c_double, C.c_int, C.c_int,
                                             C.c_int, _ip, _dp, _ip])
        L.or_block_jacobi_async.restype = C.c_int
        L.or_cg.argtypes = [C.c_long] * 3 + [_dp, _dp, C.c_double, C.c_int, _dp, _ip]
        L.or_cg.restype = C.c_int
        L.or_overlap_cells.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                       [C.c_int, C.c_int])
        L.or_overlap_cells.restype = C.c_long
        L.or_block_jacobi_ovl.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                          [C.c_int, _dp, _dp, C.c_double, C.c_int, C.c_double,
                                           C.c_int, _dp, _ip, _lp])
        L.or_block_jacobi_ovl.restype = C.c_int
        L.or_ovl_sweep_some.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                        [C.c_int, _dp, _dp, C.c_int, _ip, C.c_int, C.c_double,
                                         _dp])
        L.or_ovl_sweep_some.restype = C.c_int
        L.or_multisplit.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                    [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_int,
                                     C.c_double, C.c_int, _dp, _ip, _lp])
        L.or_multisplit.restype = C.c_int
        L.or_multisplit_sweep_some.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                               [C.c_int, C.c_int, _dp, _dp, C.c_int, _ip,
                                                C.c_int, C.c_double, _dp])
        L.or_multisplit_sweep_some.restype = C.c_int
        L.or_async_replay.argtypes = ([C.c_long] * 3 + [C.c_int] * 3 + [_ip] * 3 +
                                      [_dp, _dp, C.c_int, C.c_int, C.c_int, _ip, _ip, _ip])
        L.or_async_replay.restype = C.c_int
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = C.c_int
        self.L = L

    def num_threads(self) -> int:
        return int(self.L.or_num_threads())

    # ---- helpers -----------------------------------------------------
    @staticmethod
    def _d(a):
        if a is None:
            return None
        assert a.dtype == np.float64 and a.flags.c_contiguous
        return a.ctypes.data_as(_dp)

    @staticmethod
    def _i(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        return a, a.ctypes.data_as(_ip)

    # ---- operator ----------------------------------------------------
    def apply(self, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        y = np.empty_like(u)
        nx, ny, nz = u.shape
        self.L.or_apply(nx, ny, nz, self._d(u), self._d(y))
        return y

    def lift_bc(self, b: np.ndarray | None, faces, shape=None) -> np.ndarray:
        """b_eff = b + boundary values; faces = 6 arrays (or None) -x,+x,-y,+y,-z,+z."""
        if b is not None:
            b = np.ascontiguousarray(b, dtype=np.float64)
            shape = b.shape
        nx, ny, nz = shape
        fs = [None if f is None else np.ascontiguousarray(f, dtype=np.float64)
              for f in (faces or [None] * 6)]
        want = [(ny, nz), (ny, nz), (nx, nz), (nx, nz), (nx, ny), (nx, ny)]
        for f, w in zip(fs, want):
            assert f is None or f.shape == w, (f.shape, w)
        out = np.empty((nx, ny, nz), dtype=np.float64)
        self.L.or_lift_bc(nx, ny, nz, self._d(b), *[self._d(f) for f in fs], self._d(out))
        return out

    def residual(self, beff: np.ndarray, x: np.ndarray, want_r: bool = False):
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        nx, ny, nz = x.shape
        r = np.empty_like(x) if want_r else None
        nrm = self.L.or_residual(nx, ny, nz, self._d(beff), self._d(x), self._d(r))
        return (nrm, r) if want_r else nrm

    # ---- solvers -----------------------------------------------------
    def block_jacobi(self, beff, x0, cuts, tol, m, inner_tol=0.0, max_sweeps=100000,
                     precision=0):
        """Synchronous block Jacobi with CG inner solves.

        Returns (status, x, sweeps, inner_iters, history)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, order="C", copy=True)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        hist = np.full(max_sweeps + 1, np.nan)
        sw = C.c_int(0); inn = C.c_long(0)
        st = self.L.or_block_jacobi(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                    pcx, pcy, pcz, self._d(beff), self._d(x), tol, m,
                                    inner_tol, max_sweeps, precision, self._d(hist),
                                    C.byref(sw), C.byref(inn))
        return st, x, sw.value, inn.value, hist[: sw.value + 1]

    def block_sweep_some(self, beff, x, cuts, blocks, m, inner_tol=0.0):
        """New values of the listed blocks after one sweep from x (others = x)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        bl, pbl = self._i(blocks)
        out = x.copy()
        st = self.L.or_block_sweep_some(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                        pcx, pcy, pcz, self._d(beff), self._d(x), len(bl),
                                        pbl, m, inner_tol, self._d(out))
        assert st == OK, st
        return out

    def overlap_cells(self, shape, cuts, overlap, block) -> int:
        """Cells in block `block`'s region for overlap `overlap`."""
        nx, ny, nz = shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        return int(self.L.or_overlap_cells(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                           pcx, pcy, pcz, int(overlap), int(block)))

    def block_jacobi_ovl(self, beff, x0, cuts, overlap, tol, m, inner_tol=0.0,
                         max_sweeps=100000):
        """Synchronous block Jacobi on overlapping regions (FP64).

        Returns (status, x, sweeps, inner_iters, history)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, order="C", copy=True)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        hist = np.full(max_sweeps + 1, np.nan)
        sw = C.c_int(0); inn = C.c_long(0)
        st = self.L.or_block_jacobi_ovl(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                        pcx, pcy, pcz, int(overlap), self._d(beff), self._d(x),
                                        tol, m, inner_tol, max_sweeps, self._d(hist),
                                        C.byref(sw), C.byref(inn))
        return st, x, sw.value, inn.value, hist[: sw.value + 1]

    def ovl_sweep_some(self, beff, x, cuts, overlap, blocks, m, inner_tol=0.0):
        """New owned values of the listed blocks after one overlapping sweep
        from x (other cells = x)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        bl, pbl = self._i(blocks)
        out = x.copy()
        st = self.L.or_ovl_sweep_some(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                      pcx, pcy, pcz, int(overlap), self._d(beff), self._d(x),
                                      len(bl), pbl, m, inner_tol, self._d(out))
        assert st == OK, st
        return out

    INNER = {"cg": 0, "gmres": 1}

    def multisplit(self, beff, x0, cuts, tol, m, overlap=0, inner="cg", inner_tol=0.0,
                   max_sweeps=100000):
        """Synchronous multisplitting, any overlap, CG or GMRES inner solves.

        Returns (status, x, sweeps, inner_iters, history)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, order="C", copy=True)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        hist = np.full(max_sweeps + 1, np.nan)
        sw = C.c_int(0); inn = C.c_long(0)
        st = self.L.or_multisplit(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                  pcx, pcy, pcz, int(overlap), self.INNER[inner], self._d(beff),
                                  self._d(x), tol, m, inner_tol, max_sweeps, self._d(hist),
                                  C.byref(sw), C.byref(inn))
        return st, x, sw.value, inn.value, hist[: sw.value + 1]

    def multisplit_sweep_some(self, beff, x, cuts, blocks, m, overlap=0, inner="cg",
                              inner_tol=0.0):
        """New owned values of the listed blocks after one sweep from x."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        bl, pbl = self._i(blocks)
        out = x.copy()
        st = self.L.or_multisplit_sweep_some(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                             pcx, pcy, pcz, int(overlap), self.INNER[inner],
                                             self._d(beff), self._d(x), len(bl), pbl, m,
                                             inner_tol, self._d(out))
        assert st == OK, st
        return out

    def block_jacobi_async(self, beff, x0, cuts, tol, m, max_sweeps, S, delays):
        """Bounded-delay asynchronous block Jacobi.  delays: int array
        [max_sweeps, nblocks, 6] or None.  Returns (status, x, sweeps, history)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, order="C", copy=True)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        nb = (len(cx) - 1) * (len(cy) - 1) * (len(cz) - 1)
        if delays is not None:
            delays = np.ascontiguousarray(delays, dtype=np.int32)
            assert delays.shape == (max_sweeps, nb, 6)
            pd = delays.ctypes.data_as(_ip)
        else:
            pd = None
        hist = np.full(max_sweeps + 1, np.nan)
        sw = C.c_int(0)
        st = self.L.or_block_jacobi_async(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                          pcx, pcy, pcz, self._d(beff), self._d(x), tol, m,
                                          max_sweeps, S, pd, self._d(hist), C.byref(sw))
        return st, x, sw.value, hist[: sw.value + 1]

    def async_replay(self, beff, x0, cuts, m, events, seen, precision=0):
        """Asynchronous block sweeps replayed from a schedule: event e sweeps
        block events[e] once from its own latest values, reading the
        neighbour across face f at that block's version seen[e, f].
        Returns (status, x, sweeps per block)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, order="C", copy=True)
        nx, ny, nz = x.shape
        cx, pcx = self._i(cuts[0]); cy, pcy = self._i(cuts[1]); cz, pcz = self._i(cuts[2])
        nb = (len(cx) - 1) * (len(cy) - 1) * (len(cz) - 1)
        ev, pev = self._i(events)
        sn, psn = self._i(np.asarray(seen).reshape(-1, 6))
        assert sn.shape == (len(ev), 6)
        sw, psw = self._i(np.zeros(nb))
        st = self.L.or_async_replay(nx, ny, nz, len(cx) - 1, len(cy) - 1, len(cz) - 1,
                                    pcx, pcy, pcz, self._d(beff), self._d(x), int(m),
                                    int(precision), len(ev), pev, psn, psw)
        return st, x, sw

    def cg(self, beff, x0, tol, max_iters=100000):
        """Global CG.  Returns (status, x, iters, history)."""
        beff = np.ascontiguousarray(beff, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, order="C", copy=True)
        nx, ny, nz = x.shape
        hist = np.full(max_iters + 1, np.nan)
        it = C.c_int(0)
        st = self.L.or_cg(nx, ny, nz, self._d(beff), self._d(x), tol, max_iters,
                          self._d(hist), C.byref(it))
        return st, x, it.value, hist[: it.value + 1]


_cache: dict[int, Oracle] = {}


def load(mutant: int = 0) -> Oracle:
    """Load (building first if no library is there) the oracle library."""
    if mutant not in _cache:
        p = lib_path(mutant)
        if not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(SRC):
            build(mutant)
        _cache[mutant] = Oracle(p)
    return _cache[mutant]
