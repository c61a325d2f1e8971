"""Pins for the CPU oracle: facts fixed by the paper or by mathematics, each
computed WITHOUT the oracle's own code path (dense matrices built from
Kronecker sums, closed-form eigenpairs, the point-Jacobi update of Section
2.1, the block formula of Section 3 with dense inverses, exact solutions).

Each pin takes an oracle instance and raises AssertionError on failure, so
the same list can be run against planted-mistake builds of the oracle to show
that every planted mistake is caught by at least one pin.
"""
from __future__ import annotations

import numpy as np

from paper_2009_12638_amd import inputs


# ----------------------------------------------------------------------
# independent constructions
# ----------------------------------------------------------------------

def second_difference(n: int) -> np.ndarray:
    """1D Dirichlet second-difference matrix tridiag(-1, 2, -1), n x n."""
    T = 2.0 * np.eye(n)
    T -= np.eye(n, k=1)
    T -= np.eye(n, k=-1)
    return T


def dense_laplacian(nx: int, ny: int, nz: int) -> np.ndarray:
    """7-point operator as the Kronecker sum of 1D second differences; with
    z fastest in C order, the z factor is the last Kronecker factor."""
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(np.kron(second_difference(nx), Iy), Iz)
            + np.kron(np.kron(Ix, second_difference(ny)), Iz)
            + np.kron(np.kron(Ix, Iy), second_difference(nz)))


def block_index_sets(shape, cuts):
    """Flat index arrays of every block, in the library's block order."""
    nx, ny, nz = shape
    idx = np.arange(nx * ny * nz).reshape(shape)
    sets = []
    cx, cy, cz = cuts
    for a in range(len(cx) - 1):
        for b in range(len(cy) - 1):
            for c in range(len(cz) - 1):
                sets.append(idx[cx[a]:cx[a + 1], cy[b]:cy[b + 1], cz[c]:cz[c + 1]].ravel())
    return sets


def point_jacobi_sweep(x: np.ndarray, beff: np.ndarray) -> np.ndarray:
    """Section 2.1 update x_i <- (b_i - sum_{j != i} a_ij x_j) / a_ii for the
    7-point stencil: one sixth of (b + the six neighbours), zero outside."""
    xp = np.pad(x, 1)
    nb = (xp[2:, 1:-1, 1:-1] + xp[:-2, 1:-1, 1:-1] + xp[1:-1, 2:, 1:-1]
          + xp[1:-1, :-2, 1:-1] + xp[1:-1, 1:-1, 2:] + xp[1:-1, 1:-1, :-2])
    return (beff + nb) / 6.0


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ----------------------------------------------------------------------
# pins
# ----------------------------------------------------------------------

def pin_operator_dense(o):
    """Matrix-free apply equals the assembled Kronecker-sum matrix."""
    shape = (5, 4, 6)
    u = np.random.default_rng(1).standard_normal(shape)
    A = dense_laplacian(*shape)
    want = (A @ u.ravel()).reshape(shape)
    got = o.apply(u)
    assert np.max(np.abs(got - want)) <= 1e-13, np.max(np.abs(got - want))
    # symmetry x.Ay == y.Ax on the oracle's own apply
    v = np.random.default_rng(2).standard_normal(shape)
    assert abs(np.vdot(u, o.apply(v)) - np.vdot(v, o.apply(u))) < 1e-11


def pin_operator_eigen(o):
    """Closed-form eigenpairs: sin modes with eigenvalue
    sum over axes of 2 - 2 cos(a pi / (n + 1))."""
    shape = (7, 5, 9)
    for (a, b, c) in [(1, 1, 1), (3, 2, 5), (7, 5, 9)]:
        ix = np.sin(a * np.pi * (np.arange(shape[0]) + 1) / (shape[0] + 1))
        iy = np.sin(b * np.pi * (np.arange(shape[1]) + 1) / (shape[1] + 1))
        iz = np.sin(c * np.pi * (np.arange(shape[2]) + 1) / (shape[2] + 1))
        v = np.einsum("i,j,k->ijk", ix, iy, iz)
        lam = sum(2 - 2 * np.cos(t * np.pi / (n + 1)) for t, n in zip((a, b, c), shape))
        assert np.max(np.abs(o.apply(v) - lam * v)) < 1e-12


def pin_harmonic_lift(o):
    """u = x^2 - y^2 + xyz is reproduced exactly by the 7-point stencil when
    h_x = h_y, so A u_interior must equal b_eff from the boundary values."""
    shape = (7, 7, 9)
    u = inputs.harmonic_interior(*shape)
    beff = o.lift_bc(np.zeros(shape), inputs.harmonic_faces(*shape))
    err = np.max(np.abs(o.apply(u) - beff))
    assert err < 1e-13, err
    # and the residual of the exact solution is at rounding level
    assert o.residual(beff, u) / np.linalg.norm(beff) < 1e-14


def pin_residual_identity(o):
    """Residual norm equals ||b_eff - A x|| from the dense matrix."""
    shape = (4, 5, 3)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(shape)
    faces = inputs.random_faces(*shape, seed=4)
    beff = o.lift_bc(b, faces)
    # independent lifting: each boundary node value enters its neighbour once
    want_beff = b.copy()
    want_beff[0, :, :] += faces[0]
    want_beff[-1, :, :] += faces[1]
    want_beff[:, 0, :] += faces[2]
    want_beff[:, -1, :] += faces[3]
    want_beff[:, :, 0] += faces[4]
    want_beff[:, :, -1] += faces[5]
    assert np.max(np.abs(beff - want_beff)) < 1e-15
    x = rng.standard_normal(shape)
    want = np.linalg.norm(want_beff.ravel() - dense_laplacian(*shape) @ x.ravel())
    got = o.residual(beff, x)
    assert abs(got - want) <= 1e-12 * want


def pin_dense_fixed_point(o):
    """Block Jacobi + CG converges to the dense LU solution (uneven blocks)."""
    shape = (6, 6, 6)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(shape)
    faces = inputs.random_faces(*shape, seed=6)
    beff = o.lift_bc(b, faces)
    xstar = np.linalg.solve(dense_laplacian(*shape), beff.ravel()).reshape(shape)
    cuts = [np.array([0, 2, 6]), np.array([0, 3, 6]), np.array([0, 4, 6])]
    st, x, sw, _, hist = o.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-13, m=3,
                                        max_sweeps=3000)
    assert st == 0, st
    assert hist[-1] <= 1e-13
    assert rel(x, xstar) < 1e-11, rel(x, xstar)


def pin_point_jacobi(o):
    """1x1x1 blocks with one inner CG step are the point-Jacobi iteration of
    Section 2.1: one CG step on the 1x1 system 6 d = r gives d = r / 6."""
    shape = (6, 5, 4)
    rng = np.random.default_rng(7)
    beff = rng.standard_normal(shape)
    cuts = [np.arange(n + 1) for n in shape]
    K = 9
    st, x, sw, inner, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=1,
                                         max_sweeps=K)
    assert st == 0 and sw == K
    ref = np.zeros(shape)
    for _ in range(K):
        ref = point_jacobi_sweep(ref, beff)
    assert rel(x, ref) < 1e-14, rel(x, ref)


def pin_exact_block_jacobi(o):
    """2x2x2 blocks: A_ii has 4 distinct eigenvalues (3,5,7,9), so 4 CG
    steps solve each block exactly and the sweep is Section 3's
    X_i = A_ii^{-1}(B_i - sum_j A_ij X_j) with dense inverses."""
    shape = (4, 6, 4)
    rng = np.random.default_rng(8)
    beff = rng.standard_normal(shape)
    cuts = [np.arange(0, n + 1, 2) for n in shape]
    A = dense_laplacian(*shape)
    sets = block_index_sets(shape, cuts)
    K = 6
    st, x, sw, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=4, max_sweeps=K)
    assert st == 0 and sw == K
    xr = np.zeros(A.shape[0])
    bf = beff.ravel()
    for _ in range(K):
        xn = xr.copy()
        for S in sets:
            rhs = bf[S] - A[S] @ xr + A[np.ix_(S, S)] @ xr[S]
            xn[S] = np.linalg.solve(A[np.ix_(S, S)], rhs)
        xr = xn
    assert rel(x.ravel(), xr) < 1e-12, rel(x.ravel(), xr)


def pin_contraction_rate(o):
    """With exact block solves the residual contracts per sweep by the
    spectral radius of the block Jacobi iteration matrix I - M^{-1} A
    (Section 2.3: converges iff that radius is below 1)."""
    shape = (8, 8, 8)
    cuts = [np.array([0, 4, 8])] * 3
    A = dense_laplacian(*shape)
    M = np.zeros_like(A)
    for S in block_index_sets(shape, cuts):
        M[np.ix_(S, S)] = A[np.ix_(S, S)]
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - np.linalg.solve(M, A))))
    beff = np.random.default_rng(9).standard_normal(shape)
    st, x, sw, _, hist = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=40,
                                        max_sweeps=60)
    ratio = (hist[60] / hist[40]) ** (1.0 / 20)
    assert abs(ratio - rho) < 2e-3, (ratio, rho)
    assert rho < 1.0


def pin_cg_dense(o):
    """Global CG reaches the dense solution."""
    shape = (6, 5, 7)
    rng = np.random.default_rng(10)
    beff = rng.standard_normal(shape)
    xstar = np.linalg.solve(dense_laplacian(*shape), beff.ravel()).reshape(shape)
    st, x, it, hist = o.cg(beff, np.zeros(shape), tol=1e-14, max_iters=1000)
    assert st == 0
    assert rel(x, xstar) < 1e-12, rel(x, xstar)
    # finite termination: at most n distinct eigenvalues, far fewer than n here
    assert it <= 210


def pin_analytic_solution(o):
    """32^3 harmonic Laplace problem solved to 1e-12 reproduces u to 1e-10."""
    w = inputs.workload("laplace32")
    beff = o.lift_bc(w["b"], w["faces"])
    st, x, sw, _, hist = o.block_jacobi(beff, np.zeros(w["shape"]), w["cuts"], tol=1e-12,
                                        m=w["m"], max_sweeps=2000)
    assert st == 0
    u = inputs.harmonic_interior(*w["shape"])
    assert rel(x, u) <= 1e-10, rel(x, u)


def pin_async_zero_delay(o):
    """The bounded-delay model with every delay 0 is the synchronous method,
    and with delays up to S it still reaches the dense solution."""
    shape = (8, 8, 8)
    cuts = [np.array([0, 4, 8])] * 3
    rng = np.random.default_rng(11)
    beff = rng.standard_normal(shape)
    K = 12
    _, xs, _, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=5, max_sweeps=K)
    st, xa, sw, _ = o.block_jacobi_async(beff, np.zeros(shape), cuts, tol=0.0, m=5,
                                         max_sweeps=K, S=3, delays=np.zeros((K, 8, 6)))
    assert np.array_equal(xa, xs)
    xstar = np.linalg.solve(dense_laplacian(*shape), beff.ravel()).reshape(shape)
    D = inputs.async_delays(400, 8, 2, seed=12)
    st, xa, sw, hist = o.block_jacobi_async(beff, np.zeros(shape), cuts, tol=1e-12, m=5,
                                            max_sweeps=400, S=2, delays=D)
    assert st == 0, st
    assert rel(xa, xstar) < 1e-10


def pin_mixed_reference(o):
    """FP32 inner solves with FP64 residual/update refine to the FP64 answer."""
    shape = (16, 16, 16)
    cuts = [np.array([0, 8, 16])] * 3
    beff = inputs.poisson_randn(shape, 13)
    st64, x64, s64, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-8, m=10)
    st32, x32, s32, _, h32 = o.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-8, m=10,
                                            precision=1)
    assert st64 == 0 and st32 == 0
    assert h32[-1] <= 1e-8
    assert rel(x32, x64) < 1e-6, rel(x32, x64)


def pin_sweep_semantics(o):
    """tol <= 0 runs exactly max_sweeps; x = 0 when b_eff = 0; a tol above the
    starting residual returns at once with zero sweeps."""
    shape = (4, 4, 4)
    cuts = [np.array([0, 2, 4])] * 3
    beff = np.random.default_rng(14).standard_normal(shape)
    st, x, sw, inner, hist = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=2,
                                            max_sweeps=5)
    assert st == 0 and sw == 5 and len(hist) == 6
    assert inner == 5 * 8 * 2
    st, x, sw, _, _ = o.block_jacobi(np.zeros(shape), np.ones(shape), cuts, tol=1e-8, m=2)
    assert st == 0 and sw == 0 and not x.any()
    st, x, sw, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=2.0, m=2)
    assert st == 0 and sw == 0
    st, x, sw, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-30, m=2,
                                     max_sweeps=3)
    assert st == 4 and sw == 3


def pin_block_sweep_some(o):
    """Per-block sweep on listed blocks equals the same blocks of a full sweep."""
    shape = (8, 6, 10)
    cuts = [np.array([0, 3, 8]), np.array([0, 6]), np.array([0, 4, 10])]
    rng = np.random.default_rng(15)
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    _, x1, _, _, _ = o.block_jacobi(beff, x0, cuts, tol=0.0, m=4, max_sweeps=1)
    part = o.block_sweep_some(beff, x0, cuts, [1, 2], m=4)
    sets = block_index_sets(shape, cuts)
    for b in (1, 2):
        assert np.array_equal(part.ravel()[sets[b]], x1.ravel()[sets[b]])
    for b in (0, 3):
        assert np.array_equal(part.ravel()[sets[b]], x0.ravel()[sets[b]])


def pin_single_block_is_global_cg(o):
    """A partition into one block: one sweep of m inner iterations from x = 0
    is m iterations of the global Krylov solve (the same CG recurrences on
    the same operator and right-hand side, the conventional solver the paper
    compares against), bit for bit; a second sweep is CG restarted from the
    new residual."""
    shape = (7, 6, 9)
    rng = np.random.default_rng(21)
    beff = rng.standard_normal(shape)
    one = [np.array([0, n]) for n in shape]
    for m in (1, 5, 23):
        _, xb, sw, inner, _ = o.block_jacobi(beff, np.zeros(shape), one, tol=0.0, m=m,
                                             max_sweeps=1)
        st, xc, it, _ = o.cg(beff, np.zeros(shape), tol=0.0, max_iters=m)
        assert sw == 1 and inner == m and it == m
        assert np.array_equal(xb, xc), m


def _block_coords(cuts):
    """(bi, bj, bk) of every block in the library's block order."""
    gx, gy, gz = (len(c) - 1 for c in cuts)
    return [(a, b, c) for a in range(gx) for b in range(gy) for c in range(gz)]


def _face_neighbours(cuts):
    """nbr[i][f]: the block across face f (-x,+x,-y,+y,-z,+z) of block i, or -1."""
    g = [len(c) - 1 for c in cuts]
    coords = _block_coords(cuts)
    index = {c: n for n, c in enumerate(coords)}
    out = []
    for (a, b, c) in coords:
        row = []
        for ax, step in ((0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)):
            q = [a, b, c]
            q[ax] += step
            row.append(index[tuple(q)] if 0 <= q[ax] < g[ax] else -1)
        out.append(row)
    return out


def _steepest_step(Ab, r):
    """One CG step from 0 on Ab d = r in closed form: d = (r.r / r.Ab r) r."""
    rr = float(r @ r)
    if rr == 0.0:
        return np.zeros_like(r)
    return (rr / float(r @ (Ab @ r))) * r


def _delayed_reference(shape, cuts, beff, K, S, delays, block_solve):
    """Section 2.3's bounded-delay iteration written with dense matrices: in
    sweep s block i solves with its own sweep-s values and the values of the
    neighbour across face f from sweep s - min(delay, s)."""
    A = dense_laplacian(*shape)
    sets = block_index_sets(shape, cuts)
    nbr = _face_neighbours(cuts)
    bf = beff.ravel()
    X = [np.zeros(A.shape[0])]
    for s in range(K):
        xn = X[s].copy()
        for i, Si in enumerate(sets):
            rhs = bf[Si] - A[np.ix_(Si, Si)] @ X[s][Si]
            for f in range(6):
                j = nbr[i][f]
                if j < 0:
                    continue
                d = min(int(delays[s, i, f]), S, s)
                rhs = rhs - A[np.ix_(Si, sets[j])] @ X[s - d][sets[j]]
            xn[Si] = X[s][Si] + block_solve(A[np.ix_(Si, Si)], rhs)
        X.append(xn)
    return X[K].reshape(shape)


def pin_async_delay_table(o):
    """The bounded-delay model follows its delay table: with exact block
    solves (2x2x2 blocks, 4 CG steps) and with one CG step on 1x1x2 blocks
    (the closed-form steepest-descent step), K sweeps under seeded nonzero
    delays equal the dense iteration that reads each neighbour from the
    sweep its delay names; the synchronous iterate differs from both."""
    rng = np.random.default_rng(31)
    cases = [((4, 4, 2), [np.array([0, 2, 4]), np.array([0, 2, 4]), np.array([0, 2])], 4,
              lambda Ab, r: np.linalg.solve(Ab, r)),
             ((2, 2, 6), [np.array([0, 1, 2]), np.array([0, 1, 2]), np.array([0, 2, 4, 6])], 1,
              _steepest_step)]
    for shape, cuts, m, solve in cases:
        beff = rng.standard_normal(shape)
        nb = (len(cuts[0]) - 1) * (len(cuts[1]) - 1) * (len(cuts[2]) - 1)
        K, S = 9, 2
        D = rng.integers(0, S + 1, size=(K, nb, 6)).astype(np.int32)
        st, xa, sw, _ = o.block_jacobi_async(beff, np.zeros(shape), cuts, tol=0.0, m=m,
                                             max_sweeps=K, S=S, delays=D)
        assert st == 0 and sw == K
        want = _delayed_reference(shape, cuts, beff, K, S, D, solve)
        assert rel(xa, want) < 1e-12, rel(xa, want)
        _, xs, _, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=m, max_sweeps=K)
        assert rel(xs, want) > 1e-6, rel(xs, want)


def pin_fp32_inner_cg(o):
    """The FP32 inner stage (mixed precision) is CG: on 2x2x2 blocks four
    FP32 steps solve each block to single-precision accuracy (Section 3's
    block formula with dense inverses, in FP64), and on 4x4x4 blocks m FP32
    steps agree with m FP64 CG steps on the dense block to ~1e-6; FP32 and
    FP64 runs are not bitwise equal, so the FP32 path really ran."""
    rng = np.random.default_rng(32)
    shape = (4, 6, 4)
    cuts = [np.arange(0, n + 1, 2) for n in shape]
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    A = dense_laplacian(*shape)
    sets = block_index_sets(shape, cuts)
    bf, xr = beff.ravel(), x0.ravel()
    want = xr.copy()
    for S in sets:
        want[S] = np.linalg.solve(A[np.ix_(S, S)], bf[S] - A[S] @ xr + A[np.ix_(S, S)] @ xr[S])
    _, x32, _, _, _ = o.block_jacobi(beff, x0, cuts, tol=0.0, m=4, max_sweeps=1, precision=1)
    _, x64, _, _, _ = o.block_jacobi(beff, x0, cuts, tol=0.0, m=4, max_sweeps=1)
    e32 = rel(x32.ravel() - xr, want - xr)
    assert e32 < 2e-6, e32
    assert rel(x64.ravel() - xr, want - xr) < 1e-13
    assert not np.array_equal(x32, x64)
    # larger blocks, inexact: m FP32 CG steps against m FP64 CG steps on the
    # dense block (the textbook recurrences in NumPy)
    shape = (8, 4, 4)
    cuts = [np.array([0, 4, 8]), np.array([0, 4]), np.array([0, 4])]
    beff = rng.standard_normal(shape)
    A = dense_laplacian(*shape)
    m = 5
    want = np.zeros(A.shape[0])
    for S in block_index_sets(shape, cuts):
        Ab = A[np.ix_(S, S)]
        r = beff.ravel()[S].copy()
        d, p, rho = np.zeros_like(r), r.copy(), float(r @ r)
        for _ in range(m):
            q = Ab @ p
            a = rho / float(p @ q)
            d += a * p
            r -= a * q
            rn = float(r @ r)
            p = r + (rn / rho) * p
            rho = rn
        want[S] = d
    _, x32, _, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=m, max_sweeps=1,
                                     precision=1)
    assert rel(x32.ravel(), want) < 5e-6, rel(x32.ravel(), want)


def _replay_reference(shape, cuts, beff, x0, events, seen, block_solve):
    """A schedule of block sweeps written with dense matrices: event e solves
    block events[e] from its own latest values and the neighbour across face
    f at that block's version seen[e, f]."""
    A = dense_laplacian(*shape)
    sets = block_index_sets(shape, cuts)
    nbr = _face_neighbours(cuts)
    bf = beff.ravel()
    hist = [[x0.ravel()[S].copy()] for S in sets]
    for e, i in enumerate(events):
        Si = sets[i]
        own = hist[i][-1]
        rhs = bf[Si] - A[np.ix_(Si, Si)] @ own
        for f in range(6):
            j = nbr[i][f]
            if j >= 0:
                rhs = rhs - A[np.ix_(Si, sets[j])] @ hist[j][int(seen[e][f])]
        hist[i].append(own + block_solve(A[np.ix_(Si, Si)], rhs))
    x = np.zeros(A.shape[0])
    for S, h in zip(sets, hist):
        x[S] = h[-1]
    return x.reshape(shape), [len(h) - 1 for h in hist]


def _latest_schedule(nbr, order):
    """seen versions for an event order in which every sweep reads the
    neighbours' latest versions."""
    ver = [0] * len(nbr)
    seen = []
    for i in order:
        seen.append([ver[j] if j >= 0 else -1 for j in nbr[i]])
        ver[i] += 1
    return seen


def pin_async_replay(o):
    """The schedule replay: (i) lockstep sweeps that read version s of every
    neighbour are Section 3's block Jacobi with dense inverses (2x2x2 blocks,
    exact 4-step CG); (ii) red blocks then black blocks, each reading the
    latest values, is block Gauss-Seidel in red-black order (dense); (iii) a
    seeded random schedule with reads up to two versions old, one CG step on
    1x1x2 blocks (closed-form step) and on 2x2x2 blocks with exact solves,
    equals the dense replay; in FP32 (mixed precision) it agrees to ~1e-6."""
    rng = np.random.default_rng(33)
    shape = (4, 4, 4)
    cuts = [np.array([0, 2, 4])] * 3
    nb = 8
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    exact = lambda Ab, r: np.linalg.solve(Ab, r)   # noqa: E731
    # (i) lockstep = block Jacobi
    K = 5
    events = [b for s in range(K) for b in range(nb)]
    seen = [[s] * 6 for s in range(K) for b in range(nb)]
    st, x, sw = o.async_replay(beff, x0, cuts, 4, events, seen)
    assert st == 0 and list(sw) == [K] * nb
    A = dense_laplacian(*shape)
    sets = block_index_sets(shape, cuts)
    xr, bf = x0.ravel().copy(), beff.ravel()
    for _ in range(K):
        xn = xr.copy()
        for S in sets:
            xn[S] = np.linalg.solve(A[np.ix_(S, S)], bf[S] - A[S] @ xr + A[np.ix_(S, S)] @ xr[S])
        xr = xn
    assert rel(x.ravel(), xr) < 1e-12, rel(x.ravel(), xr)
    # (ii) red-black block Gauss-Seidel
    nbr = _face_neighbours(cuts)
    coords = _block_coords(cuts)
    red = [b for b, c in enumerate(coords) if sum(c) % 2 == 0]
    black = [b for b, c in enumerate(coords) if sum(c) % 2 == 1]
    order = [b for _ in range(K) for b in red + black]
    st, x, _ = o.async_replay(beff, x0, cuts, 4, order, _latest_schedule(nbr, order))
    assert st == 0
    xr = x0.ravel().copy()
    for _ in range(K):
        for colour in (red, black):
            for b in colour:
                S = sets[b]
                xr[S] = np.linalg.solve(A[np.ix_(S, S)],
                                        bf[S] - A[S] @ xr + A[np.ix_(S, S)] @ xr[S])
    assert rel(x.ravel(), xr) < 1e-12, rel(x.ravel(), xr)
    # (iii) random schedules with stale reads
    for shape, cuts, m, solve in (
            ((2, 2, 6), [np.array([0, 1, 2]), np.array([0, 1, 2]), np.array([0, 2, 4, 6])], 1,
             _steepest_step),
            ((4, 4, 4), [np.array([0, 2, 4])] * 3, 4, exact)):
        nbr = _face_neighbours(cuts)
        nb = len(nbr)
        beff = rng.standard_normal(shape)
        x0 = rng.standard_normal(shape)
        ver = [0] * nb
        events, seen = [], []
        for _ in range(12 * nb):
            i = int(rng.integers(nb))
            events.append(i)
            seen.append([max(0, ver[j] - int(rng.integers(3))) if j >= 0 else -1
                         for j in nbr[i]])
            ver[i] += 1
        st, x, sw = o.async_replay(beff, x0, cuts, m, events, seen)
        assert st == 0 and list(sw) == ver
        want, vers = _replay_reference(shape, cuts, beff, x0, events, seen, solve)
        assert vers == ver
        assert rel(x, want) < 1e-12, rel(x, want)
        latest, _ = _replay_reference(shape, cuts, beff, x0, events,
                                      _latest_schedule(nbr, events), solve)
        assert rel(latest, want) > 1e-6
        st, x32, _ = o.async_replay(beff, x0, cuts, m, events, seen, precision=1)
        assert st == 0 and rel(x32, want) < 1e-5, rel(x32, want)
    # a version that no earlier event produced
    st, _, _ = o.async_replay(beff, x0, cuts, 1, [0], [[1] * 6])
    assert st != 0


# ----------------------------------------------------------------------
# overlapping blocks (Section 3.2: block overlap; Section 2.3: weights D_i)
# ----------------------------------------------------------------------

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def region_index_sets(shape, cuts, overlap):
    """Brute-force regions: for each block, the flat indices of the cells that
    are inside the block, or outside it along exactly one axis by at most
    `overlap` (a face slab), and which of those the block owns."""
    nx, ny, nz = shape
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    out = []
    cx, cy, cz = cuts

    def dist(c, a, b):
        return np.where(c < a, a - c, np.where(c >= b, c - b + 1, 0))
    for a in range(len(cx) - 1):
        for b in range(len(cy) - 1):
            for c in range(len(cz) - 1):
                dx, dy, dz = dist(I, cx[a], cx[a + 1]), dist(J, cy[b], cy[b + 1]), dist(K, cz[c], cz[c + 1])
                nout = (dx > 0).astype(int) + (dy > 0) + (dz > 0)
                reg = (nout == 0) | ((nout == 1) & (dx + dy + dz <= overlap))
                own = nout == 0
                idx = np.flatnonzero(reg.ravel())
                out.append((idx, own.ravel()[idx]))
    return out


def pin_overlap_counts(o):
    """The paper's extra-unknown counts for 50^3 blocks with neighbours on
    all sides (golden file), a corner block's count o(xy+yz+zx), and the
    region sizes of a small uneven partition against brute force."""
    rows = [tuple(int(v) for v in ln.split()) for ln in open(f"{GOLDEN}/overlap_counts.txt")
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    cuts = [np.array([0, 50, 100, 150])] * 3
    for ov, extra in rows:
        assert o.overlap_cells((150, 150, 150), cuts, ov, 13) - 125000 == extra, (ov, extra)
        assert o.overlap_cells((150, 150, 150), cuts, ov, 0) - 125000 == ov * 3 * 2500
    shape = (9, 7, 8)
    cuts = [np.array([0, 2, 6, 9]), np.array([0, 4, 7]), np.array([0, 3, 8])]
    for ov in (0, 1, 2, 5):
        sets = region_index_sets(shape, cuts, ov)
        for b, (idx, _) in enumerate(sets):
            assert o.overlap_cells(shape, cuts, ov, b) == len(idx), (ov, b)


def pin_overlap_zero(o):
    """Overlap 0 is block Jacobi itself, bit for bit."""
    shape = (9, 7, 8)
    cuts = [np.array([0, 2, 6, 9]), np.array([0, 4, 7]), np.array([0, 3, 8])]
    rng = np.random.default_rng(16)
    beff = rng.standard_normal(shape)
    _, xa, sa, ia, ha = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=4, max_sweeps=7)
    _, xb, sb, ib, hb = o.block_jacobi_ovl(beff, np.zeros(shape), cuts, 0, tol=0.0, m=4,
                                           max_sweeps=7)
    assert np.array_equal(xa, xb) and sa == sb and ia == ib
    assert np.array_equal(ha, hb)


def _ras_step(A, bf, x, sets):
    """One restricted-weight sweep with exact region solves (dense)."""
    r = bf - A @ x
    xn = x.copy()
    for idx, own in sets:
        d = np.linalg.solve(A[np.ix_(idx, idx)], r[idx])
        xn[idx[own]] = x[idx[own]] + d[own]
    return xn


def pin_overlap_dense_step(o):
    """Sweeps with region solves run to convergence equal the dense
    multisplitting step x + sum_i D_i R_i^T A_RR^{-1} R_i (b - A x), D_i the
    indicator of block i's own cells (overlap 1 and 2, uneven blocks)."""
    shape = (6, 5, 7)
    cuts = [np.array([0, 3, 6]), np.array([0, 2, 5]), np.array([0, 4, 7])]
    A = dense_laplacian(*shape)
    rng = np.random.default_rng(17)
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    for ov in (1, 2):
        sets = region_index_sets(shape, cuts, ov)
        xr = x0.ravel().copy()
        for _ in range(3):
            xr = _ras_step(A, beff.ravel(), xr, sets)
        st, x, sw, _, _ = o.block_jacobi_ovl(beff, x0, cuts, ov, tol=0.0, m=300,
                                             inner_tol=1e-15, max_sweeps=3)
        assert st == 0 and sw == 3
        assert rel(x.ravel(), xr) < 1e-11, (ov, rel(x.ravel(), xr))


def pin_overlap_fixed_point(o):
    """Overlapping sweeps reach the dense solution."""
    shape = (8, 7, 6)
    cuts = [np.array([0, 3, 8]), np.array([0, 4, 7]), np.array([0, 2, 6])]
    rng = np.random.default_rng(18)
    beff = rng.standard_normal(shape)
    xstar = np.linalg.solve(dense_laplacian(*shape), beff.ravel()).reshape(shape)
    for ov in (1, 3):
        st, x, sw, _, _ = o.block_jacobi_ovl(beff, np.zeros(shape), cuts, ov, tol=1e-13, m=8,
                                             max_sweeps=3000)
        assert st == 0, st
        assert rel(x, xstar) < 1e-11, (ov, rel(x, xstar))


def pin_overlap_contraction(o):
    """With exact region solves the residual contracts per sweep by the
    spectral radius of the dense iteration matrix
    I - sum_i D_i R_i^T A_RR^{-1} R_i A, and overlap lowers that radius
    (the paper's observation that some overlap speeds convergence)."""
    shape = (8, 8, 8)
    cuts = [np.array([0, 4, 8])] * 3
    A = dense_laplacian(*shape)
    n = A.shape[0]
    beff = np.random.default_rng(19).standard_normal(shape)
    radii = {}
    for ov in (0, 1):
        B = np.zeros_like(A)
        for idx, own in region_index_sets(shape, cuts, ov):
            inv = np.linalg.inv(A[np.ix_(idx, idx)])
            B[np.ix_(idx[own], idx)] += inv[own]
        rho = np.max(np.abs(np.linalg.eigvals(np.eye(n) - B @ A)))
        st, x, sw, _, hist = o.block_jacobi_ovl(beff, np.zeros(shape), cuts, ov, tol=0.0, m=60,
                                                inner_tol=1e-15, max_sweeps=45)
        ratio = (hist[45] / hist[30]) ** (1.0 / 15)
        assert abs(ratio - rho) < 3e-3, (ov, ratio, rho)
        radii[ov] = rho
    assert radii[1] < radii[0] < 1.0, radii


def pin_ovl_sweep_some(o):
    """Per-block overlapping sweep equals the owned cells of a full sweep."""
    shape = (8, 6, 10)
    cuts = [np.array([0, 3, 8]), np.array([0, 6]), np.array([0, 4, 10])]
    rng = np.random.default_rng(20)
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    _, x1, _, _, _ = o.block_jacobi_ovl(beff, x0, cuts, 2, tol=0.0, m=4, max_sweeps=1)
    part = o.ovl_sweep_some(beff, x0, cuts, 2, [1, 2], m=4)
    sets = block_index_sets(shape, cuts)
    for b in (1, 2):
        assert np.array_equal(part.ravel()[sets[b]], x1.ravel()[sets[b]])
    for b in (0, 3):
        assert np.array_equal(part.ravel()[sets[b]], x0.ravel()[sets[b]])


# ----------------------------------------------------------------------
# GMRES inner solves (Sections 3.1 and 4: the paper's inner solver)
# ----------------------------------------------------------------------

def _krylov_min_residual(Ab, r, k):
    """argmin ||r - Ab d|| over span{r, Ab r, ..., Ab^{k-1} r}: orthonormal
    basis by QR of the power basis, then dense least squares."""
    K = np.empty((len(r), k))
    v = r.copy()
    for i in range(k):
        K[:, i] = v
        v = Ab @ v
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(Ab @ Q, r, rcond=None)
    return Q @ y


def pin_gmres_minimal_residual(o):
    """One sweep with GMRES(m) inner solves: every block's (or region's)
    correction minimises its residual over the Krylov space of dimension m
    (dense least squares), combined with the owner weights; overlap 0 and 1,
    uneven blocks."""
    shape = (6, 5, 7)
    cuts = [np.array([0, 3, 6]), np.array([0, 2, 5]), np.array([0, 4, 7])]
    A = dense_laplacian(*shape)
    rng = np.random.default_rng(22)
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    r = beff.ravel() - A @ x0.ravel()
    for ov in (0, 1):
        for m in (1, 3):
            want = x0.ravel().copy()
            for idx, own in region_index_sets(shape, cuts, ov):
                d = _krylov_min_residual(A[np.ix_(idx, idx)], r[idx], m)
                want[idx[own]] += d[own]
            st, x, sw, inner, _ = o.multisplit(beff, x0, cuts, tol=0.0, m=m, overlap=ov,
                                               inner="gmres", max_sweeps=1)
            assert st == 0 and sw == 1 and inner == 8 * m
            assert rel(x.ravel(), want) < 1e-11, (ov, m, rel(x.ravel(), want))


def pin_gmres_exact_block_jacobi(o):
    """2x2x2 blocks: A_ii has 4 distinct eigenvalues, so GMRES(4) solves each
    block exactly and the sweep is Section 3's block formula with dense
    inverses (the same pin as for CG)."""
    shape = (4, 6, 4)
    rng = np.random.default_rng(23)
    beff = rng.standard_normal(shape)
    cuts = [np.arange(0, n + 1, 2) for n in shape]
    A = dense_laplacian(*shape)
    sets = block_index_sets(shape, cuts)
    K = 5
    st, x, sw, _, _ = o.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=4, inner="gmres",
                                   max_sweeps=K)
    assert st == 0 and sw == K
    xr = np.zeros(A.shape[0])
    bf = beff.ravel()
    for _ in range(K):
        xn = xr.copy()
        for S in sets:
            rhs = bf[S] - A[S] @ xr + A[np.ix_(S, S)] @ xr[S]
            xn[S] = np.linalg.solve(A[np.ix_(S, S)], rhs)
        xr = xn
    assert rel(x.ravel(), xr) < 1e-12, rel(x.ravel(), xr)


def pin_gmres_fixed_point(o):
    """GMRES inner solves (with and without overlap) reach the dense solution;
    CG inner solves through the same driver are block_jacobi bit for bit."""
    shape = (8, 7, 6)
    cuts = [np.array([0, 3, 8]), np.array([0, 4, 7]), np.array([0, 2, 6])]
    rng = np.random.default_rng(24)
    beff = rng.standard_normal(shape)
    xstar = np.linalg.solve(dense_laplacian(*shape), beff.ravel()).reshape(shape)
    for ov in (0, 2):
        st, x, sw, _, _ = o.multisplit(beff, np.zeros(shape), cuts, tol=1e-13, m=6, overlap=ov,
                                       inner="gmres", max_sweeps=3000)
        assert st == 0, st
        assert rel(x, xstar) < 1e-11, (ov, rel(x, xstar))
    _, xa, _, _, _ = o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=4, max_sweeps=6)
    _, xb, _, _, _ = o.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=4, max_sweeps=6)
    assert np.array_equal(xa, xb)


def pin_gmres_sweep_some(o):
    """Per-block GMRES sweep equals the owned cells of a full sweep."""
    shape = (8, 6, 10)
    cuts = [np.array([0, 3, 8]), np.array([0, 6]), np.array([0, 4, 10])]
    rng = np.random.default_rng(25)
    beff = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    for ov in (0, 2):
        _, x1, _, _, _ = o.multisplit(beff, x0, cuts, tol=0.0, m=5, overlap=ov, inner="gmres",
                                      max_sweeps=1)
        part = o.multisplit_sweep_some(beff, x0, cuts, [0, 3], m=5, overlap=ov, inner="gmres")
        sets = block_index_sets(shape, cuts)
        for b in (0, 3):
            assert np.array_equal(part.ravel()[sets[b]], x1.ravel()[sets[b]])
        for b in (1, 2):
            assert np.array_equal(part.ravel()[sets[b]], x0.ravel()[sets[b]])


ALL_PINS = [
    pin_operator_dense,
    pin_operator_eigen,
    pin_harmonic_lift,
    pin_residual_identity,
    pin_dense_fixed_point,
    pin_point_jacobi,
    pin_exact_block_jacobi,
    pin_contraction_rate,
    pin_cg_dense,
    pin_analytic_solution,
    pin_async_zero_delay,
    pin_async_delay_table,
    pin_async_replay,
    pin_mixed_reference,
    pin_fp32_inner_cg,
    pin_sweep_semantics,
    pin_block_sweep_some,
    pin_single_block_is_global_cg,
    pin_overlap_counts,
    pin_overlap_zero,
    pin_overlap_dense_step,
    pin_overlap_fixed_point,
    pin_overlap_contraction,
    pin_ovl_sweep_some,
    pin_gmres_minimal_residual,
    pin_gmres_exact_block_jacobi,
    pin_gmres_fixed_point,
    pin_gmres_sweep_some,
]

# fast subset used against planted-mistake builds
FAST_PINS = [p for p in ALL_PINS if p is not pin_analytic_solution]
