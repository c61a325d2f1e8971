"""Seeded synthetic inputs for the 3D Laplace/Poisson workloads.

This module only draws and lays out input data (sources, boundary faces,
block cuts, delay tables).  It holds none of the solver's arithmetic, and it
is the one module that both the GPU tests and the CPU oracle's tests use.

Coordinates: interior point (i, j, k) of an nx*ny*nz grid on the unit cube
sits at ((i+1) h_x, (j+1) h_y, (k+1) h_z) with h_a = 1/(n_a + 1).  The six
boundary faces are ordered -x, +x, -y, +y, -z, +z; x faces are [ny][nz],
y faces [nx][nz], z faces [nx][ny].  The paper's experiments (Section 4) use
the 3D Laplace equation with Dirichlet boundaries on 50^3 points per core;
these generators stand in for its unpublished boundary data and sizes.
"""
from __future__ import annotations

import numpy as np


def spacing(n: int) -> float:
    return 1.0 / (n + 1)


def axis_coords(n: int) -> np.ndarray:
    """Interior coordinates (length n) and the two boundary coordinates."""
    h = spacing(n)
    return (np.arange(n, dtype=np.float64) + 1.0) * h


def face_shapes(nx: int, ny: int, nz: int):
    return [(ny, nz), (ny, nz), (nx, nz), (nx, nz), (nx, ny), (nx, ny)]


# --------------------------------------------------------------------------
# Harmonic cubic u = x^2 - y^2 + x y z (its Laplacian is zero, and the
# 7-point stencil reproduces it exactly when h_x == h_y).
# --------------------------------------------------------------------------

def harmonic_u(x, y, z):
    return x * x - y * y + x * y * z


def harmonic_faces(nx: int, ny: int, nz: int):
    """Dirichlet faces g = u on the boundary of the unit cube."""
    X, Y, Z = axis_coords(nx), axis_coords(ny), axis_coords(nz)
    f = []
    Yg, Zg = np.meshgrid(Y, Z, indexing="ij")
    f.append(harmonic_u(0.0, Yg, Zg))
    f.append(harmonic_u(1.0, Yg, Zg))
    Xg, Zg = np.meshgrid(X, Z, indexing="ij")
    f.append(harmonic_u(Xg, 0.0, Zg))
    f.append(harmonic_u(Xg, 1.0, Zg))
    Xg, Yg = np.meshgrid(X, Y, indexing="ij")
    f.append(harmonic_u(Xg, Yg, 0.0))
    f.append(harmonic_u(Xg, Yg, 1.0))
    return [np.ascontiguousarray(a, dtype=np.float64) for a in f]


def harmonic_interior(nx: int, ny: int, nz: int) -> np.ndarray:
    X, Y, Z = np.meshgrid(axis_coords(nx), axis_coords(ny), axis_coords(nz), indexing="ij")
    return np.ascontiguousarray(harmonic_u(X, Y, Z))


# --------------------------------------------------------------------------
# Sources (b = h^2 f for -lap u = f; the cube has one h when nx = ny = nz)
# --------------------------------------------------------------------------

def poisson_randn(shape, seed: int) -> np.ndarray:
    """b = h^2 f with f ~ N(0,1) i.i.d. per cell (h from the x axis)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(int(np.prod(shape))).reshape(shape)
    h = spacing(shape[0])
    return np.ascontiguousarray(h * h * f)


def gaussian_bumps(shape, seed_bumps: int, seed_noise: int, nbumps: int = 8,
                   sigma: float = 0.05, noise_std: float = 1e-3) -> np.ndarray:
    """b = h^2 f, f = sum of nbumps Gaussian bumps (centres U(0.1,0.9)^3,
    amplitudes U(-1,1), width sigma) plus N(0, noise_std) noise per cell.

    Built one x-slab at a time so a 512^3 grid needs no 3 GB temporaries."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed_bumps)
    centres = rng.uniform(0.1, 0.9, (nbumps, 3))
    amps = rng.uniform(-1.0, 1.0, nbumps)
    nrng = np.random.default_rng(seed_noise)
    X, Y, Z = axis_coords(nx), axis_coords(ny), axis_coords(nz)
    h = spacing(nx)
    out = np.empty(shape, dtype=np.float64)
    # separable Gaussians: exp(-|p-c|^2/2s^2) = gx(x) gy(y) gz(z)
    gxs = [np.exp(-(X - c[0]) ** 2 / (2 * sigma * sigma)) for c in centres]
    gys = [np.exp(-(Y - c[1]) ** 2 / (2 * sigma * sigma)) for c in centres]
    gzs = [np.exp(-(Z - c[2]) ** 2 / (2 * sigma * sigma)) for c in centres]
    yz = [np.multiply.outer(gy, gz) for gy, gz in zip(gys, gzs)]
    slab = 16
    for i0 in range(0, nx, slab):
        i1 = min(nx, i0 + slab)
        f = nrng.normal(0.0, noise_std, (i1 - i0) * ny * nz).reshape(i1 - i0, ny, nz)
        for a, gx, gyz in zip(amps, gxs, yz):
            f += a * gx[i0:i1, None, None] * gyz[None, :, :]
        out[i0:i1] = h * h * f
    return out


def smooth_field(shape, seed: int, kmax: int = 3) -> np.ndarray:
    """Seeded smooth target: sum over a,b,c <= kmax of N(0,1)/(a^2+b^2+c^2)
    sin(a pi x) sin(b pi y) sin(c pi z) on the interior points."""
    rng = np.random.default_rng(seed)
    X, Y, Z = (axis_coords(n) for n in shape)
    out = np.zeros(shape)
    for a in range(1, kmax + 1):
        for b in range(1, kmax + 1):
            for c in range(1, kmax + 1):
                w = rng.standard_normal() / (a * a + b * b + c * c)
                out += w * np.einsum("i,j,k->ijk", np.sin(a * np.pi * X), np.sin(b * np.pi * Y),
                                     np.sin(c * np.pi * Z))
    return out


def random_faces(nx: int, ny: int, nz: int, seed: int, lo=-1.0, hi=1.0):
    """Boundary data g ~ U(lo, hi) per face node, faces drawn in order."""
    rng = np.random.default_rng(seed)
    return [np.ascontiguousarray(rng.uniform(lo, hi, s)) for s in face_shapes(nx, ny, nz)]


# --------------------------------------------------------------------------
# Partitions
# --------------------------------------------------------------------------

def uniform_cuts(n: int, g: int) -> np.ndarray:
    if n % g:
        raise ValueError(f"{n} points do not split evenly into {g} blocks")
    return np.arange(0, n + 1, n // g, dtype=np.int32)


def uneven_cuts(n: int, seed: int, choices=(32, 48, 64, 96)) -> np.ndarray:
    """Cut an axis of n points into edges drawn from `choices` (seeded).
    Redraws rather than leave a remainder that no choice can fill."""
    rng = np.random.default_rng(seed)
    small = min(choices)
    for _ in range(10000):
        cuts = [0]
        while cuts[-1] < n:
            left = n - cuts[-1]
            if left in choices:
                cuts.append(n)
                break
            opts = [c for c in choices if c < left and (left - c >= small)]
            if not opts:
                break
            cuts.append(cuts[-1] + int(rng.choice(opts)))
        if cuts[-1] == n:
            return np.asarray(cuts, dtype=np.int32)
    raise ValueError(f"cannot cut {n} into {choices}")


def async_delays(max_sweeps: int, nblocks: int, S: int, seed: int) -> np.ndarray:
    """Delay table [sweep, block, face] with entries uniform in [0, S]."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, S + 1, size=(max_sweeps, nblocks, 6), dtype=np.int32)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def workload(name: str):
    """Return dict(shape, cuts, b, faces, m, tol) for a named workload.

    laplace32   32^3 Laplace, harmonic Dirichlet data, 2x2x2 blocks of 16^3, m=10
    poisson256  256^3 Poisson, f ~ N(0,1) seed 20, zero Dirichlet, 4^3 blocks of 64^3
    bumps512    512^3 Poisson, 8 Gaussian bumps (seed 30) + noise (seed 31),
                zero Dirichlet, 8^3 blocks of 64^3, m=10
    uneven384   384x320x448 Poisson, per-axis block edges drawn from
                {32, 48, 64, 96} (seeds 40, 41, 42), 16 right-hand sides
                f_k ~ N(0,1) (seed 400+k), zero Dirichlet; b is [16, nx, ny, nz]
    diff128     128^3, 4^3 blocks of 32^3: source f ~ N(0,1) (seed 50), faces
                g ~ U(-1,1) (seed 51), target u_t = smooth_field (seed 52);
                returns f (not h^2 f) under "f"; directions from diff_direction;
                adjoint_tol 1e-11: the adjoint solution is ~360x its right-hand
                side in norm, which puts its FP64 residual floor near 1e-12
    """
    if name == "laplace32":
        n = 32
        return dict(shape=(n, n, n), cuts=[uniform_cuts(n, 2)] * 3,
                    b=np.zeros((n, n, n)), faces=harmonic_faces(n, n, n), m=10, tol=1e-8)
    if name == "poisson256":
        n = 256
        return dict(shape=(n, n, n), cuts=[uniform_cuts(n, 4)] * 3,
                    b=poisson_randn((n, n, n), 20), faces=[None] * 6, m=10, tol=1e-8)
    if name == "bumps512":
        n = 512
        return dict(shape=(n, n, n), cuts=[uniform_cuts(n, 8)] * 3,
                    b=gaussian_bumps((n, n, n), 30, 31), faces=[None] * 6, m=10, tol=1e-8)
    if name.startswith("uneven384"):
        nrhs = int(name.split(":")[1]) if ":" in name else 16
        shape = (384, 320, 448)
        cuts = [uneven_cuts(n, 40 + a) for a, n in enumerate(shape)]
        b = np.empty((nrhs,) + shape)
        for k in range(nrhs):
            b[k] = poisson_randn(shape, 400 + k)
        return dict(shape=shape, cuts=cuts, b=b, faces=[None] * 6, m=10, tol=1e-8)
    if name == "diff128":
        n = 128
        rng = np.random.default_rng(50)
        return dict(shape=(n, n, n), cuts=[uniform_cuts(n, 4)] * 3,
                    f=rng.standard_normal((n, n, n)), faces=random_faces(n, n, n, 51),
                    ut=smooth_field((n, n, n), 52), m=10, tol=1e-13, adjoint_tol=1e-11)
    raise KeyError(name)


def diff_direction(shape, j: int):
    """Seeded direction j (seed 53 + j) in (source, faces) space for
    directional derivatives.  The source part is N(0,1) / h^2 per cell, so
    that the change it makes to the right-hand side h^2 f is N(0,1) per cell,
    like the face part (N(0,1) per face node).  Kinds by j mod 4: 0 and 2 both
    parts, 1 source only, 3 faces only."""
    rng = np.random.default_rng(53 + j)
    h = spacing(shape[0])
    df = rng.standard_normal(shape) / (h * h)
    dg = [rng.standard_normal(s) for s in face_shapes(*shape)]
    if j % 4 == 1:
        dg = [np.zeros_like(a) for a in dg]
    elif j % 4 == 3:
        df = np.zeros_like(df)
    return df, dg
