// HIP kernels of libms for gfx950: outer residual with in-memory halo reads,
// the two phases of the inner block CG, the fused final update, the
// persistent asynchronous sweep, the global CG baseline and the
// deterministic reductions behind every convergence test.
//
// Tiling.  Block-local work is cut into tiles of 256 threads.  A thread owns
// R consecutive rows (y) of VZ consecutive z cells of one block and marches
// along x over up to `tx` planes.  x neighbours come from a register
// pipeline (previous / current / next plane), y neighbours from the
// thread's own rows except the two rows bordering its group (loaded), and z
// neighbours from the adjacent lanes (shuffles; memory only at wavefront or
// block edges).  Loads are VZ wide (16 bytes when VZ*sizeof(T) = 16), so a
// wavefront reads whole contiguous z runs.
//
// Reductions.  A tile's partial sum is reduced across its wavefronts
// (lane shuffles, then LDS) and written to a per-tile slot.  Consumers add a
// block's tile slots in tile order, so every reduction has a fixed order and
// synchronous results are bitwise reproducible run to run.
#include "ms_internal.h"
#include "ms_device.h"
#include "ms_tiles.h"

#include <math.h>

#include <algorithm>

namespace ms {

// ----------------------------------------------------------------------
// synchronous phase kernels: one tile per workgroup
// ----------------------------------------------------------------------

template <typename T, int VZ, int R, bool STORE, bool OVL>
__global__ __launch_bounds__(kThreads) void k_resid(Geom g, int t0, long long goff,
                                                    const double *__restrict__ b,
                                                    const double *__restrict__ x, Faces F,
                                                    T *__restrict__ r, double *__restrict__ p64,
                                                    T *__restrict__ pT, const Ctrl *ctrl,
                                                    Batch bt) {
    // workgroup w of the launch: right-hand side k, tile t0 + (w mod nt)
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int kk = w / bt.nt;
    const int k = bt.k0 + kk;
    if (ctrl && ctrl[k].done) return;
    const int tile = t0 + (w - kk * bt.nt);
    if (b) b += k * bt.vs;
    if (x) x += k * bt.vs;
    if (r) r += k * bt.is;
    p64 += (long long)k * bt.ps;
    pT += (long long)k * bt.ps;
    const Tile t = decode_tile<VZ, R>(g, tile, threadIdx.x);
    double acc64 = 0.0;
    T accT = T(0);
    // 16-byte x accesses: loads requested a plane ahead (measured at 512^3
    // FP64: 53.5 -> 43.9 us per group launch).  Wider accesses already keep
    // more bytes in flight per load, and the lookahead's registers would cut
    // the waves per SIMD below what a launch supplies (measured mixed with
    // 4-cell vectors: 73.9 -> 85.6 us), so they keep the plain body.
    if constexpr (VZ <= 2)
        tile_resid_pf<T, VZ, R, STORE, OVL>(g, t, goff, b, x, F, r, acc64, accT);
    else
        tile_resid<T, VZ, R, STORE, OVL>(g, t, goff, b, x, F, r, acc64, accT);
    const double s64 = wg_allsum<double, kThreads>(acc64);
    // FP64 without overlap: the region and own sums coincide (pT == p64)
    if (sizeof(T) == sizeof(double) && !OVL) {
        if (threadIdx.x == 0) p64[tile] = s64;
    } else {
        const T sT = wg_allsum<T, kThreads>(accT);
        if (threadIdx.x == 0) { p64[tile] = s64; pT[tile] = sT; }
    }
}

template <typename T, int VZ, int R>
__global__ __launch_bounds__(kThreads) void k_stencil(Geom g, int t0, long long goff,
                                                      const T *__restrict__ r,
                                                      const T *__restrict__ pold,
                                                      T *__restrict__ pnew, T *__restrict__ psig,
                                                      const T *__restrict__ prho_cur,
                                                      const T *__restrict__ prho_prev,
                                                      const T *__restrict__ prho0,
                                                      int *active, int iter, double inner_tol,
                                                      Ctrl *ctrl, Batch bt) {
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int kk = w / bt.nt;
    const int k = bt.k0 + kk;
    if (ctrl[k].done) return;
    const int tile = t0 + (w - kk * bt.nt);
    r += k * bt.is;
    pold += k * bt.is;
    pnew += k * bt.is;
    psig += (long long)k * bt.ps;
    prho_cur += (long long)k * bt.ps;
    prho_prev += (long long)k * bt.ps;
    prho0 += (long long)k * bt.ps;
    active += (long long)k * bt.bs;
    const Tile t = decode_tile<VZ, R>(g, tile, threadIdx.x);
    const T rho = tiles_sum(prho_cur, t.B.tile0, t.B.ntiles);
    bool act;
    T beta = T(0);
    if (iter == 0) {
        act = rho > T(0);            // a block with zero residual has nothing to solve
        if (t.first && threadIdx.x == 0) active[t.b] = act ? 1 : 0;
    } else {
        act = active[t.b] != 0;
        if (act && inner_tol > 0.0) {
            const T rho0 = tiles_sum(prho0, t.B.tile0, t.B.ntiles);
            if (sqrt((double)rho) <= inner_tol * sqrt((double)rho0)) {
                act = false;
                if (t.first && threadIdx.x == 0) active[t.b] = 0;
            }
        }
        if (act) beta = rho / tiles_sum(prho_prev, t.B.tile0, t.B.ntiles);
    }
    if (!act) return;   // uniform over the workgroup
    const T acc = tile_stencil<T, VZ, R>(t, goff, r, pold, pnew, beta, iter > 0);
    const T s = wg_allsum<T, kThreads>(acc);
    if (threadIdx.x == 0) psig[tile] = s;
}

template <typename T, int VZ, int R, bool LAST, bool OVL>
__global__ __launch_bounds__(kThreads) void k_update(Geom g, int t0, long long goff,
                                                     T *__restrict__ r,
                                                     const T *__restrict__ p,
                                                     T *__restrict__ d,
                                                     const T *__restrict__ psig,
                                                     const T *__restrict__ prho_cur,
                                                     T *__restrict__ prho_next, int *active,
                                                     int iter, const double *__restrict__ xa,
                                                     double *__restrict__ xb, Ctrl *ctrl,
                                                     Batch bt) {
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int kk = w / bt.nt;
    const int k = bt.k0 + kk;
    ctrl += k;
    if (ctrl->done) return;
    const int tile = t0 + (w - kk * bt.nt);
    r += k * bt.is;
    p += k * bt.is;
    d += k * bt.is;
    psig += (long long)k * bt.ps;
    prho_cur += (long long)k * bt.ps;
    prho_next += (long long)k * bt.ps;
    active += (long long)k * bt.bs;
    if (LAST) {
        xa += k * bt.vs;
        xb += k * bt.vs;
    }
    const Tile t = decode_tile<VZ, R>(g, tile, threadIdx.x);
    bool act = active[t.b] != 0;
    T alpha = T(0);
    if (act) {
        const T sigma = tiles_sum(psig, t.B.tile0, t.B.ntiles);
        if (!(sigma > T(0))) {     // breakdown guard: stop this block's inner solve
            act = false;
            if (t.first && threadIdx.x == 0) active[t.b] = 0;
        } else {
            alpha = tiles_sum(prho_cur, t.B.tile0, t.B.ntiles) / sigma;
        }
    }
    if (act && t.first && threadIdx.x == 0) atomicAdd(&ctrl->inner_iters, 1ull);
    if (LAST) {
        // x_new = x_old + d + alpha p, for every block (inactive ones too);
        // x_new is a separate buffer, so every block's residual of this sweep
        // saw only x_old (Section 3: X_i^(k) from sweep k-1 values)
        tile_final<T, VZ, R, OVL>(g, t, goff, p, d, alpha, iter > 0, act, xa, xb);
        return;
    }
    if (!act) {
        // a block that stops before its first step keeps a zero correction
        if (iter == 0) {
            const int bz = t.B.bz;
            const long long P = (long long)t.B.by * bz;
            const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
            T z[VZ];
#pragma unroll
            for (int v = 0; v < VZ; v++) z[v] = T(0);
            for (int i = t.xbeg; i < t.xend; i++)
#pragma unroll
                for (int rr = 0; rr < R; rr++)
                    if (rr < t.nrows) vstore<T, VZ>(d + base + (long long)i * P + (long long)rr * bz, z);
        }
        return;
    }
    const T acc = tile_update<T, T, VZ, R, OVL>(t, goff, r, p, d, alpha, iter > 0);
    const T s = wg_allsum<T, kThreads>(acc);
    if (threadIdx.x == 0) prho_next[tile] = s;
}

// ----------------------------------------------------------------------
// global CG baseline (the conventional whole-system Krylov solve the paper
// compares against, Section 4): the grid is a single block and the scalars
// live on the device (scal[0] = rho, scal[1] = alpha, scal[2] = beta)
// ----------------------------------------------------------------------

template <int VZ, int R>
__global__ __launch_bounds__(kThreads) void k_gcg_stencil(Geom g, const double *__restrict__ r,
                                                          const double *__restrict__ pold,
                                                          double *__restrict__ pnew,
                                                          double *__restrict__ psig,
                                                          const double *scal, int iter,
                                                          const Ctrl *ctrl) {
    if (ctrl->done) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = decode_tile<VZ, R>(g, tile, threadIdx.x);
    const double beta = iter > 0 ? scal[2] : 0.0;
    const double acc = tile_stencil_pf<double, VZ, R>(t, 0, r, pold, pnew, beta, iter > 0);
    const double s = wg_allsum<double, kThreads>(acc);
    if (threadIdx.x == 0) psig[tile] = s;
}

template <int VZ, int R>
__global__ __launch_bounds__(kThreads) void k_gcg_update(Geom g, double *__restrict__ r,
                                                         const double *__restrict__ p,
                                                         double *__restrict__ x,
                                                         double *__restrict__ prho,
                                                         const double *scal, const Ctrl *ctrl) {
    if (ctrl->done) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = decode_tile<VZ, R>(g, tile, threadIdx.x);
    const double acc = tile_update_pf<double, double, VZ, R>(t, 0, r, p, x, scal[1], true);
    const double s = wg_allsum<double, kThreads>(acc);
    if (threadIdx.x == 0) prho[tile] = s;
}

__device__ double fixed_sum_1wg(const double *__restrict__ v, int n) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    for (int t = threadIdx.x; t < n; t += kThreads) s += v[t];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

// which: 0 after the initial residual, 1 after a stencil (alpha), 2 after an
// update (test on the recurrence residual, beta).
__global__ __launch_bounds__(kThreads) void k_gcg_reduce(const double *__restrict__ part,
                                                         int ntiles, int which, double tol,
                                                         int max_iters, double *history,
                                                         int history_cap, double *scal,
                                                         Ctrl *ctrl) {
    if (ctrl->done) return;
    const double total = fixed_sum_1wg(part, ntiles);
    if (threadIdx.x != 0) return;
    if (which == 1) {
        if (!(total > 0.0)) {                 // breakdown: the search direction vanished
            ctrl->status = 0;
            ctrl->final_sweep = ctrl->sweep;
            ctrl->done = 1;
        } else {
            scal[1] = scal[0] / total;
        }
        return;
    }
    const int it = which == 0 ? 0 : ctrl->sweep + 1;
    ctrl->sweep = it;
    const double res = sqrt(total) / ctrl->nbeff;
    if (it < history_cap) history[it] = res;
    ctrl->last_res = res;
    int status = -1;
    if (!isfinite(res)) status = 5;
    else if (tol > 0.0 && res <= tol) status = 0;
    else if (it >= max_iters) status = tol > 0.0 ? 4 : 0;
    if (status >= 0) {
        ctrl->status = status;
        ctrl->final_sweep = it;
        ctrl->done = 1;
        return;
    }
    if (which == 2) scal[2] = total / scal[0];
    scal[0] = total;
}

// ----------------------------------------------------------------------
// asynchronous outer iterations (Section 2.1: a block goes on with
// whatever halo values it has; Section 2.3 and Section 3: the next inner
// solve uses the latest neighbour values received).  A persistent
// workgroup works on one block at a time: it claims an eligible block,
// computes that block's residual from the x values in memory now
// (neighbour faces included), runs the inner CG, adds the correction to x
// in place, publishes the block's new version and moves on.  A block may
// start sweep v+1 only when every neighbour has finished at least v+1-S
// sweeps, which bounds how stale the neighbour data can be.  No workgroup
// ever waits for a particular block held by another, so progress does not
// depend on how many workgroups are resident.
// ----------------------------------------------------------------------

constexpr int kSub = kAsyncThreads / kThreads;

template <typename T, int VZ, int R, bool OVL>
__global__ __launch_bounds__(kAsyncThreads) void k_async(Geom g, const double *__restrict__ b,
                                                         double *x, Faces F, T *r, T *p0,
                                                         T *p1, T *d, AsyncState as, int m,
                                                         int S, int max_sweeps, double tol2,
                                                         double inner_tol, Ctrl *ctrl) {
    __shared__ AsyncShared sh;
    const int tid = threadIdx.x;
    const int sub = tid / kThreads;
    const int ltid = tid % kThreads;
    const int nb = g.nblocks;
    for (;;) {
        const int blk = async_claim<kAsyncThreads>(g, as, S, max_sweeps, ctrl, sh);
        if (blk == -2) return;                      // stop flag, or every block finished
        if (blk < 0) {                              // nothing eligible right now
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        // ---- one sweep of block blk ----
        const BlockInfo B = g.blocks[blk];
        double acc64 = 0.0;
        T accT = T(0);
        for (int lt = sub; lt < B.ntiles; lt += kSub) {
            const Tile t = decode_tile<VZ, R>(g, B.tile0 + lt, ltid);
            tile_resid<T, VZ, R, true, OVL>(g, t, 0, b, x, F, r, acc64, accT);
        }
        const double res2 = wg_allsum<double, kAsyncThreads>(acc64);
        T rho = wg_allsum<T, kAsyncThreads>(accT);
        const T rho0 = rho;
        if (tid == 0) __hip_atomic_store(&as.board[blk], res2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int iters = 0;          // inner iterations whose correction is in d
        bool applied = false;   // x already updated by the last iteration
        if (rho > T(0)) {
            T beta = T(0);
            for (int j = 0; j < m; j++) {
                T *pold = (j % 2) ? p0 : p1;
                T *pnew = (j % 2) ? p1 : p0;
                T acc = T(0);
                for (int lt = sub; lt < B.ntiles; lt += kSub) {
                    const Tile t = decode_tile<VZ, R>(g, B.tile0 + lt, ltid);
                    acc += tile_stencil<T, VZ, R>(t, 0, r, pold, pnew, beta, j > 0);
                }
                const T sigma = wg_allsum<T, kAsyncThreads>(acc);
                if (!(sigma > T(0))) break;          // breakdown guard
                const T alpha = rho / sigma;
                if (j == m - 1) {
                    for (int lt = sub; lt < B.ntiles; lt += kSub) {
                        const Tile t = decode_tile<VZ, R>(g, B.tile0 + lt, ltid);
                        tile_final<T, VZ, R, OVL>(g, t, 0, pnew, d, alpha, j > 0, true, x, x);
                    }
                    applied = true;
                    iters = m;
                    break;
                }
                acc = T(0);
                for (int lt = sub; lt < B.ntiles; lt += kSub) {
                    const Tile t = decode_tile<VZ, R>(g, B.tile0 + lt, ltid);
                    acc += tile_update<T, T, VZ, R, OVL>(t, 0, r, pnew, d, alpha, j > 0);
                }
                const T rho_new = wg_allsum<T, kAsyncThreads>(acc);
                iters = j + 1;
                if (inner_tol > 0.0 && sqrt((double)rho_new) <= inner_tol * sqrt((double)rho0)) break;
                beta = rho_new / rho;
                rho = rho_new;
            }
        }
        if (!applied && iters > 0) {
            for (int lt = sub; lt < B.ntiles; lt += kSub) {
                const Tile t = decode_tile<VZ, R>(g, B.tile0 + lt, ltid);
                tile_final<T, VZ, R, OVL>(g, t, 0, (const T *)nullptr, d, T(0), true, false, x, x);
            }
        }
        async_publish(as, blk, max_sweeps, iters, tol2, ctrl, sh, nb);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------
// global residual and convergence test (Section 3: global residual = root
// of the sum of squared block residuals; Listing 1: loop while it is above
// the threshold; Section 2.1: stop on ||Ax - b||)
// ----------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_check(const double *__restrict__ p64, int ntiles,
                                                    double tol, int final_check,
                                                    double *history, int history_cap,
                                                    Ctrl *ctrl, Batch bt) {
    // workgroup k checks right-hand side k
    const int k = blockIdx.x;
    ctrl += k;
    p64 += (long long)k * bt.ps;
    history += (long long)k * history_cap;
    if (ctrl->done) return;
    const double total = fixed_sum_1wg(p64, ntiles);
    if (threadIdx.x != 0) return;
    const int s = ctrl->sweep;
    const double res = sqrt(total) / ctrl->nbeff;
    if (s < history_cap) history[s] = res;
    ctrl->last_res = res;
    if (s == 0) ctrl->res0 = res;
    int status = -1;
    if (!isfinite(res)) status = 5;                               // MS_ERR_NONFINITE
    else if (tol > 0.0 && res <= tol) status = 0;                 // converged
    else if (ctrl->res0 > 0.0 && res > 1e6 * ctrl->res0) status = 6;  // MS_ERR_DIVERGED
    else if (final_check) status = tol > 0.0 ? 4 : 0;             // max sweeps reached
    if (status >= 0) {
        ctrl->status = status;
        ctrl->final_sweep = s;
        ctrl->done = 1;
    } else {
        ctrl->sweep = s + 1;
        ctrl->inner_snap = ctrl->inner_iters;
    }
}

__global__ __launch_bounds__(kThreads) void k_norm(const double *__restrict__ p64, int ntiles,
                                                   Ctrl *ctrl) {
    const double total = fixed_sum_1wg(p64, ntiles);
    if (threadIdx.x == 0) ctrl->nbeff = sqrt(total);
}

__global__ __launch_bounds__(kThreads) void k_sum(const double *__restrict__ v, int n,
                                                  double *out) {
    const double total = fixed_sum_1wg(v, n);
    if (threadIdx.x == 0) *out = total;
}

// y = A u, global grid, zero outside (Section 2.1 stencil).
__global__ __launch_bounds__(kThreads) void k_apply(long long nx, long long ny, long long nz,
                                                    const double *__restrict__ u,
                                                    double *__restrict__ y) {
    const long long n = nx * ny * nz;
    for (long long c = blockIdx.x * (long long)kThreads + threadIdx.x; c < n;
         c += (long long)gridDim.x * kThreads) {
        const long long k = c % nz, j = (c / nz) % ny, i = c / (ny * nz);
        double s = 6.0 * u[c];
        if (i > 0) s -= u[c - ny * nz];
        if (i < nx - 1) s -= u[c + ny * nz];
        if (j > 0) s -= u[c - nz];
        if (j < ny - 1) s -= u[c + nz];
        if (k > 0) s -= u[c - 1];
        if (k < nz - 1) s -= u[c + 1];
        y[c] = s;
    }
}

// Right-hand side assembly (Section 2.1: Dirichlet data moved to the
// right-hand side): out = s f + the boundary values next to each cell, added
// in the face order -x,+x,-y,+y,-z,+z as the residual tiles add them.
__global__ __launch_bounds__(kThreads) void k_lift(long long nx, long long ny, long long nz,
                                                   const double *__restrict__ f, double s,
                                                   Faces F, double *__restrict__ out) {
    const long long n = nx * ny * nz;
    for (long long c = blockIdx.x * (long long)kThreads + threadIdx.x; c < n;
         c += (long long)gridDim.x * kThreads) {
        const long long k = c % nz, j = (c / nz) % ny, i = c / (ny * nz);
        double v = s * f[c];
        if (i == 0 && F.f[0]) v += F.f[0][j * nz + k];
        if (i == nx - 1 && F.f[1]) v += F.f[1][j * nz + k];
        if (j == 0 && F.f[2]) v += F.f[2][i * nz + k];
        if (j == ny - 1 && F.f[3]) v += F.f[3][i * nz + k];
        if (k == 0 && F.f[4]) v += F.f[4][i * ny + j];
        if (k == nz - 1 && F.f[5]) v += F.f[5][i * ny + j];
        out[c] = v;
    }
}

// Transpose of k_lift: gf = s lam, and each requested face takes lam at the
// interior cells next to it (a face value enters exactly one cell's
// right-hand side, with weight 1).
__global__ __launch_bounds__(kThreads) void k_lift_adjoint(long long nx, long long ny,
                                                           long long nz,
                                                           const double *__restrict__ lam,
                                                           double s, double *__restrict__ gf) {
    const long long n = nx * ny * nz;
    for (long long c = blockIdx.x * (long long)kThreads + threadIdx.x; c < n;
         c += (long long)gridDim.x * kThreads)
        gf[c] = s * lam[c];
}

struct FaceOut {
    double *f[6];
};

__global__ __launch_bounds__(kThreads) void k_face_gather(long long nx, long long ny,
                                                          long long nz,
                                                          const double *__restrict__ lam,
                                                          FaceOut G) {
    const long long sz[6] = {ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny};
    for (int t = 0; t < 6; t++) {
        double *out = G.f[t];
        if (!out) continue;
        for (long long q = blockIdx.x * (long long)kThreads + threadIdx.x; q < sz[t];
             q += (long long)gridDim.x * kThreads) {
            long long c;
            if (t < 2) {          // q = j * nz + k on the plane i = 0 or nx - 1
                c = (t == 0 ? 0 : (nx - 1) * ny * nz) + q;
            } else if (t < 4) {   // q = i * nz + k on the plane j = 0 or ny - 1
                const long long i = q / nz, k = q % nz;
                c = (i * ny + (t == 2 ? 0 : ny - 1)) * nz + k;
            } else {              // q = i * ny + j on the plane k = 0 or nz - 1
                c = q * nz + (t == 4 ? 0 : nz - 1);
            }
            out[q] = lam[c];
        }
    }
}

// ----------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------

#define MS_CASE(vz_, r_, ...)                                         \
    case vz_ * 8 + r_: {                                              \
        constexpr int VZ = vz_, RR = r_;                              \
        __VA_ARGS__;                                                  \
        break;                                                        \
    }
// Synchronous phase kernels: z vectors of 1, 2, 4 or 8 cells (up to 32
// bytes per thread and row, split into 16-byte accesses).
#define MS_DISPATCH(vz, rows, ...)                                    \
    switch ((vz) * 8 + (rows)) {                                      \
        MS_CASE(1, 1, __VA_ARGS__) MS_CASE(1, 2, __VA_ARGS__) MS_CASE(1, 4, __VA_ARGS__) \
        MS_CASE(2, 1, __VA_ARGS__) MS_CASE(2, 2, __VA_ARGS__) MS_CASE(2, 4, __VA_ARGS__) \
        MS_CASE(4, 1, __VA_ARGS__) MS_CASE(4, 2, __VA_ARGS__) MS_CASE(4, 4, __VA_ARGS__) \
        MS_CASE(8, 1, __VA_ARGS__) MS_CASE(8, 2, __VA_ARGS__) MS_CASE(8, 4, __VA_ARGS__) \
        default: return hipErrorInvalidValue;                         \
    }
// The persistent asynchronous kernel: up to 4 cells.
#define MS_DISPATCH_A(vz, rows, ...)                                  \
    switch ((vz) * 8 + (rows)) {                                      \
        MS_CASE(1, 1, __VA_ARGS__) MS_CASE(1, 2, __VA_ARGS__) MS_CASE(1, 4, __VA_ARGS__) \
        MS_CASE(2, 1, __VA_ARGS__) MS_CASE(2, 2, __VA_ARGS__) MS_CASE(2, 4, __VA_ARGS__) \
        MS_CASE(4, 1, __VA_ARGS__) MS_CASE(4, 2, __VA_ARGS__) MS_CASE(4, 4, __VA_ARGS__) \
        default: return hipErrorInvalidValue;                         \
    }
// FP64 vectors use at most 16-byte accesses (VZ <= 2)
#define MS_DISPATCH64(vz, rows, ...)                                  \
    switch ((vz) * 8 + (rows)) {                                      \
        MS_CASE(1, 1, __VA_ARGS__) MS_CASE(1, 2, __VA_ARGS__) MS_CASE(1, 4, __VA_ARGS__) \
        MS_CASE(2, 1, __VA_ARGS__) MS_CASE(2, 2, __VA_ARGS__) MS_CASE(2, 4, __VA_ARGS__) \
        default: return hipErrorInvalidValue;                         \
    }

// Grid for tiles [t0, t1) of right-hand sides [k0, k0 + nk) of the batch.
inline dim3 batch_grid(int t0, int t1, Batch &bt) {
    bt.nt = t1 - t0;
    return dim3((unsigned)((long long)bt.nt * bt.nk));
}

template <typename T>
hipError_t launch_resid(const Geom &g, int vz, int t0, int t1, long long goff,
                        const double *b, const double *x, Faces faces, T *r, double *p64,
                        T *pT, const Ctrl *ctrl, Batch bt, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    const dim3 grid = batch_grid(t0, t1, bt);
#define MS_RESID(STORE, OVL)                                                               \
    MS_DISPATCH(vz, g.rows, launch((k_resid<T, VZ, RR, STORE, OVL>), grid,      \
                                               dim3(kThreads), 0, st, g, t0, goff, b, x,   \
                                               faces, r, p64, pT, ctrl, bt))
    if (r) {
        if (g.ovl) { MS_RESID(true, true); } else { MS_RESID(true, false); }
    } else {
        if (g.ovl) { MS_RESID(false, true); } else { MS_RESID(false, false); }
    }
#undef MS_RESID
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const Geom &g, int vz, int t0, int t1, long long goff,
                          const T *r, const T *p_old, T *p_new, T *psig, const T *prho_cur,
                          const T *prho_prev, const T *prho0, int *active, int iter,
                          double inner_tol, Ctrl *ctrl, Batch bt, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    const dim3 grid = batch_grid(t0, t1, bt);
    MS_DISPATCH(vz, g.rows, launch((k_stencil<T, VZ, RR>), grid,
                                               dim3(kThreads), 0, st, g, t0, goff, r, p_old,
                                               p_new, psig, prho_cur, prho_prev, prho0, active,
                                               iter, inner_tol, ctrl, bt));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const Geom &g, int vz, int t0, int t1, long long goff, T *r,
                         const T *p, T *d, const T *psig, const T *prho_cur, T *prho_next,
                         int *active, int iter, int last, const double *xa, double *xb,
                         Ctrl *ctrl, Batch bt, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    const dim3 grid = batch_grid(t0, t1, bt);
#define MS_UPDATE(LAST, OVL)                                                                \
    MS_DISPATCH(vz, g.rows, launch((k_update<T, VZ, RR, LAST, OVL>), grid,       \
                                               dim3(kThreads), 0, st, g, t0, goff, r, p, d, \
                                               psig, prho_cur, prho_next, active, iter, xa, \
                                               xb, ctrl, bt))
    if (last) {
        if (g.ovl) { MS_UPDATE(true, true); } else { MS_UPDATE(true, false); }
    } else {
        if (g.ovl) { MS_UPDATE(false, true); } else { MS_UPDATE(false, false); }
    }
#undef MS_UPDATE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_async(const Geom &g, int vz, int grid, const double *b, double *x, Faces faces,
                        T *r, T *p0, T *p1, T *d, AsyncState as, int m, int S, int max_sweeps,
                        double tol2, double inner_tol, Ctrl *ctrl, hipStream_t st) {
    if (grid < 1) return hipErrorInvalidValue;
    if (g.ovl) {
        MS_DISPATCH_A(vz, g.rows, launch((k_async<T, VZ, RR, true>), dim3(grid),
                                                     dim3(kAsyncThreads), 0, st, g, b, x, faces,
                                                     r, p0, p1, d, as, m, S, max_sweeps, tol2,
                                                     inner_tol, ctrl));
    } else {
        MS_DISPATCH_A(vz, g.rows, launch((k_async<T, VZ, RR, false>), dim3(grid),
                                                     dim3(kAsyncThreads), 0, st, g, b, x, faces,
                                                     r, p0, p1, d, as, m, S, max_sweeps, tol2,
                                                     inner_tol, ctrl));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t async_occupancy(int vz, int rows, int ovl, int *per_cu) {
    *per_cu = 0;
    if (ovl) {
        MS_DISPATCH_A(vz, rows, return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  per_cu, (const void *)k_async<T, VZ, RR, true>, kAsyncThreads, 0));
    } else {
        MS_DISPATCH_A(vz, rows, return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  per_cu, (const void *)k_async<T, VZ, RR, false>, kAsyncThreads, 0));
    }
    return hipSuccess;
}

hipError_t launch_gcg_stencil(const Geom &g, int vz, int ntiles, const double *r,
                              const double *pold, double *pnew, double *psig, const double *scal,
                              int iter, const Ctrl *ctrl, hipStream_t st) {
    MS_DISPATCH64(vz, g.rows, launch((k_gcg_stencil<VZ, RR>), dim3(ntiles),
                                                 dim3(kThreads), 0, st, g, r, pold, pnew, psig,
                                                 scal, iter, ctrl));
    return hipGetLastError();
}

hipError_t launch_gcg_update(const Geom &g, int vz, int ntiles, double *r, const double *p,
                             double *x, double *prho, const double *scal, const Ctrl *ctrl,
                             hipStream_t st) {
    MS_DISPATCH64(vz, g.rows, launch((k_gcg_update<VZ, RR>), dim3(ntiles),
                                                 dim3(kThreads), 0, st, g, r, p, x, prho, scal,
                                                 ctrl));
    return hipGetLastError();
}

hipError_t launch_gcg_reduce(const double *part, int ntiles, int which, double tol, int max_iters,
                             double *history, int history_cap, double *scal, Ctrl *ctrl,
                             hipStream_t st) {
    launch(k_gcg_reduce, dim3(1), dim3(kThreads), 0, st, part, ntiles, which, tol,
                       max_iters, history, history_cap, scal, ctrl);
    return hipGetLastError();
}

hipError_t launch_check(const double *p64, int ntiles, double tol, int final_check,
                        double *history, int history_cap, Ctrl *ctrl, Batch bt,
                        hipStream_t st) {
    launch(k_check, dim3(bt.nrhs), dim3(kThreads), 0, st, p64, ntiles, tol,
                       final_check, history, history_cap, ctrl, bt);
    return hipGetLastError();
}

hipError_t launch_norm(const double *p64, int ntiles, Ctrl *ctrl, hipStream_t st) {
    launch(k_norm, dim3(1), dim3(kThreads), 0, st, p64, ntiles, ctrl);
    return hipGetLastError();
}

hipError_t launch_sum(const double *v, int n, double *out, hipStream_t st) {
    launch(k_sum, dim3(1), dim3(kThreads), 0, st, v, n, out);
    return hipGetLastError();
}

static unsigned grid_for(long long n) {
    long long grid = (n + kThreads - 1) / kThreads;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    return (unsigned)grid;
}

hipError_t launch_lift(long long nx, long long ny, long long nz, const double *f, double s,
                       Faces F, double *out, hipStream_t st) {
    launch(k_lift, dim3(grid_for(nx * ny * nz)), dim3(kThreads), 0, st, nx, ny, nz, f, s, F, out);
    return hipGetLastError();
}

hipError_t launch_lift_adjoint(long long nx, long long ny, long long nz, const double *lam,
                               double s, double *gf, double *const gfaces[6], hipStream_t st) {
    if (gf) {
        launch(k_lift_adjoint, dim3(grid_for(nx * ny * nz)), dim3(kThreads), 0, st, nx, ny, nz,
               lam, s, gf);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    FaceOut G;
    bool any = false;
    for (int t = 0; t < 6; t++) {
        G.f[t] = gfaces[t];
        any = any || gfaces[t];
    }
    if (!any) return hipSuccess;
    const long long big = std::max(ny * nz, std::max(nx * nz, nx * ny));
    launch(k_face_gather, dim3(grid_for(big)), dim3(kThreads), 0, st, nx, ny, nz, lam, G);
    return hipGetLastError();
}

hipError_t launch_apply(long long nx, long long ny, long long nz, const double *u, double *y,
                        hipStream_t st) {
    const long long n = nx * ny * nz;
    long long grid = (n + kThreads - 1) / kThreads;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    launch(k_apply, dim3((unsigned)grid), dim3(kThreads), 0, st, nx, ny, nz, u, y);
    return hipGetLastError();
}

#define MS_INST(T)                                                                          \
    template hipError_t launch_resid<T>(const Geom &, int, int, int, long long, const double *, \
                                        const double *, Faces, T *, double *, T *,            \
                                        const Ctrl *, Batch, hipStream_t);                    \
    template hipError_t launch_stencil<T>(const Geom &, int, int, int, long long, const T *,  \
                                          const T *, T *, T *, const T *, const T *,          \
                                          const T *, int *, int, double, Ctrl *, Batch,       \
                                          hipStream_t);                                       \
    template hipError_t launch_update<T>(const Geom &, int, int, int, long long, T *,         \
                                         const T *, T *, const T *, const T *, T *, int *,    \
                                         int, int, const double *, double *, Ctrl *, Batch,   \
                                         hipStream_t);                                        \
    template hipError_t launch_async<T>(const Geom &, int, int, const double *, double *,     \
                                        Faces, T *, T *, T *, T *, AsyncState, int, int, int, \
                                        double, double, Ctrl *, hipStream_t);                 \
    template hipError_t async_occupancy<T>(int, int, int, int *);
MS_INST(double)
MS_INST(float)

}  // namespace ms
