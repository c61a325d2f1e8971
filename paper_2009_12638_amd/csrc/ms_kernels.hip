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

#include <math.h>

namespace ms {

// ----------------------------------------------------------------------
// tile bodies
// ----------------------------------------------------------------------

// Outer residual r = b_eff - A x on one tile (Section 3: the right-hand side
// B_i - sum_j A_ij X_j of a block, with neighbour-block values read straight
// from x: the halo exchange of Listing 1).  x == nullptr means x = 0.
// Adds r.r in FP64 to acc64 and in T to accT; stores r packed when STORE.
// OVL (overlap regions): r is zero outside the region; acc64 counts the
// block's own cells only (every cell of the grid once), accT the region.
template <typename T, int VZ, int R, bool STORE, bool OVL = false>
__device__ __forceinline__ void tile_resid(const Geom &g, const Tile &t, long long goff,
                                           const double *__restrict__ b, const double *x,
                                           const Faces &F, T *__restrict__ r, double &acc64,
                                           T &accT) {
    const long long nx = g.nx, ny = g.ny, nz = g.nz;
    const long long J0 = t.B.j0 + t.j0, K = t.B.k0 + t.k;
    const long long P = (long long)t.B.by * t.B.bz;
    auto gidx = [&](long long I, int rr) { return (I * ny + J0 + rr) * nz + K; };
    const bool zm_in = K > 0, zp_in = K + VZ < nz;        // z neighbour exists in the grid
    const bool zm_sh = t.zc > 0 && t.lane > 0;            // ... and sits in the lane to the left
    const bool zp_sh = t.zc < t.tpr - 1 && t.lane < 63;
    const bool ym_ld = t.nrows > 0 && J0 > 0;              // row above the group
    const bool yp_ld = t.nrows > 0 && J0 + t.nrows < ny;   // row below the group
    const bool ym_sh = t.j0 > 0 && t.lane >= t.tpr;         // ... held by a lane of this wave
    const bool yp_sh = t.j0 + t.nrows < t.B.by && t.lane + t.tpr < 64;
    double xm[R][VZ], xc[R][VZ], xp[R][VZ];
#pragma unroll
    for (int rr = 0; rr < R; rr++)
#pragma unroll
        for (int v = 0; v < VZ; v++) { xm[rr][v] = 0.0; xc[rr][v] = 0.0; xp[rr][v] = 0.0; }
    const long long I0 = t.B.i0 + t.xbeg;
    if (x) {
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            if (rr < t.nrows) {
                if (I0 > 0) vload<double, VZ>(x + gidx(I0 - 1, rr), xm[rr]);
                vload<double, VZ>(x + gidx(I0, rr), xc[rr]);
            }
        }
    }
    for (int i = t.xbeg; i < t.xend; i++) {
        const long long I = t.B.i0 + i;
        double ym[VZ], yp[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) { ym[v] = 0.0; yp[v] = 0.0; }
        // rows next to the group: from the neighbouring group tpr lanes away
        // when it is in this wavefront and in this block, else from memory
        double ysu[VZ], ysd[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            ysu[v] = __shfl_up(xc[R - 1][v], t.tpr, 64);
            ysd[v] = __shfl_down(xc[0][v], t.tpr, 64);
        }
        if (x) {
#pragma unroll
            for (int rr = 0; rr < R; rr++)
                if (rr < t.nrows && I + 1 < nx) vload<double, VZ>(x + gidx(I + 1, rr), xp[rr]);
            if (ym_ld) {
                if (ym_sh) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) ym[v] = ysu[v];
                } else {
                    vload<double, VZ>(x + gidx(I, -1), ym);
                }
            }
            if (yp_ld) {
                if (yp_sh) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) yp[v] = ysd[v];
                } else {
                    vload<double, VZ>(x + gidx(I, t.nrows), yp);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            const double sl = from_left(xc[rr][VZ - 1]);
            const double sr = from_right(xc[rr][0]);
            if (rr >= t.nrows) continue;
            const long long c = gidx(I, rr);
            double zm = 0.0, zp = 0.0;
            if (x && zm_in) zm = zm_sh ? sl : x[c - 1];
            if (x && zp_in) zp = zp_sh ? sr : x[c + VZ];
            double bb[VZ];
            if (b) {
                vload<double, VZ>(b + c, bb);
            } else {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[v] = 0.0;
            }
            const long long J = J0 + rr;
            // Dirichlet lifting: boundary neighbours' g moved to the right
            if (I == 0 && F.f[0]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[v] += F.f[0][J * nz + K + v];
            }
            if (I == nx - 1 && F.f[1]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[v] += F.f[1][J * nz + K + v];
            }
            if (J == 0 && F.f[2]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[v] += F.f[2][I * nz + K + v];
            }
            if (J == ny - 1 && F.f[3]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[v] += F.f[3][I * nz + K + v];
            }
            if (K == 0 && F.f[4]) bb[0] += F.f[4][I * ny + J];
            if (K + VZ == nz && F.f[5]) bb[VZ - 1] += F.f[5][I * ny + J];
            T out[VZ];
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const double left = v == 0 ? zm : xc[rr][v - 1];
                const double right = v == VZ - 1 ? zp : xc[rr][v + 1];
                const double up = rr == 0 ? ym[v] : xc[rr - 1][v];
                const double down = (rr == R - 1 || rr + 1 == t.nrows) ? yp[v] : xc[rr + 1][v];
                const double ax = 6.0 * xc[rr][v] - xm[rr][v] - xp[rr][v] - up - down - left - right;
                double rv = bb[v] - ax;
                if (OVL) {
                    const int n = axes_out(t.B, i, t.j0 + rr, t.k + v);
                    if (n > 1) rv = 0.0;
                    if (n == 0) acc64 += rv * rv;
                } else {
                    acc64 += rv * rv;
                }
                out[v] = (T)rv;
                accT += out[v] * out[v];
            }
            if (STORE)
                vstore<T, VZ>(r + (t.B.off - goff) + (long long)i * P +
                                  (long long)(t.j0 + rr) * t.B.bz + t.k, out);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int v = 0; v < VZ; v++) { xm[rr][v] = xc[rr][v]; xc[rr][v] = xp[rr][v]; xp[rr][v] = 0.0; }
    }
}

// Inner CG phase 1 on one tile (Section 3: the inner Krylov solve of a
// block on A_ii, here CG): p_new = r + beta p_old (p_new = r when !use_old),
// returns the thread's part of p_new . A_ii p_new (zero outside the block).
template <typename T, int VZ, int R>
__device__ __forceinline__ T tile_stencil(const Tile &t, long long goff,
                                          const T *__restrict__ r, const T *__restrict__ pold,
                                          T *__restrict__ pnew, T beta, bool use_old) {
    const int bz = t.B.bz, by = t.B.by, bx = t.B.bx;
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const bool zm_in = t.zc > 0, zp_in = t.zc < t.tpr - 1;
    const bool zm_sh = zm_in && t.lane > 0, zp_sh = zp_in && t.lane < 63;
    const bool ym_ld = t.nrows > 0 && t.j0 > 0;
    const bool yp_ld = t.nrows > 0 && t.j0 + t.nrows < by;
    const bool ym_sh = t.lane >= t.tpr, yp_sh = t.lane + t.tpr < 64;
    auto pv = [&](long long o, T(&out)[VZ]) {
        vload<T, VZ>(r + o, out);
        if (use_old) {
            T po[VZ];
            vload<T, VZ>(pold + o, po);
#pragma unroll
            for (int v = 0; v < VZ; v++) out[v] = out[v] + beta * po[v];
        }
    };
    auto ps = [&](long long o) -> T {
        T v = r[o];
        if (use_old) v = v + beta * pold[o];
        return v;
    };
    T pm[R][VZ], pc[R][VZ], pp[R][VZ];
#pragma unroll
    for (int rr = 0; rr < R; rr++)
#pragma unroll
        for (int v = 0; v < VZ; v++) { pm[rr][v] = T(0); pc[rr][v] = T(0); pp[rr][v] = T(0); }
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        if (rr < t.nrows) {
            if (t.xbeg > 0) pv(base + (long long)(t.xbeg - 1) * P + (long long)rr * bz, pm[rr]);
            pv(base + (long long)t.xbeg * P + (long long)rr * bz, pc[rr]);
        }
    }
    T acc = T(0);
    for (int i = t.xbeg; i < t.xend; i++) {
        const long long o = base + (long long)i * P;
        T ym[VZ], yp[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) { ym[v] = T(0); yp[v] = T(0); }
        T ysu[VZ], ysd[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            ysu[v] = __shfl_up(pc[R - 1][v], t.tpr, 64);
            ysd[v] = __shfl_down(pc[0][v], t.tpr, 64);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++)
            if (rr < t.nrows && i + 1 < bx) pv(o + P + (long long)rr * bz, pp[rr]);
        if (ym_ld) {
            if (ym_sh) {
#pragma unroll
                for (int v = 0; v < VZ; v++) ym[v] = ysu[v];
            } else {
                pv(o - bz, ym);
            }
        }
        if (yp_ld) {
            if (yp_sh) {
#pragma unroll
                for (int v = 0; v < VZ; v++) yp[v] = ysd[v];
            } else {
                pv(o + (long long)t.nrows * bz, yp);
            }
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            const T sl = from_left(pc[rr][VZ - 1]);
            const T sr = from_right(pc[rr][0]);
            if (rr >= t.nrows) continue;
            const long long orow = o + (long long)rr * bz;
            T zm = T(0), zp = T(0);
            if (zm_in) zm = zm_sh ? sl : ps(orow - 1);
            if (zp_in) zp = zp_sh ? sr : ps(orow + VZ);
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[rr][v - 1];
                const T right = v == VZ - 1 ? zp : pc[rr][v + 1];
                const T up = rr == 0 ? ym[v] : pc[rr - 1][v];
                const T down = (rr == R - 1 || rr + 1 == t.nrows) ? yp[v] : pc[rr + 1][v];
                const T q = T(6) * pc[rr][v] - pm[rr][v] - pp[rr][v] - up - down - left - right;
                acc += pc[rr][v] * q;
            }
            vstore<T, VZ>(pnew + orow, pc[rr]);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int v = 0; v < VZ; v++) { pm[rr][v] = pc[rr][v]; pc[rr][v] = pp[rr][v]; pp[rr][v] = T(0); }
    }
    return acc;
}

// Inner CG phase 2 on one tile: d += alpha p (d taken as 0 when !have_d);
// r -= alpha A_ii p; returns the thread's part of r.r.  OVL: A_ii p is taken
// as zero outside the region, so r (and d, p) stay zero there.
template <typename T, typename TD, int VZ, int R, bool OVL = false>
__device__ __forceinline__ T tile_update(const Tile &t, long long goff, T *__restrict__ r,
                                         const T *__restrict__ p, TD *__restrict__ d, T alpha,
                                         bool have_d) {
    const int bz = t.B.bz, by = t.B.by, bx = t.B.bx;
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const bool zm_in = t.zc > 0, zp_in = t.zc < t.tpr - 1;
    const bool zm_sh = zm_in && t.lane > 0, zp_sh = zp_in && t.lane < 63;
    const bool ym_ld = t.nrows > 0 && t.j0 > 0;
    const bool yp_ld = t.nrows > 0 && t.j0 + t.nrows < by;
    const bool ym_sh = t.lane >= t.tpr, yp_sh = t.lane + t.tpr < 64;
    T pm[R][VZ], pc[R][VZ], pp[R][VZ];
#pragma unroll
    for (int rr = 0; rr < R; rr++)
#pragma unroll
        for (int v = 0; v < VZ; v++) { pm[rr][v] = T(0); pc[rr][v] = T(0); pp[rr][v] = T(0); }
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        if (rr < t.nrows) {
            if (t.xbeg > 0) vload<T, VZ>(p + base + (long long)(t.xbeg - 1) * P + (long long)rr * bz, pm[rr]);
            vload<T, VZ>(p + base + (long long)t.xbeg * P + (long long)rr * bz, pc[rr]);
        }
    }
    T acc = T(0);
    for (int i = t.xbeg; i < t.xend; i++) {
        const long long o = base + (long long)i * P;
        T ym[VZ], yp[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) { ym[v] = T(0); yp[v] = T(0); }
        T ysu[VZ], ysd[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            ysu[v] = __shfl_up(pc[R - 1][v], t.tpr, 64);
            ysd[v] = __shfl_down(pc[0][v], t.tpr, 64);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++)
            if (rr < t.nrows && i + 1 < bx) vload<T, VZ>(p + o + P + (long long)rr * bz, pp[rr]);
        if (ym_ld) {
            if (ym_sh) {
#pragma unroll
                for (int v = 0; v < VZ; v++) ym[v] = ysu[v];
            } else {
                vload<T, VZ>(p + o - bz, ym);
            }
        }
        if (yp_ld) {
            if (yp_sh) {
#pragma unroll
                for (int v = 0; v < VZ; v++) yp[v] = ysd[v];
            } else {
                vload<T, VZ>(p + o + (long long)t.nrows * bz, yp);
            }
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            const T sl = from_left(pc[rr][VZ - 1]);
            const T sr = from_right(pc[rr][0]);
            if (rr >= t.nrows) continue;
            const long long orow = o + (long long)rr * bz;
            T zm = T(0), zp = T(0);
            if (zm_in) zm = zm_sh ? sl : p[orow - 1];
            if (zp_in) zp = zp_sh ? sr : p[orow + VZ];
            T rv[VZ];
            TD dd[VZ];
            vload<T, VZ>(r + orow, rv);
            if (have_d) {
                vload<TD, VZ>(d + orow, dd);
            } else {
#pragma unroll
                for (int v = 0; v < VZ; v++) dd[v] = TD(0);
            }
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[rr][v - 1];
                const T right = v == VZ - 1 ? zp : pc[rr][v + 1];
                const T up = rr == 0 ? ym[v] : pc[rr - 1][v];
                const T down = (rr == R - 1 || rr + 1 == t.nrows) ? yp[v] : pc[rr + 1][v];
                T q = T(6) * pc[rr][v] - pm[rr][v] - pp[rr][v] - up - down - left - right;
                if (OVL && axes_out(t.B, i, t.j0 + rr, t.k + v) > 1) q = T(0);
                dd[v] = dd[v] + alpha * pc[rr][v];
                rv[v] = rv[v] - alpha * q;
                acc += rv[v] * rv[v];
            }
            vstore<TD, VZ>(d + orow, dd);
            vstore<T, VZ>(r + orow, rv);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int v = 0; v < VZ; v++) { pm[rr][v] = pc[rr][v]; pc[rr][v] = pp[rr][v]; pp[rr][v] = T(0); }
    }
    return acc;
}

// Outer update on one tile (Section 3: X_i^(k) = X_i^(k-1) + correction):
// xb = xa + d (when have_d) + alpha p (when use_p), in FP64.  xb may equal xa.
// OVL: only the block's own cells are written (each cell takes its owner's
// correction: the multisplitting weights D_i of Section 2.3 are 0/1); the
// vector width divides the own box's z offset and extent, so a z vector is
// wholly own or wholly not.
template <typename T, int VZ, int R, bool OVL = false>
__device__ __forceinline__ void tile_final(const Geom &g, const Tile &t, long long goff,
                                           const T *p, const T *d, T alpha, bool have_d,
                                           bool use_p, const double *xa, double *xb) {
    const int bz = t.B.bz, by = t.B.by;
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const long long J0 = t.B.j0 + t.j0, K = t.B.k0 + t.k;
    for (int i = t.xbeg; i < t.xend; i++) {
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            if (rr >= t.nrows) continue;
            if (OVL && axes_out(t.B, i, t.j0 + rr, t.k) != 0) continue;
            const long long o = base + (long long)i * P + (long long)rr * bz;
            const long long gI = ((long long)(t.B.i0 + i) * g.ny + J0 + rr) * g.nz + K;
            double xo[VZ];
            vload<double, VZ>(xa + gI, xo);
            if (have_d) {
                T dd[VZ];
                vload<T, VZ>(d + o, dd);
#pragma unroll
                for (int v = 0; v < VZ; v++) xo[v] += (double)dd[v];
            }
            if (use_p) {
                T pc[VZ];
                vload<T, VZ>(p + o, pc);
#pragma unroll
                for (int v = 0; v < VZ; v++) xo[v] += (double)(alpha * pc[v]);
            }
            vstore<double, VZ>(xb + gI, xo);
        }
    }
}

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
    const int k = w / bt.nt;
    if (ctrl && ctrl[k].done) return;
    const int tile = t0 + (w - k * bt.nt);
    if (b) b += k * bt.vs;
    if (x) x += k * bt.vs;
    if (r) r += k * bt.is;
    p64 += (long long)k * bt.ps;
    pT += (long long)k * bt.ps;
    const Tile t = decode_tile<VZ, R>(g, tile, threadIdx.x);
    double acc64 = 0.0;
    T accT = T(0);
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
    const int k = w / bt.nt;
    if (ctrl[k].done) return;
    const int tile = t0 + (w - k * bt.nt);
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
    const int k = w / bt.nt;
    ctrl += k;
    if (ctrl->done) return;
    const int tile = t0 + (w - k * bt.nt);
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
    const double acc = tile_stencil<double, VZ, R>(t, 0, r, pold, pnew, beta, iter > 0);
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
    const double acc = tile_update<double, double, VZ, R>(t, 0, r, p, x, scal[1], true);
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
    __shared__ int s_blk;
    __shared__ int s_gap;
    __shared__ unsigned long long s_key[kAsyncThreads / 64];
    const int tid = threadIdx.x;
    const int sub = tid / kThreads;
    const int ltid = tid % kThreads;
    const int nb = g.nblocks;
    for (;;) {
        // ---- the eligible unclaimed block with the lowest version ----
        unsigned long long best = ~0ull;
        for (int c = tid; c < nb; c += kAsyncThreads) {
            const int blk = (c + (int)blockIdx.x * 7) % nb;   // spread the start per worker
            if (__hip_atomic_load(&as.claim[blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
            const int v = __hip_atomic_load(&as.version[blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v >= max_sweeps) continue;
            bool ok = true;
            for (int f = 0; f < 6 && ok; f++) {
                const int nbk = as.nbr[blk * 6 + f];
                if (nbk < 0) continue;
                const int vn = __hip_atomic_load(&as.version[nbk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = vn >= v + 1 - S;
            }
            if (!ok) continue;
            const unsigned long long key = ((unsigned long long)(unsigned)v << 32) | (unsigned)blk;
            best = key < best ? key : best;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long other = __shfl_xor(best, o, 64);
            best = other < best ? other : best;
        }
        if ((tid & 63) == 0) s_key[tid >> 6] = best;
        __syncthreads();
        if (tid == 0) {
            unsigned long long k = ~0ull;
            for (int w = 0; w < kAsyncThreads / 64; w++) k = s_key[w] < k ? s_key[w] : k;
            int pick = -1;
            if (__hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                k = ~0ull;       // the residual estimate is below tol: start nothing new
            }
            if (k != ~0ull) {
                const int cand = (int)(k & 0xffffffffu);
                int zero = 0;
                if (__hip_atomic_compare_exchange_strong(&as.claim[cand], &zero, 1, __ATOMIC_ACQUIRE,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    pick = cand;
            }
            if (pick < 0) {
                const bool stop = __hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                const int fin = __hip_atomic_load(as.finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (stop || fin >= nb) pick = -2;
            } else {
                // staleness this sweep will see, then acquire the neighbours'
                // published x values
                const int v = __hip_atomic_load(&as.version[pick], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                int gap = 0;
                for (int f = 0; f < 6; f++) {
                    const int nbk = as.nbr[pick * 6 + f];
                    if (nbk < 0) continue;
                    const int vn = __hip_atomic_load(&as.version[nbk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    gap = max(gap, v - vn);
                }
                s_gap = gap;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_blk = pick;
        }
        __syncthreads();
        const int blk = s_blk;
        __syncthreads();
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
        // ---- publish: x of this block, then its version ----
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            const int v = __hip_atomic_load(&as.version[blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
            __hip_atomic_store(&as.version[blk], v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&as.claim[blk], 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (v >= max_sweeps) atomicAdd(as.finished, 1);
            atomicAdd(&ctrl->inner_iters, (unsigned long long)iters);
            atomicAdd(&ctrl->work_items, 1ull);
            atomicMax(&ctrl->max_stale, s_gap);
            if (tol2 > 0.0) {
                // residual estimate from the latest published block residuals
                // (Section 3: an estimate that may be some sweeps old)
                double est = 0.0;
                for (int q = 0; q < nb; q++)
                    est += __hip_atomic_load(&as.board[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (est <= tol2) __hip_atomic_store(&ctrl->stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
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

// Grid for tiles [t0, t1) of every right-hand side of the batch.
inline dim3 batch_grid(int t0, int t1, Batch &bt) {
    bt.nt = t1 - t0;
    return dim3((unsigned)((long long)bt.nt * bt.nrhs));
}

template <typename T>
hipError_t launch_resid(const Geom &g, int vz, int t0, int t1, long long goff,
                        const double *b, const double *x, Faces faces, T *r, double *p64,
                        T *pT, const Ctrl *ctrl, Batch bt, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    const dim3 grid = batch_grid(t0, t1, bt);
#define MS_RESID(STORE, OVL)                                                               \
    MS_DISPATCH(vz, g.rows, hipLaunchKernelGGL((k_resid<T, VZ, RR, STORE, OVL>), grid,      \
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
    MS_DISPATCH(vz, g.rows, hipLaunchKernelGGL((k_stencil<T, VZ, RR>), grid,
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
    MS_DISPATCH(vz, g.rows, hipLaunchKernelGGL((k_update<T, VZ, RR, LAST, OVL>), grid,       \
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
        MS_DISPATCH_A(vz, g.rows, hipLaunchKernelGGL((k_async<T, VZ, RR, true>), dim3(grid),
                                                     dim3(kAsyncThreads), 0, st, g, b, x, faces,
                                                     r, p0, p1, d, as, m, S, max_sweeps, tol2,
                                                     inner_tol, ctrl));
    } else {
        MS_DISPATCH_A(vz, g.rows, hipLaunchKernelGGL((k_async<T, VZ, RR, false>), dim3(grid),
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
    MS_DISPATCH64(vz, g.rows, hipLaunchKernelGGL((k_gcg_stencil<VZ, RR>), dim3(ntiles),
                                                 dim3(kThreads), 0, st, g, r, pold, pnew, psig,
                                                 scal, iter, ctrl));
    return hipGetLastError();
}

hipError_t launch_gcg_update(const Geom &g, int vz, int ntiles, double *r, const double *p,
                             double *x, double *prho, const double *scal, const Ctrl *ctrl,
                             hipStream_t st) {
    MS_DISPATCH64(vz, g.rows, hipLaunchKernelGGL((k_gcg_update<VZ, RR>), dim3(ntiles),
                                                 dim3(kThreads), 0, st, g, r, p, x, prho, scal,
                                                 ctrl));
    return hipGetLastError();
}

hipError_t launch_gcg_reduce(const double *part, int ntiles, int which, double tol, int max_iters,
                             double *history, int history_cap, double *scal, Ctrl *ctrl,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_gcg_reduce, dim3(1), dim3(kThreads), 0, st, part, ntiles, which, tol,
                       max_iters, history, history_cap, scal, ctrl);
    return hipGetLastError();
}

hipError_t launch_check(const double *p64, int ntiles, double tol, int final_check,
                        double *history, int history_cap, Ctrl *ctrl, Batch bt,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_check, dim3(bt.nrhs), dim3(kThreads), 0, st, p64, ntiles, tol,
                       final_check, history, history_cap, ctrl, bt);
    return hipGetLastError();
}

hipError_t launch_norm(const double *p64, int ntiles, Ctrl *ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(kThreads), 0, st, p64, ntiles, ctrl);
    return hipGetLastError();
}

hipError_t launch_sum(const double *v, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, st, v, n, out);
    return hipGetLastError();
}

hipError_t launch_apply(long long nx, long long ny, long long nz, const double *u, double *y,
                        hipStream_t st) {
    const long long n = nx * ny * nz;
    long long grid = (n + kThreads - 1) / kThreads;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_apply, dim3((unsigned)grid), dim3(kThreads), 0, st, nx, ny, nz, u, y);
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
