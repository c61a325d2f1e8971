// Tile bodies shared by the HIP sources of libms: the outer residual with
// in-memory halo reads, the two phases of the inner block CG and the outer
// update, each on one tile of a block (thread geometry in ms_device.h).
// Not part of the public ABI.
#pragma once
#include "ms_internal.h"
#include "ms_device.h"

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

// The outer residual with its loads requested one plane ahead (as the CG
// phases below): while plane i is computed, plane i + 2 of x (plane i + 1's
// x + 1 neighbour), plane i + 1 of b and plane i + 1's row and z neighbours
// that sit in memory are requested, and taken up at the top of the next
// iteration.  Same arithmetic in the same order as tile_resid.  The residual
// streams x and b from HBM (neither is re-read within a sweep), which is
// where the lookahead pays.
template <typename T, int VZ, int R, bool STORE, bool OVL = false>
__device__ __forceinline__ void tile_resid_pf(const Geom &g, const Tile &t, long long goff,
                                              const double *__restrict__ b, const double *x,
                                              const Faces &F, T *__restrict__ r, double &acc64,
                                              T &accT) {
    const long long nx = g.nx, ny = g.ny, nz = g.nz;
    const long long J0 = t.B.j0 + t.j0, K = t.B.k0 + t.k;
    const long long P = (long long)t.B.by * t.B.bz;
    auto gidx = [&](long long I, int rr) { return (I * ny + J0 + rr) * nz + K; };
    const bool zm_in = K > 0, zp_in = K + VZ < nz;
    const bool zm_sh = t.zc > 0 && t.lane > 0;
    const bool zp_sh = t.zc < t.tpr - 1 && t.lane < 63;
    const bool ym_ld = t.nrows > 0 && J0 > 0;
    const bool yp_ld = t.nrows > 0 && J0 + t.nrows < ny;
    const bool ym_sh = t.j0 > 0 && t.lane >= t.tpr;
    const bool yp_sh = t.j0 + t.nrows < t.B.by && t.lane + t.tpr < 64;
    const bool have_x = x != nullptr;
    const bool ym_mem = have_x && ym_ld && !ym_sh, yp_mem = have_x && yp_ld && !yp_sh;
    const bool zm_mem = have_x && zm_in && !zm_sh, zp_mem = have_x && zp_in && !zp_sh;
    const int lim = t.xend + 1;   // tile-local planes of x this tile reads end here
    // x of tile-local plane i on the owned rows (zero outside the grid)
    auto ld_x = [&](int i, double(&a)[R][VZ]) {
        const long long I = t.B.i0 + i;
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
#pragma unroll
            for (int v = 0; v < VZ; v++) a[rr][v] = 0.0;
            if (have_x && rr < t.nrows && i < lim && I >= 0 && I < nx)
                vload<double, VZ>(x + gidx(I, rr), a[rr]);
        }
    };
    // b and the memory-held row and z neighbours of plane i
    double nb[R][VZ], yv[2][VZ], zv[R][2];
#pragma unroll
    for (int v = 0; v < VZ; v++) { yv[0][v] = 0.0; yv[1][v] = 0.0; }
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        zv[rr][0] = zv[rr][1] = 0.0;
#pragma unroll
        for (int v = 0; v < VZ; v++) nb[rr][v] = 0.0;
    }
    auto ld_aux = [&](int i) {
        const long long I = t.B.i0 + i;
        if (ym_mem) vload<double, VZ>(x + gidx(I, -1), yv[0]);
        if (yp_mem) vload<double, VZ>(x + gidx(I, t.nrows), yv[1]);
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            if (rr >= t.nrows) continue;
            const long long c = gidx(I, rr);
            if (b) vload<double, VZ>(b + c, nb[rr]);
            if (zm_mem) zv[rr][0] = x[c - 1];
            if (zp_mem) zv[rr][1] = x[c + VZ];
        }
    };
    double xm[R][VZ], xc[R][VZ], xn[R][VZ];
    ld_x(t.xbeg - 1, xm);
    ld_x(t.xbeg, xc);
    ld_x(t.xbeg + 1, xn);
    if (t.xbeg < t.xend) ld_aux(t.xbeg);
    for (int i = t.xbeg; i < t.xend; i++) {
        const long long I = t.B.i0 + i;
        // take up what was requested for this plane
        double xp[R][VZ], bb[R][VZ], ym[VZ], yp[VZ], zmv[R], zpv[R];
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            zmv[rr] = zv[rr][0];
            zpv[rr] = zv[rr][1];
#pragma unroll
            for (int v = 0; v < VZ; v++) { xp[rr][v] = xn[rr][v]; bb[rr][v] = nb[rr][v]; }
        }
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            const double su = __shfl_up(xc[R - 1][v], t.tpr, 64);
            const double sd = __shfl_down(xc[0][v], t.tpr, 64);
            ym[v] = (have_x && ym_ld) ? (ym_sh ? su : yv[0][v]) : 0.0;
            yp[v] = (have_x && yp_ld) ? (yp_sh ? sd : yv[1][v]) : 0.0;
        }
        // request plane i + 1's data
        ld_x(i + 2, xn);
        if (i + 1 < t.xend) ld_aux(i + 1);
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            const double sl = from_left(xc[rr][VZ - 1]);
            const double sr = from_right(xc[rr][0]);
            if (rr >= t.nrows) continue;
            double zm = 0.0, zp = 0.0;
            if (have_x && zm_in) zm = zm_sh ? sl : zmv[rr];
            if (have_x && zp_in) zp = zp_sh ? sr : zpv[rr];
            const long long J = J0 + rr;
            // Dirichlet lifting: boundary neighbours' g moved to the right
            if (I == 0 && F.f[0]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[rr][v] += F.f[0][J * nz + K + v];
            }
            if (I == nx - 1 && F.f[1]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[rr][v] += F.f[1][J * nz + K + v];
            }
            if (J == 0 && F.f[2]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[rr][v] += F.f[2][I * nz + K + v];
            }
            if (J == ny - 1 && F.f[3]) {
#pragma unroll
                for (int v = 0; v < VZ; v++) bb[rr][v] += F.f[3][I * nz + K + v];
            }
            if (K == 0 && F.f[4]) bb[rr][0] += F.f[4][I * ny + J];
            if (K + VZ == nz && F.f[5]) bb[rr][VZ - 1] += F.f[5][I * ny + J];
            T out[VZ];
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const double left = v == 0 ? zm : xc[rr][v - 1];
                const double right = v == VZ - 1 ? zp : xc[rr][v + 1];
                const double up = rr == 0 ? ym[v] : xc[rr - 1][v];
                const double down = (rr == R - 1 || rr + 1 == t.nrows) ? yp[v] : xc[rr + 1][v];
                const double ax = 6.0 * xc[rr][v] - xm[rr][v] - xp[rr][v] - up - down - left - right;
                double rv = bb[rr][v] - ax;
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
            for (int v = 0; v < VZ; v++) { xm[rr][v] = xc[rr][v]; xc[rr][v] = xp[rr][v]; }
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

// ---- the two CG phases with their loads requested one plane ahead --------
// Vector loads complete in order, so a value used in the iteration that
// requests it makes the wavefront wait for every load issued before it.
// These versions request, while plane i is computed, everything plane i + 1
// needs (its x + 1 neighbour plane, its row and z neighbours held in memory,
// and in the update phase its r and d), and take them up at the top of the
// next iteration.  A wavefront then waits for loads that have had a whole
// plane of compute to arrive.  Same arithmetic in the same order as
// tile_stencil and tile_update.  Planes beyond the tile's last x + 1
// neighbour are not requested.
//
// Used by the global CG, whose passes stream the whole grid from HBM
// (measured at 512^3 FP64: update pass 1145 -> 1060 us).  The block phases
// run on cache-sized groups whose data comes from the on-package cache at
// lower latency; there the extra registers (lower occupancy) cost more
// than the lookahead gains (measured: mixed sweep unchanged, FP64 sweep
// 16.0 -> 17.9 ms), so they keep tile_stencil and tile_update.

template <typename T, int VZ, int R>
__device__ __forceinline__ T tile_stencil_pf(const Tile &t, long long goff,
                                             const T *__restrict__ r, const T *__restrict__ pold,
                                             T *__restrict__ pnew, T beta, bool use_old) {
    const int bz = t.B.bz, by = t.B.by;
    const int lim = min(t.B.bx, t.xend + 1);   // planes this tile reads
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const bool zm_in = t.zc > 0, zp_in = t.zc < t.tpr - 1;
    const bool zm_sh = zm_in && t.lane > 0, zp_sh = zp_in && t.lane < 63;
    const bool zm_mem = zm_in && !zm_sh, zp_mem = zp_in && !zp_sh;
    const bool ym_ld = t.nrows > 0 && t.j0 > 0;
    const bool yp_ld = t.nrows > 0 && t.j0 + t.nrows < by;
    const bool ym_sh = t.lane >= t.tpr, yp_sh = t.lane + t.tpr < 64;
    const bool ym_mem = ym_ld && !ym_sh, yp_mem = yp_ld && !yp_sh;
    // p = r + beta p_old, formed where the value is used
    auto comb = [&](T rv, T ov) -> T { return use_old ? rv + beta * ov : rv; };
    // r and p_old of plane i on the owned rows (zero where there is none)
    auto ld_plane = [&](int i, T(&a)[R][VZ], T(&c)[R][VZ]) {
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
#pragma unroll
            for (int v = 0; v < VZ; v++) { a[rr][v] = T(0); c[rr][v] = T(0); }
            if (rr < t.nrows && i < lim) {
                const long long o = base + (long long)i * P + (long long)rr * bz;
                vload<T, VZ>(r + o, a[rr]);
                if (use_old) vload<T, VZ>(pold + o, c[rr]);
            }
        }
    };
    // row and z neighbours of plane i that come from memory
    T yr[2][VZ], yo[2][VZ], zr[R][2], zo[R][2];
#pragma unroll
    for (int v = 0; v < VZ; v++) { yr[0][v] = yr[1][v] = yo[0][v] = yo[1][v] = T(0); }
#pragma unroll
    for (int rr = 0; rr < R; rr++) { zr[rr][0] = zr[rr][1] = zo[rr][0] = zo[rr][1] = T(0); }
    auto ld_nbr = [&](int i) {
        const long long o = base + (long long)i * P;
        if (ym_mem) {
            vload<T, VZ>(r + o - bz, yr[0]);
            if (use_old) vload<T, VZ>(pold + o - bz, yo[0]);
        }
        if (yp_mem) {
            vload<T, VZ>(r + o + (long long)t.nrows * bz, yr[1]);
            if (use_old) vload<T, VZ>(pold + o + (long long)t.nrows * bz, yo[1]);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            if (rr >= t.nrows) continue;
            const long long orow = o + (long long)rr * bz;
            if (zm_mem) {
                zr[rr][0] = r[orow - 1];
                if (use_old) zo[rr][0] = pold[orow - 1];
            }
            if (zp_mem) {
                zr[rr][1] = r[orow + VZ];
                if (use_old) zo[rr][1] = pold[orow + VZ];
            }
        }
    };
    T pm[R][VZ], pc[R][VZ], nr[R][VZ], no[R][VZ];
#pragma unroll
    for (int rr = 0; rr < R; rr++)
#pragma unroll
        for (int v = 0; v < VZ; v++) pm[rr][v] = T(0);
    {
        T a[R][VZ], c[R][VZ];
        if (t.xbeg > 0) {
            ld_plane(t.xbeg - 1, a, c);
#pragma unroll
            for (int rr = 0; rr < R; rr++)
#pragma unroll
                for (int v = 0; v < VZ; v++) pm[rr][v] = comb(a[rr][v], c[rr][v]);
        }
        ld_plane(t.xbeg, a, c);
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int v = 0; v < VZ; v++) pc[rr][v] = comb(a[rr][v], c[rr][v]);
    }
    ld_plane(t.xbeg + 1, nr, no);
    if (t.xbeg < t.xend) ld_nbr(t.xbeg);
    T acc = T(0);
    for (int i = t.xbeg; i < t.xend; i++) {
        const long long o = base + (long long)i * P;
        // take up what was requested for this plane
        T pp[R][VZ], ym[VZ], yp[VZ], zmv[R], zpv[R];
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int v = 0; v < VZ; v++) pp[rr][v] = comb(nr[rr][v], no[rr][v]);
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            const T su = __shfl_up(pc[R - 1][v], t.tpr, 64);
            const T sd = __shfl_down(pc[0][v], t.tpr, 64);
            ym[v] = ym_ld ? (ym_sh ? su : comb(yr[0][v], yo[0][v])) : T(0);
            yp[v] = yp_ld ? (yp_sh ? sd : comb(yr[1][v], yo[1][v])) : T(0);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            zmv[rr] = comb(zr[rr][0], zo[rr][0]);
            zpv[rr] = comb(zr[rr][1], zo[rr][1]);
        }
        // request plane i + 1's data
        ld_plane(i + 2, nr, no);
        if (i + 1 < t.xend) ld_nbr(i + 1);
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            const T sl = from_left(pc[rr][VZ - 1]);
            const T sr = from_right(pc[rr][0]);
            if (rr >= t.nrows) continue;
            const long long orow = o + (long long)rr * bz;
            T zm = T(0), zp = T(0);
            if (zm_in) zm = zm_sh ? sl : zmv[rr];
            if (zp_in) zp = zp_sh ? sr : zpv[rr];
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
            for (int v = 0; v < VZ; v++) { pm[rr][v] = pc[rr][v]; pc[rr][v] = pp[rr][v]; }
    }
    return acc;
}

template <typename T, typename TD, int VZ, int R, bool OVL = false>
__device__ __forceinline__ T tile_update_pf(const Tile &t, long long goff, T *__restrict__ r,
                                            const T *__restrict__ p, TD *__restrict__ d, T alpha,
                                            bool have_d) {
    const int bz = t.B.bz, by = t.B.by;
    const int lim = min(t.B.bx, t.xend + 1);   // planes of p this tile reads
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const bool zm_in = t.zc > 0, zp_in = t.zc < t.tpr - 1;
    const bool zm_sh = zm_in && t.lane > 0, zp_sh = zp_in && t.lane < 63;
    const bool zm_mem = zm_in && !zm_sh, zp_mem = zp_in && !zp_sh;
    const bool ym_ld = t.nrows > 0 && t.j0 > 0;
    const bool yp_ld = t.nrows > 0 && t.j0 + t.nrows < by;
    const bool ym_sh = t.lane >= t.tpr, yp_sh = t.lane + t.tpr < 64;
    const bool ym_mem = ym_ld && !ym_sh, yp_mem = yp_ld && !yp_sh;
    // p of plane i on the owned rows (zero where there is none)
    auto ld_p = [&](int i, T(&a)[R][VZ]) {
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
#pragma unroll
            for (int v = 0; v < VZ; v++) a[rr][v] = T(0);
            if (rr < t.nrows && i < lim)
                vload<T, VZ>(p + base + (long long)i * P + (long long)rr * bz, a[rr]);
        }
    };
    // r, d and the memory-held row and z neighbours of plane i
    T nrv[R][VZ], yv[2][VZ], zv[R][2];
    TD ndd[R][VZ];
#pragma unroll
    for (int v = 0; v < VZ; v++) { yv[0][v] = T(0); yv[1][v] = T(0); }
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        zv[rr][0] = zv[rr][1] = T(0);
#pragma unroll
        for (int v = 0; v < VZ; v++) { nrv[rr][v] = T(0); ndd[rr][v] = TD(0); }
    }
    auto ld_aux = [&](int i) {
        const long long o = base + (long long)i * P;
        if (ym_mem) vload<T, VZ>(p + o - bz, yv[0]);
        if (yp_mem) vload<T, VZ>(p + o + (long long)t.nrows * bz, yv[1]);
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            if (rr >= t.nrows) continue;
            const long long orow = o + (long long)rr * bz;
            vload<T, VZ>(r + orow, nrv[rr]);
            if (have_d) vload<TD, VZ>(d + orow, ndd[rr]);
            if (zm_mem) zv[rr][0] = p[orow - 1];
            if (zp_mem) zv[rr][1] = p[orow + VZ];
        }
    };
    T pm[R][VZ], pc[R][VZ], pn[R][VZ];
#pragma unroll
    for (int rr = 0; rr < R; rr++)
#pragma unroll
        for (int v = 0; v < VZ; v++) pm[rr][v] = T(0);
    if (t.xbeg > 0) ld_p(t.xbeg - 1, pm);
    ld_p(t.xbeg, pc);
    ld_p(t.xbeg + 1, pn);
    if (t.xbeg < t.xend) ld_aux(t.xbeg);
    T acc = T(0);
    for (int i = t.xbeg; i < t.xend; i++) {
        const long long o = base + (long long)i * P;
        // take up what was requested for this plane
        T pp[R][VZ], rv[R][VZ], ym[VZ], yp[VZ], zmv[R], zpv[R];
        TD dd[R][VZ];
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            zmv[rr] = zv[rr][0];
            zpv[rr] = zv[rr][1];
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                pp[rr][v] = pn[rr][v];
                rv[rr][v] = nrv[rr][v];
                dd[rr][v] = have_d ? ndd[rr][v] : TD(0);
            }
        }
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            const T su = __shfl_up(pc[R - 1][v], t.tpr, 64);
            const T sd = __shfl_down(pc[0][v], t.tpr, 64);
            ym[v] = ym_ld ? (ym_sh ? su : yv[0][v]) : T(0);
            yp[v] = yp_ld ? (yp_sh ? sd : yv[1][v]) : T(0);
        }
        // request plane i + 1's data
        ld_p(i + 2, pn);
        if (i + 1 < t.xend) ld_aux(i + 1);
#pragma unroll
        for (int rr = 0; rr < R; rr++) {
            const T sl = from_left(pc[rr][VZ - 1]);
            const T sr = from_right(pc[rr][0]);
            if (rr >= t.nrows) continue;
            const long long orow = o + (long long)rr * bz;
            T zm = T(0), zp = T(0);
            if (zm_in) zm = zm_sh ? sl : zmv[rr];
            if (zp_in) zp = zp_sh ? sr : zpv[rr];
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[rr][v - 1];
                const T right = v == VZ - 1 ? zp : pc[rr][v + 1];
                const T up = rr == 0 ? ym[v] : pc[rr - 1][v];
                const T down = (rr == R - 1 || rr + 1 == t.nrows) ? yp[v] : pc[rr + 1][v];
                T q = T(6) * pc[rr][v] - pm[rr][v] - pp[rr][v] - up - down - left - right;
                if (OVL && axes_out(t.B, i, t.j0 + rr, t.k + v) > 1) q = T(0);
                dd[rr][v] = dd[rr][v] + alpha * pc[rr][v];
                rv[rr][v] = rv[rr][v] - alpha * q;
                acc += rv[rr][v] * rv[rr][v];
            }
            vstore<TD, VZ>(d + orow, dd[rr]);
            vstore<T, VZ>(r + orow, rv[rr]);
        }
#pragma unroll
        for (int rr = 0; rr < R; rr++)
#pragma unroll
            for (int v = 0; v < VZ; v++) { pm[rr][v] = pc[rr][v]; pc[rr][v] = pp[rr][v]; }
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

}  // namespace ms
