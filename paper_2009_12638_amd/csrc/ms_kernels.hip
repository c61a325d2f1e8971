// HIP kernels of libms for gfx950: outer residual with in-memory halo reads,
// the two phases of the inner block CG, the fused final update, and the
// deterministic reductions behind the convergence test.
//
// Tiling.  Every block-local kernel runs one 256-thread workgroup per tile.
// A tile is a run of 256*VZ consecutive cells of a block's y-z plane (z
// fastest, each thread owning VZ consecutive z cells of one row) marched
// along x over up to `tx` planes.  The x neighbours come from a register
// pipeline (previous / current / next plane); y and z neighbours are loaded
// (they are mostly cache hits: the rows belong to the same or an adjacent
// workgroup).  Loads are VZ-wide (16 bytes for VZ*sizeof(T) = 16), so a
// 64-lane wavefront reads whole contiguous z runs.
//
// Reductions.  A tile's partial sum is reduced across its wavefronts
// (lane shuffles, then LDS) and written to a per-tile slot.  Consumers add a
// block's tile slots in tile order, so every reduction has a fixed order and
// results are bitwise reproducible run to run.
#include "ms_internal.h"

#include <math.h>

namespace ms {

// ----------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------

template <typename T, int N>
struct alignas(sizeof(T) * N) VecT {
    T v[N];
};

// N consecutive values starting at p (p aligned to sizeof(T)*N).
template <typename T, int N>
__device__ __forceinline__ void vload(const T *__restrict__ p, T (&o)[N]) {
    constexpr int C = (sizeof(T) * N <= 16) ? N : (int)(16 / sizeof(T));
#pragma unroll
    for (int c = 0; c < N; c += C) {
        VecT<T, C> t = *reinterpret_cast<const VecT<T, C> *>(p + c);
#pragma unroll
        for (int v = 0; v < C; v++) o[c + v] = t.v[v];
    }
}

template <typename T, int N>
__device__ __forceinline__ void vstore(T *__restrict__ p, const T (&o)[N]) {
    constexpr int C = (sizeof(T) * N <= 16) ? N : (int)(16 / sizeof(T));
#pragma unroll
    for (int c = 0; c < N; c += C) {
        VecT<T, C> t;
#pragma unroll
        for (int v = 0; v < C; v++) t.v[v] = o[c + v];
        *reinterpret_cast<VecT<T, C> *>(p + c) = t;
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256 threads of the workgroup; the result is valid in thread 0.
// Fixed shape: lanes by butterfly, then waves 0..3 as (w0 + w1) + (w2 + w3).
template <typename T>
__device__ __forceinline__ T wg_sum(T v) {
    __shared__ T sh[kThreads / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return s;
}

// Sum of a block's tile partials in tile order.  Every thread computes it
// (uniform loads), so no broadcast is needed.
template <typename T>
__device__ __forceinline__ T tiles_sum(const T *__restrict__ part, int t0, int n) {
    T s = T(0);
    for (int t = 0; t < n; t++) s += part[t0 + t];
    return s;
}

struct Tile {
    int b;             // block number
    BlockInfo B;
    int q0;            // first plane cell of this thread (j*bz + k)
    bool live;         // thread owns cells
    int j, k;          // row and first z of the thread's cells
    int xbeg, xend;    // planes marched
    bool first;        // first tile of its block
};

template <int VZ>
__device__ __forceinline__ Tile decode_tile(const Geom &g, int tile) {
    Tile t;
    t.b = g.tile_block[tile];
    t.B = g.blocks[t.b];
    const int local = tile - t.B.tile0;
    const int pt = local % t.B.nplane;
    const int xc = local / t.B.nplane;
    const int P = t.B.by * t.B.bz;
    t.q0 = (pt * kThreads + (int)threadIdx.x) * VZ;
    t.live = t.q0 < P;
    const int q = t.live ? t.q0 : 0;
    t.j = q / t.B.bz;
    t.k = q % t.B.bz;
    t.xbeg = xc * g.tx;
    t.xend = min(t.B.bx, t.xbeg + g.tx);
    t.first = (local == 0);
    return t;
}

// ----------------------------------------------------------------------
// outer residual r = b_eff - A x (Section 3: the right-hand side
// B_i - sum_j A_ij X_j of every block, with neighbour-block values read
// straight from x: the halo exchange of Listing 1)
// ----------------------------------------------------------------------

template <typename T, int VZ, bool STORE>
__global__ __launch_bounds__(kThreads) void k_resid(Geom g, int t0, long long goff,
                                                    const double *__restrict__ b,
                                                    const double *__restrict__ x, Faces F,
                                                    T *__restrict__ r, double *__restrict__ p64,
                                                    T *__restrict__ pT, const Ctrl *ctrl) {
    if (ctrl && ctrl->done) return;
    const int tile = t0 + blockIdx.x;
    const Tile t = decode_tile<VZ>(g, tile);
    const long long nx = g.nx, ny = g.ny, nz = g.nz;
    double acc64 = 0.0;
    T accT = T(0);
    if (t.live) {
        const long long P = (long long)t.B.by * t.B.bz;
        const long long J = t.B.j0 + t.j, K = t.B.k0 + t.k;
        const bool ym_ok = J > 0, yp_ok = J < ny - 1, zm_ok = K > 0, zp_ok = K + VZ < nz;
        const long long sx = ny * nz;  // x stride in the global layout
        auto gidx = [&](long long I) { return (I * ny + J) * nz + K; };
        double xm[VZ], xc[VZ], xp[VZ];
        const long long I0 = t.B.i0 + t.xbeg;
#pragma unroll
        for (int v = 0; v < VZ; v++) { xm[v] = 0.0; xc[v] = 0.0; }
        if (x) {
            if (I0 > 0) vload<double, VZ>(x + gidx(I0 - 1), xm);
            vload<double, VZ>(x + gidx(I0), xc);
        }
        T *rrow = r + (t.B.off - goff) + t.q0;
        for (int i = t.xbeg; i < t.xend; i++) {
            const long long I = t.B.i0 + i;
            const long long c = gidx(I);
            double ym[VZ], yp[VZ], bb[VZ];
            double zm = 0.0, zp = 0.0;
#pragma unroll
            for (int v = 0; v < VZ; v++) { xp[v] = 0.0; ym[v] = 0.0; yp[v] = 0.0; bb[v] = 0.0; }
            if (x) {
                if (I + 1 < nx) vload<double, VZ>(x + c + sx, xp);
                if (ym_ok) vload<double, VZ>(x + c - nz, ym);
                if (yp_ok) vload<double, VZ>(x + c + nz, yp);
                if (zm_ok) zm = x[c - 1];
                if (zp_ok) zp = x[c + VZ];
            }
            if (b) vload<double, VZ>(b + c, bb);
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
                const double left = v == 0 ? zm : xc[v - 1];
                const double right = v == VZ - 1 ? zp : xc[v + 1];
                const double ax = 6.0 * xc[v] - xm[v] - xp[v] - ym[v] - yp[v] - left - right;
                const double rv = bb[v] - ax;
                acc64 += rv * rv;
                out[v] = (T)rv;
                accT += out[v] * out[v];
            }
            if (STORE) vstore<T, VZ>(rrow + (long long)i * P, out);
#pragma unroll
            for (int v = 0; v < VZ; v++) { xm[v] = xc[v]; xc[v] = xp[v]; }
        }
    }
    const double s64 = wg_sum(acc64);
    if (sizeof(T) == sizeof(double)) {
        if (threadIdx.x == 0) p64[tile] = s64;
    } else {
        const T sT = wg_sum(accT);
        if (threadIdx.x == 0) { p64[tile] = s64; pT[tile] = sT; }
    }
}

// ----------------------------------------------------------------------
// inner CG, phase 1 (Section 3: the inner Krylov solve of each block on
// A_ii; here CG): p_new = r + beta p_old, sigma = p_new . A_ii p_new
// ----------------------------------------------------------------------

template <typename T, int VZ>
__global__ __launch_bounds__(kThreads) void k_stencil(Geom g, int t0, long long goff,
                                                      const T *__restrict__ r,
                                                      const T *__restrict__ pold,
                                                      T *__restrict__ pnew, T *__restrict__ psig,
                                                      const T *__restrict__ prho_cur,
                                                      const T *__restrict__ prho_prev,
                                                      const T *__restrict__ prho0,
                                                      int *active, int iter, double inner_tol,
                                                      Ctrl *ctrl) {
    if (ctrl->done) return;
    const int tile = t0 + blockIdx.x;
    const Tile t = decode_tile<VZ>(g, tile);
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
    const bool use_old = iter > 0;
    T acc = T(0);
    if (t.live) {
        const int bz = t.B.bz, by = t.B.by, bx = t.B.bx;
        const long long P = (long long)by * bz;
        const long long base = (t.B.off - goff) + t.q0;
        const bool ym_ok = t.j > 0, yp_ok = t.j < by - 1, zm_ok = t.k > 0,
                   zp_ok = t.k + VZ < bz;
        // p_new at VZ cells starting at offset o
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
        T pm[VZ], pc[VZ], pp[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) pm[v] = T(0);
        if (t.xbeg > 0) pv(base + (long long)(t.xbeg - 1) * P, pm);
        pv(base + (long long)t.xbeg * P, pc);
        for (int i = t.xbeg; i < t.xend; i++) {
            const long long o = base + (long long)i * P;
            T ym[VZ], yp[VZ];
            T zm = T(0), zp = T(0);
#pragma unroll
            for (int v = 0; v < VZ; v++) { pp[v] = T(0); ym[v] = T(0); yp[v] = T(0); }
            if (i + 1 < bx) pv(o + P, pp);
            if (ym_ok) pv(o - bz, ym);
            if (yp_ok) pv(o + bz, yp);
            if (zm_ok) zm = ps(o - 1);
            if (zp_ok) zp = ps(o + VZ);
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[v - 1];
                const T right = v == VZ - 1 ? zp : pc[v + 1];
                const T q = T(6) * pc[v] - pm[v] - pp[v] - ym[v] - yp[v] - left - right;
                acc += pc[v] * q;
            }
            vstore<T, VZ>(pnew + o, pc);
#pragma unroll
            for (int v = 0; v < VZ; v++) { pm[v] = pc[v]; pc[v] = pp[v]; }
        }
    }
    const T s = wg_sum(acc);
    if (threadIdx.x == 0) psig[tile] = s;
}

// ----------------------------------------------------------------------
// inner CG, phase 2: alpha = rho / sigma; d += alpha p; r -= alpha A_ii p;
// rho' = r.r.  On the last inner iteration the correction is applied to the
// outer iterate instead: x_new = x_old + d + alpha p (Section 3's update
// X_i^(k) from sweep k-1 values; x_new is a separate buffer so every block's
// residual of this sweep saw only x_old).
// ----------------------------------------------------------------------

template <typename T, int VZ, bool LAST>
__global__ __launch_bounds__(kThreads) void k_update(Geom g, int t0, long long goff,
                                                     T *__restrict__ r,
                                                     const T *__restrict__ p,
                                                     T *__restrict__ d,
                                                     const T *__restrict__ psig,
                                                     const T *__restrict__ prho_cur,
                                                     T *__restrict__ prho_next, int *active,
                                                     int iter, const double *__restrict__ xa,
                                                     double *__restrict__ xb, Ctrl *ctrl) {
    if (ctrl->done) return;
    const int tile = t0 + blockIdx.x;
    const Tile t = decode_tile<VZ>(g, tile);
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
    const int bz = t.B.bz, by = t.B.by, bx = t.B.bx;
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + t.q0;
    if (LAST) {
        // x_new = x_old + d + alpha p, for every block (inactive ones too)
        if (t.live) {
            const long long J = t.B.j0 + t.j, K = t.B.k0 + t.k;
            for (int i = t.xbeg; i < t.xend; i++) {
                const long long o = base + (long long)i * P;
                const long long gI = ((long long)(t.B.i0 + i) * g.ny + J) * g.nz + K;
                double xo[VZ];
                vload<double, VZ>(xa + gI, xo);
                if (iter > 0) {
                    T dd[VZ];
                    vload<T, VZ>(d + o, dd);
#pragma unroll
                    for (int v = 0; v < VZ; v++) xo[v] += (double)dd[v];
                }
                if (act) {
                    T pc[VZ];
                    vload<T, VZ>(p + o, pc);
#pragma unroll
                    for (int v = 0; v < VZ; v++) xo[v] += (double)(alpha * pc[v]);
                }
                vstore<double, VZ>(xb + gI, xo);
            }
        }
        return;
    }
    if (!act) {
        // a block that stops before its first step keeps a zero correction
        if (iter == 0 && t.live) {
            T z[VZ];
#pragma unroll
            for (int v = 0; v < VZ; v++) z[v] = T(0);
            for (int i = t.xbeg; i < t.xend; i++) vstore<T, VZ>(d + base + (long long)i * P, z);
        }
        return;
    }
    T acc = T(0);
    if (t.live) {
        const bool ym_ok = t.j > 0, yp_ok = t.j < by - 1, zm_ok = t.k > 0,
                   zp_ok = t.k + VZ < bz;
        T pm[VZ], pc[VZ], pp[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) pm[v] = T(0);
        if (t.xbeg > 0) vload<T, VZ>(p + base + (long long)(t.xbeg - 1) * P, pm);
        vload<T, VZ>(p + base + (long long)t.xbeg * P, pc);
        for (int i = t.xbeg; i < t.xend; i++) {
            const long long o = base + (long long)i * P;
            T ym[VZ], yp[VZ], rr[VZ], dd[VZ];
            T zm = T(0), zp = T(0);
#pragma unroll
            for (int v = 0; v < VZ; v++) { pp[v] = T(0); ym[v] = T(0); yp[v] = T(0); dd[v] = T(0); }
            if (i + 1 < bx) vload<T, VZ>(p + o + P, pp);
            if (ym_ok) vload<T, VZ>(p + o - bz, ym);
            if (yp_ok) vload<T, VZ>(p + o + bz, yp);
            if (zm_ok) zm = p[o - 1];
            if (zp_ok) zp = p[o + VZ];
            vload<T, VZ>(r + o, rr);
            if (iter > 0) vload<T, VZ>(d + o, dd);
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[v - 1];
                const T right = v == VZ - 1 ? zp : pc[v + 1];
                const T q = T(6) * pc[v] - pm[v] - pp[v] - ym[v] - yp[v] - left - right;
                dd[v] = dd[v] + alpha * pc[v];
                rr[v] = rr[v] - alpha * q;
                acc += rr[v] * rr[v];
            }
            vstore<T, VZ>(d + o, dd);
            vstore<T, VZ>(r + o, rr);
#pragma unroll
            for (int v = 0; v < VZ; v++) { pm[v] = pc[v]; pc[v] = pp[v]; }
        }
    }
    const T s = wg_sum(acc);
    if (threadIdx.x == 0) prho_next[tile] = s;
}

// ----------------------------------------------------------------------
// global residual and convergence test (Section 3: global residual = root
// of the sum of squared block residuals; Listing 1: loop while it is above
// the threshold; Section 2.1: stop on ||Ax - b||)
// ----------------------------------------------------------------------

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

__global__ __launch_bounds__(kThreads) void k_check(const double *__restrict__ p64, int ntiles,
                                                    double tol, int final_check,
                                                    double *history, int history_cap,
                                                    Ctrl *ctrl) {
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

#define MS_VZ_DISPATCH(vz, ...)                                   \
    switch (vz) {                                                 \
        case 1: { constexpr int VZ = 1; __VA_ARGS__; break; }     \
        case 2: { constexpr int VZ = 2; __VA_ARGS__; break; }     \
        case 4: { constexpr int VZ = 4; __VA_ARGS__; break; }     \
        default: return hipErrorInvalidValue;                     \
    }

template <typename T>
hipError_t launch_resid(const Geom &g, int vz, int t0, int t1, long long goff,
                        const double *b, const double *x, Faces faces, T *r, double *p64,
                        T *pT, const Ctrl *ctrl, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    if (r) {
        MS_VZ_DISPATCH(vz, hipLaunchKernelGGL((k_resid<T, VZ, true>), dim3(t1 - t0),
                                              dim3(kThreads), 0, st, g, t0, goff, b, x,
                                              faces, r, p64, pT, ctrl));
    } else {
        MS_VZ_DISPATCH(vz, hipLaunchKernelGGL((k_resid<T, VZ, false>), dim3(t1 - t0),
                                              dim3(kThreads), 0, st, g, t0, goff, b, x,
                                              faces, r, p64, pT, ctrl));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const Geom &g, int vz, int t0, int t1, long long goff,
                          const T *r, const T *p_old, T *p_new, T *psig, const T *prho_cur,
                          const T *prho_prev, const T *prho0, int *active, int iter,
                          double inner_tol, Ctrl *ctrl, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    MS_VZ_DISPATCH(vz, hipLaunchKernelGGL((k_stencil<T, VZ>), dim3(t1 - t0), dim3(kThreads),
                                          0, st, g, t0, goff, r, p_old, p_new, psig,
                                          prho_cur, prho_prev, prho0, active, iter,
                                          inner_tol, ctrl));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const Geom &g, int vz, int t0, int t1, long long goff, T *r,
                         const T *p, T *d, const T *psig, const T *prho_cur, T *prho_next,
                         int *active, int iter, int last, const double *xa, double *xb,
                         Ctrl *ctrl, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    if (last) {
        MS_VZ_DISPATCH(vz, hipLaunchKernelGGL((k_update<T, VZ, true>), dim3(t1 - t0),
                                              dim3(kThreads), 0, st, g, t0, goff, r, p, d,
                                              psig, prho_cur, prho_next, active, iter, xa,
                                              xb, ctrl));
    } else {
        MS_VZ_DISPATCH(vz, hipLaunchKernelGGL((k_update<T, VZ, false>), dim3(t1 - t0),
                                              dim3(kThreads), 0, st, g, t0, goff, r, p, d,
                                              psig, prho_cur, prho_next, active, iter, xa,
                                              xb, ctrl));
    }
    return hipGetLastError();
}

hipError_t launch_check(const double *p64, int ntiles, double tol, int final_check,
                        double *history, int history_cap, Ctrl *ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kThreads), 0, st, p64, ntiles, tol,
                       final_check, history, history_cap, ctrl);
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
                                        const Ctrl *, hipStream_t);                           \
    template hipError_t launch_stencil<T>(const Geom &, int, int, int, long long, const T *,  \
                                          const T *, T *, T *, const T *, const T *,          \
                                          const T *, int *, int, double, Ctrl *,              \
                                          hipStream_t);                                       \
    template hipError_t launch_update<T>(const Geom &, int, int, int, long long, T *,         \
                                         const T *, T *, const T *, const T *, T *, int *,    \
                                         int, int, const double *, double *, Ctrl *,          \
                                         hipStream_t);
MS_INST(double)
MS_INST(float)

}  // namespace ms
