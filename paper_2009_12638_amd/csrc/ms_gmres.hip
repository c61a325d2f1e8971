// GMRES inner solves of the synchronous multisplitting sweep (Sections 3.1
// and 4: the experiments' inner Krylov solver was GMRES; Section 3.2: a
// maximum number of inner iterations).  One GMRES(m) cycle per block and
// sweep, from a zero correction on the block's residual (or its overlap
// region's).
//
// Krylov vectors are stored unscaled: u_0 = r, u_{j+1} = A v_j minus its
// projections, with v_i = u_i / s_i and s_i = ||u_i|| kept per block, so
// no pass is spent normalising.  One Arnoldi step j is three launches:
//   k_gm_apply  w = A v_j on every tile (7-point stencil, zero outside the
//               block's box, masked outside an overlap region), stored as
//               u_{j+1}; per-tile partials of (w, u_i), i <= j, from the w
//               values still in registers;
//   k_gm_orth   h_ij = (w, u_i) / s_i from the block's partials in a fixed
//               tile order (each workgroup sums them itself), then
//               u_{j+1} = w - sum_i (h_ij / s_i) u_i (classical
//               Gram-Schmidt: all coefficients from the same w), per-tile
//               partials of its squared norm;
//   k_gm_norm   per block: h_{j+1,j} = s_{j+1}; the Givens rotations of
//               the Hessenberg column and the least-squares residual.
// After m steps (or an early stop) k_gm_solve back-substitutes y per block
// and k_gm_final writes x_new = x_old + sum_i (y_i / s_i) u_i on the
// block's own cells.  The Hessenberg arithmetic is FP64; vectors and tile
// partials are in the inner type T (FP32 in mixed precision).
#include "ms_internal.h"
#include "ms_device.h"
#include "ms_tiles.h"

#include <math.h>

namespace ms {

namespace {

// x planes one workgroup marches (the tile's w values stay in registers)
constexpr int kGmPlanes = 8;
// most inner steps a basis may hold (ms_reserve_krylov's limit)
constexpr int kGmMaxSteps = 128;

// Fields of one (right-hand side, block) GMRES record, in doubles.
struct GmRec {
    int M;
    __device__ int s() const { return 0; }                  // M+1 scales s_i
    __device__ int coef() const { return M + 1; }           // M+1 coefficients h_ij / s_i
    __device__ int g() const { return 2 * (M + 1); }        // M+1 rotated right-hand side
    __device__ int y() const { return 3 * (M + 1); }        // M   solution coefficients / s_i
    __device__ int cs() const { return 4 * M + 3; }         // M   rotation cosines
    __device__ int sn() const { return 5 * M + 3; }         // M   rotation sines
    __device__ int R() const { return 6 * M + 3; }          // (M+1) x M, row i at i*M
    __device__ int beta() const { return 6 * M + 3 + (M + 1) * M; }
    __device__ int steps() const { return beta() + 1; }
    __device__ int active() const { return beta() + 2; }
};

__device__ __forceinline__ double *rec(double *gm, const GmArgs &a, int k, int b) {
    return gm + ((long long)k * a.nblocks + b) * a.rec_stride;
}

// The whole block's tile partials of slot `slot` (FP64), summed by the 64
// lanes of one wavefront: lane l adds tiles l, l+64, ... in order, then a
// butterfly; a fixed order, and every lane gets the sum.
template <typename T>
__device__ __forceinline__ double block_sum(const T *part, long long stride, int slot,
                                            int tile0, int ntiles) {
    double s = 0.0;
    for (int t = threadIdx.x & 63; t < ntiles; t += 64)
        s += (double)part[(long long)(tile0 + t) * stride + slot];
    return wave_sum(s);
}

// Dot products reduced together (one workgroup barrier per batch).
constexpr int kDotBatch = 8;

// w = A_box u (zero outside the box; overlap: zero outside the region)
// times inv_s, on one tile of one-row threads; w kept in wv and stored.
template <typename T, int VZ, bool OVL>
__device__ __forceinline__ void tile_gm_apply(const Tile &t, long long goff,
                                              const T *__restrict__ u, T *__restrict__ w,
                                              T inv_s, T (&wv)[kGmPlanes][VZ]) {
    const int bz = t.B.bz, by = t.B.by, bx = t.B.bx;
    const long long P = (long long)by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const bool live = t.nrows > 0;
    const bool zm_in = t.zc > 0, zp_in = t.zc < t.tpr - 1;
    const bool zm_sh = zm_in && t.lane > 0, zp_sh = zp_in && t.lane < 63;
    const bool ym_ld = live && t.j0 > 0;
    const bool yp_ld = live && t.j0 + 1 < by;
    const bool ym_sh = t.lane >= t.tpr, yp_sh = t.lane + t.tpr < 64;
    T pm[VZ], pc[VZ], pp[VZ];
#pragma unroll
    for (int v = 0; v < VZ; v++) { pm[v] = T(0); pc[v] = T(0); pp[v] = T(0); }
    if (live) {
        if (t.xbeg > 0) vload<T, VZ>(u + base + (long long)(t.xbeg - 1) * P, pm);
        vload<T, VZ>(u + base + (long long)t.xbeg * P, pc);
    }
#pragma unroll
    for (int q = 0; q < kGmPlanes; q++) {
#pragma unroll
        for (int v = 0; v < VZ; v++) wv[q][v] = T(0);
        const int i = t.xbeg + q;
        if (i >= t.xend) continue;   // uniform over the workgroup
        const long long o = base + (long long)i * P;
        T ym[VZ], yp[VZ], ysu[VZ], ysd[VZ];
#pragma unroll
        for (int v = 0; v < VZ; v++) {
            ym[v] = T(0);
            yp[v] = T(0);
            ysu[v] = __shfl_up(pc[v], t.tpr, 64);
            ysd[v] = __shfl_down(pc[v], t.tpr, 64);
        }
        if (live && i + 1 < bx) vload<T, VZ>(u + o + P, pp);
        if (ym_ld) {
            if (ym_sh) {
#pragma unroll
                for (int v = 0; v < VZ; v++) ym[v] = ysu[v];
            } else {
                vload<T, VZ>(u + o - bz, ym);
            }
        }
        if (yp_ld) {
            if (yp_sh) {
#pragma unroll
                for (int v = 0; v < VZ; v++) yp[v] = ysd[v];
            } else {
                vload<T, VZ>(u + o + bz, yp);
            }
        }
        const T sl = from_left(pc[VZ - 1]);
        const T sr = from_right(pc[0]);
        if (live) {
            T zm = T(0), zp = T(0);
            if (zm_in) zm = zm_sh ? sl : u[o - 1];
            if (zp_in) zp = zp_sh ? sr : u[o + VZ];
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[v - 1];
                const T right = v == VZ - 1 ? zp : pc[v + 1];
                T qv = (T(6) * pc[v] - pm[v] - pp[v] - ym[v] - yp[v] - left - right) * inv_s;
                if (OVL && axes_out(t.B, i, t.j0, t.k + v) > 1) qv = T(0);
                wv[q][v] = qv;
            }
            vstore<T, VZ>(w + o, wv[q]);
        }
#pragma unroll
        for (int v = 0; v < VZ; v++) { pm[v] = pc[v]; pc[v] = pp[v]; pp[v] = T(0); }
    }
}

// Tile partials of (w, u_i), i = 0..j, from the w values of one tile (wv),
// reduced over the NT threads of the workgroup kDotBatch dots at a time.
// Thread c < kDotBatch then stores (ADD: adds) dot i0 + c to out[i0 + c].
// Threads of an idle tile (live = false) contribute zeros but take part.
template <typename T, int VZ, int NT, bool ADD, typename O>
__device__ __forceinline__ void gm_dots(const Tile &t, bool live, long long goff, const T *V,
                                        long long kvs, long long ko, int j,
                                        const T (&wv)[kGmPlanes][VZ], T (*sh)[kDotBatch],
                                        O *out) {
    const int bz = t.B.bz;
    const long long P = (long long)t.B.by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    for (int i0 = 0; i0 <= j; i0 += kDotBatch) {
        T acc[kDotBatch];
#pragma unroll
        for (int c = 0; c < kDotBatch; c++) acc[c] = T(0);
        if (live && t.nrows > 0) {
#pragma unroll
            for (int c = 0; c < kDotBatch; c++) {
                if (i0 + c > j) continue;
                const T *ui = V + (long long)(i0 + c) * kvs + ko + base;
#pragma unroll
                for (int q = 0; q < kGmPlanes; q++) {
                    if (t.xbeg + q >= t.xend) continue;
                    T uv[VZ];
                    vload<T, VZ>(ui + (long long)(t.xbeg + q) * P, uv);
#pragma unroll
                    for (int v = 0; v < VZ; v++) acc[c] += wv[q][v] * uv[v];
                }
            }
        }
        // lanes by butterfly, then the wavefronts in order
#pragma unroll
        for (int c = 0; c < kDotBatch; c++) {
            const T sv = wave_sum(acc[c]);
            if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][c] = sv;
        }
        __syncthreads();
        if (threadIdx.x < kDotBatch && i0 + (int)threadIdx.x <= j) {
            T sv = T(0);
#pragma unroll
            for (int w = 0; w < NT / 64; w++) sv += sh[w][threadIdx.x];
            if (ADD) out[i0 + threadIdx.x] += (O)sv;
            else out[i0 + threadIdx.x] = (O)sv;
        }
        __syncthreads();
    }
}

// u_{j+1} = w - sum_i coef[i] u_i on one tile; returns the thread's part of
// ||u_{j+1}||^2.
template <typename T, int VZ>
__device__ __forceinline__ T tile_gm_orth(const Tile &t, long long goff, T *V, long long kvs,
                                          long long ko, int j, const double *coef) {
    T *un = V + (long long)(j + 1) * kvs + ko;
    const int bz = t.B.bz;
    const long long P = (long long)t.B.by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    T wv[kGmPlanes][VZ];
    const bool live = t.nrows > 0;
#pragma unroll
    for (int q = 0; q < kGmPlanes; q++) {
#pragma unroll
        for (int v = 0; v < VZ; v++) wv[q][v] = T(0);
        if (live && t.xbeg + q < t.xend) vload<T, VZ>(un + base + (long long)(t.xbeg + q) * P, wv[q]);
    }
    for (int i = 0; i <= j; i++) {
        const T c = (T)coef[i];
        const T *ui = V + (long long)i * kvs + ko;
        if (!live) continue;
#pragma unroll
        for (int q = 0; q < kGmPlanes; q++) {
            if (t.xbeg + q >= t.xend) continue;
            T uv[VZ];
            vload<T, VZ>(ui + base + (long long)(t.xbeg + q) * P, uv);
#pragma unroll
            for (int v = 0; v < VZ; v++) wv[q][v] = wv[q][v] - c * uv[v];
        }
    }
    T acc = T(0);
    if (live) {
#pragma unroll
        for (int q = 0; q < kGmPlanes; q++) {
            if (t.xbeg + q >= t.xend) continue;
            vstore<T, VZ>(un + base + (long long)(t.xbeg + q) * P, wv[q]);
#pragma unroll
            for (int v = 0; v < VZ; v++) acc += wv[q][v] * wv[q][v];
        }
    }
    return acc;
}

// xb = xa + sum_{l < n} c[l] u_l on the tile's own cells (xb may be xa).
template <typename T, int VZ, bool OVL>
__device__ __forceinline__ void tile_gm_final(const Geom &g, const Tile &t, long long goff,
                                              const T *V, long long kvs, long long ko,
                                              const double *c, int n, const double *xa,
                                              double *xb) {
    if (t.nrows == 0) return;
    const int bz = t.B.bz;
    const long long P = (long long)t.B.by * bz;
    const long long base = (t.B.off - goff) + (long long)t.j0 * bz + t.k;
    const long long J = t.B.j0 + t.j0, K = t.B.k0 + t.k;
    // planes of this thread that hold own cells (all of them without overlap)
    bool mine[kGmPlanes];
    double xv[kGmPlanes][VZ];
#pragma unroll
    for (int q = 0; q < kGmPlanes; q++) {
        const int i = t.xbeg + q;
        mine[q] = i < t.xend && !(OVL && axes_out(t.B, i, t.j0, t.k) != 0);
        if (mine[q]) vload<double, VZ>(xa + ((long long)(t.B.i0 + i) * g.ny + J) * g.nz + K, xv[q]);
    }
    for (int l = 0; l < n; l++) {
        const double cl = c[l];
        const T *ul = V + (long long)l * kvs + ko + base;
#pragma unroll
        for (int q = 0; q < kGmPlanes; q++) {
            if (!mine[q]) continue;
            T uv[VZ];
            vload<T, VZ>(ul + (long long)(t.xbeg + q) * P, uv);
#pragma unroll
            for (int v = 0; v < VZ; v++) xv[q][v] += cl * (double)uv[v];
        }
    }
#pragma unroll
    for (int q = 0; q < kGmPlanes; q++)
        if (mine[q])
            vstore<double, VZ>(xb + ((long long)(t.B.i0 + t.xbeg + q) * g.ny + J) * g.nz + K, xv[q]);
}

// Givens step of Arnoldi step j for one block record (one thread): the
// rotations of column j with h_{j+1,j} = hn, the least-squares residual and
// the stopping rules.  Returns -1 when the step cannot be taken (nothing
// left to reduce), 0 when it was taken and the block stops, 1 when it was
// taken and the block goes on.
__device__ __forceinline__ int gm_givens(double *st, const GmRec &R, int M, int j, double hn,
                                         double inner_tol) {
    double *H = st + R.R();
    for (int i = 0; i < j; i++) {
        const double x0 = H[i * M + j], x1 = H[(i + 1) * M + j];
        const double c = st[R.cs() + i], s = st[R.sn() + i];
        H[i * M + j] = c * x0 + s * x1;
        H[(i + 1) * M + j] = -s * x0 + c * x1;
    }
    const double d = H[j * M + j];
    const double den = sqrt(d * d + hn * hn);
    if (!(den > 0.0)) {          // nothing left to reduce
        st[R.active()] = 0.0;
        return -1;
    }
    const double c = d / den, s = hn / den;
    st[R.cs() + j] = c;
    st[R.sn() + j] = s;
    H[j * M + j] = den;
    const double gj = st[R.g() + j];
    st[R.g() + j + 1] = -s * gj;
    st[R.g() + j] = c * gj;
    st[R.steps()] = (double)(j + 1);
    if (!(hn > 0.0)) {
        st[R.active()] = 0.0;   // invariant Krylov space: the block is solved
        return 0;
    }
    st[R.s() + j + 1] = hn;
    if (inner_tol > 0.0 && fabs(st[R.g() + j + 1]) <= inner_tol * st[R.beta()]) {
        st[R.active()] = 0.0;
        return 0;
    }
    return 1;
}

// y from the triangular system of a block record (one thread), stored as
// y_i / s_i into c[0..n) (c may be the record's y field).
__device__ __forceinline__ void gm_backsolve(const double *st, const GmRec &R, int M, int n,
                                             double *c) {
    const double *H = st + R.R();
    for (int i = n - 1; i >= 0; i--) {
        double s = st[R.g() + i];
        for (int l = i + 1; l < n; l++) s -= H[i * M + l] * c[l];
        c[i] = s / H[i * M + i];
    }
    for (int i = 0; i < n; i++) c[i] /= st[R.s() + i];
}

}  // namespace

// The per-block kernels below run one 64-lane workgroup per (right-hand
// side, block of the group); lane 0 does the scalar work.

// Start of a block's GMRES cycle: beta = ||r|| from the residual kernel's
// region partials.
template <typename T>
__global__ __launch_bounds__(64) void k_gm_init(const BlockInfo *blocks, int b0, int nb,
                                                const T *pT, Batch bt, GmArgs a, Ctrl *ctrl) {
    const int k = blockIdx.x / nb, b = b0 + blockIdx.x % nb;
    if (ctrl[k].done) return;
    const BlockInfo &B = blocks[b];
    const GmRec R{a.M};
    double *st = rec(a.gm, a, k, b);
    const double beta = sqrt(block_sum(pT + (long long)k * bt.ps, 1, 0, B.tile0, B.ntiles));
    if (threadIdx.x != 0) return;
    st[R.s()] = beta;
    st[R.g()] = beta;
    st[R.beta()] = beta;
    st[R.steps()] = 0.0;
    st[R.active()] = beta > 0.0 ? 1.0 : 0.0;   // a zero residual has nothing to solve
}

// Arnoldi step j, part 1: u_{j+1} = A v_j and partials of (u_{j+1}, u_i).
template <typename T, int VZ, bool OVL>
__global__ __launch_bounds__(kThreads) void k_gm_apply(Geom g, int t0, long long goff, T *V,
                                                       int j, Batch bt, GmArgs a, Ctrl *ctrl) {
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int k = w / bt.nt;
    if (ctrl[k].done) return;
    const int tile = t0 + (w - k * bt.nt);
    const Tile t = decode_tile<VZ, 1>(g, tile, threadIdx.x);
    const GmRec R{a.M};
    const double *st = rec(a.gm, a, k, t.b);
    if (st[R.active()] == 0.0) return;   // uniform over the workgroup
    const long long ko = (long long)k * bt.is;
    T wv[kGmPlanes][VZ];
    tile_gm_apply<T, VZ, OVL>(t, goff, V + (long long)j * a.kvs + ko,
                              V + (long long)(j + 1) * a.kvs + ko, T(1.0 / st[R.s() + j]), wv);
    __shared__ T sh[kThreads / 64][kDotBatch];
    gm_dots<T, VZ, kThreads, false>(t, true, goff, V, a.kvs, ko, j, wv, sh,
                                    a.gpart + ((long long)k * bt.ps + tile) * a.gstride);
}

// Arnoldi step j, part 2: h_ij = (w, u_i) / s_i, i <= j, from the block's
// tile partials (every workgroup of the block sums them in the same fixed
// order, each wavefront every fourth coefficient; the block's first tile
// records them), then u_{j+1} = w - sum_i (h_ij / s_i) u_i and partials of
// its squared norm.
template <typename T, int VZ>
__global__ __launch_bounds__(kThreads) void k_gm_orth(Geom g, int t0, long long goff, T *V, int j,
                                                      Batch bt, GmArgs a, Ctrl *ctrl) {
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int k = w / bt.nt;
    if (ctrl[k].done) return;
    const int tile = t0 + (w - k * bt.nt);
    const Tile t = decode_tile<VZ, 1>(g, tile, threadIdx.x);
    const GmRec R{a.M};
    double *st = rec(a.gm, a, k, t.b);
    if (st[R.active()] == 0.0) return;
    __shared__ double coef[kGmMaxSteps];
    const double *part = a.gpart + (long long)k * bt.ps * a.gstride;
    for (int i = (int)threadIdx.x >> 6; i <= j; i += kThreads / 64) {
        const double h = block_sum(part, a.gstride, i, t.B.tile0, t.B.ntiles) / st[R.s() + i];
        if ((threadIdx.x & 63) == 0) {
            coef[i] = h / st[R.s() + i];
            if (t.first) {
                st[R.R() + i * a.M + j] = h;
                st[R.coef() + i] = coef[i];
            }
        }
    }
    __syncthreads();
    const T acc = tile_gm_orth<T, VZ>(t, goff, V, a.kvs, (long long)k * bt.is, j, coef);
    const T s = wg_allsum<T, kThreads>(acc);
    if (threadIdx.x == 0) a.gpart[((long long)k * bt.ps + tile) * a.gstride + a.M + 1] = (double)s;
}

// Arnoldi step j, part 3 (per block): h_{j+1,j} = ||u_{j+1}||, Givens
// rotations of column j, least-squares residual and the stopping rules
// (m steps, inner_tol, an invariant Krylov space).
__global__ __launch_bounds__(64) void k_gm_norm(const BlockInfo *blocks, int b0, int nb, int j,
                                                double inner_tol, Batch bt, GmArgs a,
                                                Ctrl *ctrl) {
    const int k = blockIdx.x / nb, b = b0 + blockIdx.x % nb;
    if (ctrl[k].done) return;
    const GmRec R{a.M};
    double *st = rec(a.gm, a, k, b);
    if (st[R.active()] == 0.0) return;
    const BlockInfo &B = blocks[b];
    const double *part = a.gpart + (long long)k * bt.ps * a.gstride;
    const double hn = sqrt(block_sum(part, a.gstride, a.M + 1, B.tile0, B.ntiles));
    if (threadIdx.x != 0) return;
    if (gm_givens(st, R, a.M, j, hn, inner_tol) >= 0) atomicAdd(&ctrl[k].inner_iters, 1ull);
}

// End of the cycle (per block): y from the triangular system, stored as
// y_i / s_i, the coefficient of u_i in the correction.
__global__ void k_gm_solve(int b0, int nb, Batch bt, GmArgs a, Ctrl *ctrl) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nb * bt.nrhs) return;
    const int k = q / nb, b = b0 + q % nb;
    if (ctrl[k].done) return;
    const GmRec R{a.M};
    double *st = rec(a.gm, a, k, b);
    gm_backsolve(st, R, a.M, (int)st[R.steps()], st + R.y());
}

// x_new = x_old + sum_i (y_i / s_i) u_i on the block's own cells (every own
// cell is written, also for blocks that took no step).
template <typename T, int VZ, bool OVL>
__global__ __launch_bounds__(kThreads) void k_gm_final(Geom g, int t0, long long goff,
                                                       const T *V, const double *xa, double *xb,
                                                       Batch bt, GmArgs a, Ctrl *ctrl) {
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int k = w / bt.nt;
    if (ctrl[k].done) return;
    const int tile = t0 + (w - k * bt.nt);
    const Tile t = decode_tile<VZ, 1>(g, tile, threadIdx.x);
    const GmRec R{a.M};
    const double *st = rec(a.gm, a, k, t.b);
    tile_gm_final<T, VZ, OVL>(g, t, goff, V, a.kvs, (long long)k * bt.is, st + R.y(),
                              (int)st[R.steps()], xa + k * bt.vs, xb + k * bt.vs);
}

// ----------------------------------------------------------------------
// asynchronous sweeps with GMRES inner solves
// ----------------------------------------------------------------------

// Persistent worker (kAsyncGmThreads threads): takes one block at a time like
// the CG worker (staleness-bounded, latest values in memory, Sections 2.1
// and 2.3), runs a GMRES(m) cycle on it with the Arnoldi dots reduced inside
// the workgroup, and updates the block's own cells of x in place.  Block
// records of right-hand side 0 hold the Hessenberg/Givens state.
template <typename T, int VZ, bool OVL>
__global__ __launch_bounds__(kAsyncGmThreads) void k_async_gmres(
    Geom g, const double *__restrict__ b, double *x, Faces F, T *V, AsyncState as, int m, int S,
    int max_sweeps, double tol2, double inner_tol, GmArgs a, Ctrl *ctrl) {
    constexpr int kSubs = kAsyncGmThreads / kThreads;
    __shared__ AsyncShared sh;
    __shared__ T red[kAsyncGmThreads / 64][kDotBatch];
    __shared__ double sdot[kGmMaxSteps + 2];
    __shared__ double scoef[kGmMaxSteps + 1];
    __shared__ int sflag;
    const int tid = threadIdx.x;
    const int sub = tid / kThreads;
    const int ltid = tid % kThreads;
    const int nb = g.nblocks;
    const GmRec R{a.M};
    for (;;) {
        const int blk = async_claim<kAsyncGmThreads>(g, as, S, max_sweeps, ctrl, sh);
        if (blk == -2) return;
        if (blk < 0) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        const BlockInfo B = g.blocks[blk];
        double *st = rec(a.gm, a, 0, blk);
        // residual of the block's region, stored as u_0
        double acc64 = 0.0;
        T accT = T(0);
        for (int lt = sub; lt < B.ntiles; lt += kSubs) {
            const Tile t = decode_tile<VZ, 1>(g, B.tile0 + lt, ltid);
            tile_resid<T, VZ, 1, true, OVL>(g, t, 0, b, x, F, V, acc64, accT);
        }
        const double res2 = wg_allsum<double, kAsyncGmThreads>(acc64);
        const double beta = sqrt((double)wg_allsum<T, kAsyncGmThreads>(accT));
        if (tid == 0) {
            __hip_atomic_store(&as.board[blk], res2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st[R.s()] = beta;
            st[R.g()] = beta;
            st[R.beta()] = beta;
            st[R.steps()] = 0.0;
            st[R.active()] = beta > 0.0 ? 1.0 : 0.0;
            sflag = beta > 0.0 ? 1 : 0;
        }
        __syncthreads();
        for (int j = 0; j < m && sflag; j++) {
            // w = A v_j into u_{j+1}, dots with u_0..u_j summed over the tiles
            if (tid <= j) sdot[tid] = 0.0;
            __syncthreads();
            const T inv_s = T(1.0 / st[R.s() + j]);
            for (int l0 = 0; l0 < B.ntiles; l0 += kSubs) {
                const int lt = l0 + sub;
                const bool live = lt < B.ntiles;
                const Tile t = decode_tile<VZ, 1>(g, B.tile0 + (live ? lt : 0), ltid);
                T wv[kGmPlanes][VZ];
#pragma unroll
                for (int q = 0; q < kGmPlanes; q++)
#pragma unroll
                    for (int v = 0; v < VZ; v++) wv[q][v] = T(0);
                if (live)
                    tile_gm_apply<T, VZ, OVL>(t, 0, V + (long long)j * a.kvs,
                                              V + (long long)(j + 1) * a.kvs, inv_s, wv);
                gm_dots<T, VZ, kAsyncGmThreads, true>(t, live, 0, V, a.kvs, 0, j, wv, red, sdot);
            }
            if (tid == 0)
                for (int i = 0; i <= j; i++) {
                    const double h = sdot[i] / st[R.s() + i];
                    st[R.R() + i * a.M + j] = h;
                    scoef[i] = h / st[R.s() + i];
                }
            __syncthreads();
            // classical Gram-Schmidt and the new norm
            T nacc = T(0);
            for (int lt = sub; lt < B.ntiles; lt += kSubs) {
                const Tile t = decode_tile<VZ, 1>(g, B.tile0 + lt, ltid);
                nacc += tile_gm_orth<T, VZ>(t, 0, V, a.kvs, 0, j, scoef);
            }
            const double hn = sqrt((double)wg_allsum<T, kAsyncGmThreads>(nacc));
            if (tid == 0) sflag = gm_givens(st, R, a.M, j, hn, inner_tol) > 0 ? 1 : 0;
            __syncthreads();
        }
        const int n = (int)st[R.steps()];
        if (tid == 0) gm_backsolve(st, R, a.M, n, scoef);
        __syncthreads();
        if (n > 0) {
            for (int lt = sub; lt < B.ntiles; lt += kSubs) {
                const Tile t = decode_tile<VZ, 1>(g, B.tile0 + lt, ltid);
                tile_gm_final<T, VZ, OVL>(g, t, 0, V, a.kvs, 0, scoef, n, x, x);
            }
        }
        async_publish(as, blk, max_sweeps, n, tol2, ctrl, sh, nb);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------

#define GM_CASE(vz_, ...)                     \
    case vz_: {                               \
        constexpr int VZ = vz_;               \
        __VA_ARGS__;                          \
        break;                                \
    }
#define GM_DISPATCH(vz, ...)                                                        \
    switch (vz) {                                                                   \
        GM_CASE(1, __VA_ARGS__) GM_CASE(2, __VA_ARGS__) GM_CASE(4, __VA_ARGS__)     \
        default: return hipErrorInvalidValue;                                       \
    }

// one thread per (right-hand side, block)
static inline dim3 small_grid(int nb, int nrhs) {
    return dim3((unsigned)((nb * nrhs + 63) / 64));
}

// one 64-lane workgroup per (right-hand side, block)
static inline dim3 wave_grid(int nb, int nrhs) { return dim3((unsigned)(nb * nrhs)); }

static inline dim3 gm_batch_grid(int t0, int t1, Batch &bt) {
    bt.nt = t1 - t0;
    return dim3((unsigned)((long long)bt.nt * bt.nrhs));
}

template <typename T>
hipError_t launch_gm_init(const Geom &g, int b0, int b1, const T *pT, Batch bt, GmArgs a,
                          Ctrl *ctrl, hipStream_t st) {
    if (b1 <= b0) return hipSuccess;
    launch(k_gm_init<T>, wave_grid(b1 - b0, bt.nrhs), dim3(64), 0, st, g.blocks,
                       b0, b1 - b0, pT, bt, a, ctrl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gm_step(const Geom &g, int vz, int t0, int t1, int b0, int b1, long long goff,
                          T *V, int j, double inner_tol, Batch bt, GmArgs a, Ctrl *ctrl,
                          hipStream_t st, int part) {
    if (t1 <= t0) return hipSuccess;
    if (g.rows != 1 || g.tx > kGmPlanes) return hipErrorInvalidValue;
    if (part == 0) {
        const dim3 grid = gm_batch_grid(t0, t1, bt);
        if (g.ovl) {
            GM_DISPATCH(vz, launch((k_gm_apply<T, VZ, true>), grid, dim3(kThreads),
                                               0, st, g, t0, goff, V, j, bt, a, ctrl));
        } else {
            GM_DISPATCH(vz, launch((k_gm_apply<T, VZ, false>), grid, dim3(kThreads),
                                               0, st, g, t0, goff, V, j, bt, a, ctrl));
        }
    } else if (part == 1) {
        const dim3 grid = gm_batch_grid(t0, t1, bt);
        GM_DISPATCH(vz, launch((k_gm_orth<T, VZ>), grid, dim3(kThreads), 0, st, g,
                                           t0, goff, V, j, bt, a, ctrl));
    } else {
        launch(k_gm_norm, wave_grid(b1 - b0, bt.nrhs), dim3(64), 0, st, g.blocks, b0,
                           b1 - b0, j, inner_tol, bt, a, ctrl);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gm_finish(const Geom &g, int vz, int t0, int t1, int b0, int b1,
                            long long goff, const T *V, const double *xa, double *xb, Batch bt,
                            GmArgs a, Ctrl *ctrl, hipStream_t st, int part) {
    if (t1 <= t0) return hipSuccess;
    if (g.rows != 1 || g.tx > kGmPlanes) return hipErrorInvalidValue;
    if (part == 0) {
        launch(k_gm_solve, small_grid(b1 - b0, bt.nrhs), dim3(64), 0, st, b0,
                           b1 - b0, bt, a, ctrl);
    } else {
        const dim3 grid = gm_batch_grid(t0, t1, bt);
        if (g.ovl) {
            GM_DISPATCH(vz, launch((k_gm_final<T, VZ, true>), grid, dim3(kThreads),
                                               0, st, g, t0, goff, V, xa, xb, bt, a, ctrl));
        } else {
            GM_DISPATCH(vz, launch((k_gm_final<T, VZ, false>), grid, dim3(kThreads),
                                               0, st, g, t0, goff, V, xa, xb, bt, a, ctrl));
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_async_gmres(const Geom &g, int vz, int grid, const double *b, double *x,
                              Faces faces, T *V, AsyncState as, int m, int S, int max_sweeps,
                              double tol2, double inner_tol, GmArgs a, Ctrl *ctrl,
                              hipStream_t st) {
    if (grid < 1 || g.rows != 1 || g.tx > kGmPlanes || a.M > kGmMaxSteps)
        return hipErrorInvalidValue;
    if (g.ovl) {
        GM_DISPATCH(vz, launch((k_async_gmres<T, VZ, true>), dim3(grid),
                                           dim3(kAsyncGmThreads), 0, st, g, b, x, faces, V, as, m,
                                           S, max_sweeps, tol2, inner_tol, a, ctrl));
    } else {
        GM_DISPATCH(vz, launch((k_async_gmres<T, VZ, false>), dim3(grid),
                                           dim3(kAsyncGmThreads), 0, st, g, b, x, faces, V, as, m,
                                           S, max_sweeps, tol2, inner_tol, a, ctrl));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t async_gmres_occupancy(int vz, int ovl, int *per_cu) {
    *per_cu = 0;
    if (ovl) {
        GM_DISPATCH(vz, return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            per_cu, (const void *)k_async_gmres<T, VZ, true>, kAsyncGmThreads, 0));
    } else {
        GM_DISPATCH(vz, return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            per_cu, (const void *)k_async_gmres<T, VZ, false>, kAsyncGmThreads, 0));
    }
    return hipSuccess;
}

int gm_record_doubles(int M) { return 6 * M + 3 + (M + 1) * M + 4; }
int gm_max_planes() { return kGmPlanes; }

#define GM_INST(T)                                                                            \
    template hipError_t launch_gm_init<T>(const Geom &, int, int, const T *, Batch, GmArgs,   \
                                          Ctrl *, hipStream_t);                               \
    template hipError_t launch_gm_step<T>(const Geom &, int, int, int, int, int, long long,   \
                                          T *, int, double, Batch, GmArgs, Ctrl *,            \
                                          hipStream_t, int);                                  \
    template hipError_t launch_gm_finish<T>(const Geom &, int, int, int, int, int, long long, \
                                            const T *, const double *, double *, Batch,      \
                                            GmArgs, Ctrl *, hipStream_t, int);                \
    template hipError_t launch_async_gmres<T>(const Geom &, int, int, const double *,         \
                                              double *, Faces, T *, AsyncState, int, int, int, \
                                              double, double, GmArgs, Ctrl *, hipStream_t);   \
    template hipError_t async_gmres_occupancy<T>(int, int, int *);
GM_INST(double)
GM_INST(float)

}  // namespace ms
