// Device helpers shared by the HIP sources of libms: vector loads and
// stores, wavefront and workgroup sums, fixed-order tile sums, the thread
// geometry of a tile, the XCD-aware workgroup order and the overlap mask.
// Not part of the public ABI.
#pragma once
#include "ms_internal.h"

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

// Sum over the NT threads of the workgroup, returned to every thread.
// Fixed shape: lanes by butterfly, then the wavefront sums in order.
template <typename T, int NT>
__device__ __forceinline__ T wg_allsum(T v) {
    __shared__ T sh[NT / 64 + 1];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = T(0);
#pragma unroll
        for (int w = 0; w < NT / 64; w++) s += sh[w];
        sh[NT / 64] = s;
    }
    __syncthreads();
    const T s = sh[NT / 64];
    __syncthreads();   // sh may be reused by the next call
    return s;
}

// Sum of a block's tile partials in tile order (every thread computes it).
template <typename T>
__device__ __forceinline__ T tiles_sum(const T *__restrict__ part, int t0, int n) {
    T s = T(0);
    for (int t = 0; t < n; t++) s += part[t0 + t];
    return s;
}

// Thread geometry inside a tile.  A thread owns R consecutive rows (y) of
// VZ consecutive z cells; tpr = bz / VZ threads cover one z row, so lanes
// next to each other hold z neighbours and one wavefront covers whole rows
// whenever tpr divides 64.  Row groups of R rows are numbered g, the
// thread's slot in the block plane is q = g * tpr + zc.
struct Tile {
    int b;             // block number
    BlockInfo B;
    bool live;         // thread owns cells
    int j0;            // first row of the thread's row group
    int nrows;         // rows owned (R, fewer in a partial last group, 0 if idle)
    int k;             // first z of the thread's cells
    int zc, tpr;       // z chunk of the thread, chunks per row
    int xbeg, xend;    // planes marched
    bool first;        // first tile of its block
    int lane;
};

// ltid: thread index inside the 256-thread tile.
template <int VZ, int R>
__device__ __forceinline__ Tile decode_tile(const Geom &g, int tile, int ltid) {
    Tile t;
    t.b = g.tile_block[tile];
    t.B = g.blocks[t.b];
    const int local = tile - t.B.tile0;
    const int pt = local % t.B.nplane;
    const int xc = local / t.B.nplane;
    t.tpr = t.B.bz / VZ;
    const int ng = (t.B.by + R - 1) / R;
    const int q = pt * kThreads + ltid;
    t.live = q < ng * t.tpr;
    const int qq = t.live ? q : 0;
    t.zc = qq % t.tpr;
    t.j0 = (qq / t.tpr) * R;
    t.k = t.zc * VZ;
    t.nrows = t.live ? min(R, t.B.by - t.j0) : 0;
    t.xbeg = xc * g.tx;
    t.xend = min(t.B.bx, t.xbeg + g.tx);
    t.first = (local == 0);
    t.lane = ltid & 63;
    return t;
}

template <typename T>
__device__ __forceinline__ T from_left(T v) { return __shfl_up(v, 1, 64); }
template <typename T>
__device__ __forceinline__ T from_right(T v) { return __shfl_down(v, 1, 64); }

// Workgroups of a launch are dispatched to the XCDs in turn (workgroup w to
// XCD w % 8).  Hand each XCD one contiguous range of tiles instead, so the
// tiles of a block and of its z and y neighbours share that XCD's L2 and
// the halo rows and planes they exchange are L2 hits.  A bijection on
// [0, n) for any n; correctness does not depend on the dispatch order.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int w, int n) {
    const int q = n / kXcds, rem = n % kXcds;
    const int c = w % kXcds, k = w / kXcds;
    return c * q + min(c, rem) + k;
}

// Overlap regions (Section 3.2, block overlap): where box-local cell
// (i, j, k) lies.  0: an own cell; 1: in a face slab of the region (outside
// the own cells along one axis, by at most the overlap depth); 2 or more:
// outside the region (an edge or corner of the box, or beyond the depth in
// z where the box is grown further for alignment), kept at zero in r, d, p.
__device__ __forceinline__ int axes_out(const BlockInfo &B, int i, int j, int k) {
    const int zfar = (k < B.ok - B.dep) || (k >= B.ok + B.obz + B.dep);
    return ((unsigned)(i - B.oi) >= (unsigned)B.obx) + ((unsigned)(j - B.oj) >= (unsigned)B.oby) +
           ((unsigned)(k - B.ok) >= (unsigned)B.obz) + 2 * zfar;
}


// ---- asynchronous sweeps: choosing and publishing blocks ---------------
// (shared by the CG and GMRES workers; every thread of the workgroup calls
// these)

struct AsyncShared {
    int blk;
    int gap;
    int ver;      // version of the claimed block when it was claimed
    unsigned long long key[kAsyncThreads / 64];
};

// The eligible unclaimed block with the lowest version (every neighbour at
// least version + 1 - S), claimed by compare-and-swap; the neighbours'
// published x values are acquired.  Returns the block, -1 when nothing is
// eligible right now, -2 once the worker should exit (stop flag, or every
// block reached the launch's sweep limit).  sh.gap: the largest version gap
// to a neighbour this sweep will see.
// NT: threads of the calling workgroup (at most kAsyncThreads).
template <int NT>
__device__ __forceinline__ int async_claim(const Geom &g, AsyncState as, int S, int max_sweeps,
                                           Ctrl *ctrl, AsyncShared &sh) {
    static_assert(NT <= kAsyncThreads && NT % 64 == 0, "workgroup size");
    const int tid = threadIdx.x;
    const int nb = g.nblocks;
    // ---- the eligible unclaimed block with the lowest version ----
    unsigned long long best = ~0ull;
    for (int c = tid; c < nb; c += NT) {
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
    if ((tid & 63) == 0) sh.key[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        unsigned long long k = ~0ull;
        for (int w = 0; w < NT / 64; w++) k = sh.key[w] < k ? sh.key[w] : k;
        int pick = -1;
        if (__hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            k = ~0ull;       // the residual estimate is below tol: start nothing new
        }
        if (k != ~0ull) {
            const int cand = (int)(k & 0xffffffffu);
            int zero = 0;
            if (__hip_atomic_compare_exchange_strong(&as.claim[cand], &zero, 1, __ATOMIC_ACQUIRE,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                // The scan above read versions before the claim: another
                // worker may have swept and released the block since.  With
                // the claim held the block's version is fixed, so test the
                // rule again on fresh values and give the block back if it
                // no longer holds.  The largest version gap to a neighbour
                // this sweep will see is then at most S - 1.
                const int v = __hip_atomic_load(&as.version[cand], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bool ok = v < max_sweeps;
                int gap = 0;
                int seen[6];
                for (int f = 0; f < 6; f++) {
                    const int nbk = as.nbr[cand * 6 + f];
                    seen[f] = -1;
                    if (nbk < 0) continue;
                    const int vn = __hip_atomic_load(&as.version[nbk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    seen[f] = vn;
                    ok = ok && vn >= v + 1 - S;
                    gap = max(gap, v - vn);
                }
                if (ok) {
                    pick = cand;
                    sh.gap = gap;
                    sh.ver = v;
                    if (as.trace) {
                        const int slot = atomicAdd(as.trace_n, 1);
                        if (slot < as.trace_cap) {
                            int *rec = as.trace + (long long)slot * kTraceInts;
                            rec[0] = cand;
                            rec[1] = v;
                            for (int f = 0; f < 6; f++) rec[2 + f] = seen[f];
                        }
                    }
                    // acquire the neighbours' published x values
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                } else {
                    __hip_atomic_store(&as.claim[cand], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if (pick < 0) {
            const bool stop = __hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            const int fin = __hip_atomic_load(as.finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (stop || fin >= nb) pick = -2;
        }
        sh.blk = pick;
    }
    __syncthreads();
    const int blk = sh.blk;
    __syncthreads();
    // debugging aid: a slow block (a bounded wait before each of its sweeps,
    // so its neighbours run ahead up to the staleness bound)
    if (blk >= 0 && blk == as.slow_block)
        for (int q = 0; q < as.slow_sleep; q++) __builtin_amdgcn_s_sleep(127);
    return blk;
}

// After a block's sweep: release its new x, then publish version + 1, the
// inner iterations and the residual estimate (Section 3: an estimate that
// may be some sweeps old) from the latest published block residuals.
__device__ __forceinline__ void async_publish(AsyncState as, int blk, int max_sweeps, int iters,
                                              double tol2, Ctrl *ctrl, const AsyncShared &sh,
                                              int nb) {
    const int tid = threadIdx.x;
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
        atomicMax(&ctrl->max_stale, sh.gap);
    }
    if (tol2 > 0.0) {
        // residual estimate from the latest published block residuals
        // (Section 3: an estimate that may be some sweeps old), summed by
        // the whole workgroup: its threads load the board in parallel
        __shared__ double est_w[kAsyncThreads / 64];
        double e = 0.0;
        for (int q = tid; q < nb; q += (int)blockDim.x)
            e += __hip_atomic_load(&as.board[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        e = wave_sum(e);
        if ((tid & 63) == 0) est_w[tid >> 6] = e;
        __syncthreads();
        if (tid == 0) {
            double est = 0.0;
            for (int w = 0; w < (int)blockDim.x / 64; w++) est += est_w[w];
            if (est <= tol2) __hip_atomic_store(&ctrl->stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();   // est_w is free for the next call
    }
}

}  // namespace ms
