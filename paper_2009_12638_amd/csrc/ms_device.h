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

}  // namespace ms
