// Resident-team block solves: the inner CG of a block (Section 3: the inner
// Krylov solve of A_ii d = r_i, here CG; Section 3.2: a maximum number of
// inner iterations) carried out by a team of workgroups that keep the
// block's vectors in registers (r, d) and LDS (p) for all m iterations, so
// the inner iterations move no vector through memory; only slab faces
// travel, through the team's L2.
//
// Layout.  One 512-thread workgroup per compute unit (up to 256 registers a
// thread, so a thread can hold many cells); T workgroups of the same XCD
// (read from the hardware XCC id) form a team.  A team takes one block at a
// time.  The block's box is cut along x into T slabs, one per member; a
// member's cells are held as z vectors of VZ cells, thread t owning vectors
// t, t + 512, ..., up to Q of them.  The stencil reads every neighbour from
// the member's p in LDS, which holds, beside the member's planes, a halo
// plane on each side: the neighbouring member's face plane of p (zero at
// the box's edge).
//
// One CG iteration, two team barriers:
//   sigma = p . A p                      -> team sum (barrier 1)
//   alpha; d += alpha p; r -= alpha A p; the member's r face planes to the
//   team; rho' = r . r                   -> team sum (barrier 2, which also
//                                           publishes the r faces)
//   beta; p = r + beta p, and the neighbours' p face planes likewise from
//   their r faces and the previous p faces (the same arithmetic they do).
//
// Synchronisation.  A team shares one L2, so its barrier needs no cache
// writeback or invalidation: a workgroup's stores are complete in L2 once
// it waits for them (s_waitcnt / __syncthreads), the barrier counter is an
// atomic, and what a member reads that another member wrote (faces, partial
// sums, the work item) it reads with agent-scope atomic loads, which bypass
// the per-CU cache.  Dot products are summed per workgroup in a fixed shape
// and the team adds the members' partials in member order, so a block's
// result does not depend on which team solved it.  Every wait is bounded: a
// barrier that does not complete within max_spin polls sets an error code
// and the kernel exits.
#include "ms_internal.h"
#include "ms_device.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace ms {

namespace {

constexpr int kTeamThreads = 512;
constexpr int kSlotGroup = 2;     // vector slots whose loads are scheduled together

// layout of one team's memory (bytes); faces follow at kFaceOff
constexpr int kBarOff = 0;        // int: barrier counter
constexpr int kWorkOff = 128;     // int[2]: work item broadcast (ring)
constexpr int kPartOff = 256;     // double[2][2][32]: partial sums (ring of 2, 2 values)
constexpr int kFaceOff = 1536;    // T faces[members][2][face_stride]: the members' r face planes

__device__ __forceinline__ int ld_acq(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_sh(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_sh(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct TeamCtx {
    char *mem;        // this team's memory
    int member, T;
    int bars;         // barriers this workgroup has passed
    int max_spin;
    int *err;
    int *stop;        // async: set when a barrier fails, so other teams stop claiming
};

// A team barrier gave up: record the error; in async mode also stop every
// team from claiming more blocks (a block this team holds would never be
// published, and teams waiting for it would wait for ever).
__device__ __forceinline__ void team_fail(TeamCtx &c) {
    atomicCAS(c.err, 0, 2);   // 2: team barrier timed out
    if (c.stop) __hip_atomic_store(c.stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Team barrier: returns false (every thread) when it timed out.
__device__ __forceinline__ bool team_sync(TeamCtx &c) {
    __shared__ int ok;
    __syncthreads();   // the workgroup's stores are complete in L2
    c.bars++;
    if (threadIdx.x == 0) {
        int *cnt = (int *)(c.mem + kBarOff);
        __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int target = c.bars * c.T;
        int spins = 0;
        while (ld_acq(cnt) < target && spins < c.max_spin) {
            __builtin_amdgcn_s_sleep(1);
            spins++;
        }
        ok = spins < c.max_spin;
        if (!ok) team_fail(c);
    }
    __syncthreads();
    return ok;
}

// Sum over the team, in member order, of two values summed over the
// workgroup (wave sums, then the waves in order); every thread gets the
// results.  One team barrier: the first wavefront stores the workgroup's
// partials, arrives on the counter, polls it, and then loads every member's
// partials (one per lane) and adds them in member order.  The partial slots
// alternate with the barrier count, so a member writes a slot only after
// every member has read it two barriers earlier.
template <typename A, typename B>
__device__ __forceinline__ bool team_reduce2(TeamCtx &c, A &a, B &b) {
    constexpr int NW = kTeamThreads / 64;
    __shared__ double wsum[2][NW];
    __shared__ double res[2][2];
    __shared__ int ok;
    const A wa = wave_sum(a);
    const B wb = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        wsum[0][threadIdx.x >> 6] = (double)wa;
        wsum[1][threadIdx.x >> 6] = (double)wb;
    }
    __syncthreads();   // also completes the workgroup's global stores
    c.bars++;
    const int slot = c.bars & 1;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        double *part = (double *)(c.mem + kPartOff) + (size_t)slot * 64;
        if (lane == 0) {
            A ma = A(0);
            B mb = B(0);
            for (int w = 0; w < NW; w++) {
                ma += (A)wsum[0][w];
                mb += (B)wsum[1][w];
            }
            part[c.member] = (double)ma;
            part[32 + c.member] = (double)mb;
            __builtin_amdgcn_s_waitcnt(0);   // the partials are in L2 before arriving
            int *cnt = (int *)(c.mem + kBarOff);
            __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int target = c.bars * c.T;
            int spins = 0;
            while (ld_acq(cnt) < target && spins < c.max_spin) spins++;
            ok = spins < c.max_spin;
            if (!ok) team_fail(c);
        }
        // the lanes load the partials once lane 0 has seen every member arrive
        // (the compiler keeps the loads after the poll)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const double va = lane < c.T ? ld_sh(part + lane) : 0.0;
        const double vb = lane < c.T ? ld_sh(part + 32 + lane) : 0.0;
        A sa = A(0);
        B sb = B(0);
        for (int q = 0; q < c.T; q++) {
            sa += (A)__shfl(va, q, 64);
            sb += (B)__shfl(vb, q, 64);
        }
        if (lane == 0) {
            res[slot][0] = (double)sa;
            res[slot][1] = (double)sb;
        }
    }
    __syncthreads();
    a = (A)res[slot][0];
    b = (B)res[slot][1];
    return ok;
}

// The member's slab of the box: planes [lo, hi) along x.
__device__ __forceinline__ void slab(int bx, int T, int member, int &lo, int &hi) {
    lo = (int)(((long long)bx * member) / T);
    hi = (int)(((long long)bx * (member + 1)) / T);
}

}  // namespace

// Sweep kernel.  Sync: every work item is a block of the partition, swept
// from xa into xb (the two outer buffers of the synchronous method); the
// block's own-cell residual of xa goes to p64[block].  Async: blocks are
// claimed under the staleness rule and swept in place (xa == xb).
template <typename T, int VZ, int Q, bool OVL, bool ASYNC>
__global__ __launch_bounds__(kTeamThreads) void k_team(Geom g, TeamArgs a, AsyncState as, int S,
                                                       int max_sweeps, double tol2, Ctrl *ctrl) {
    // 16-byte aligned: p is read with 16-byte LDS accesses
    extern __shared__ __align__(16) char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    __shared__ AsyncShared ash;
    __shared__ int s_blk;
    const int tid = threadIdx.x;
    if (!ASYNC && ctrl->done) return;
    // ---- team of this workgroup ----
    // Every workgroup reads its XCD from the hardware and takes the next
    // position on it; once all have (the launch is cooperative, so all are
    // resident and the wait ends), each XCD's workgroups form
    // floor(count / T) teams in position order and the rest leave.  Only
    // the member number decides a member's part of a block, so the result
    // does not depend on which workgroup got which position.
    __shared__ int s_team, s_member;
    if (tid == 0) {
        s_team = -1;
        const int xcd = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15);   // XCC id
        if (xcd >= kXcds) {
            atomicCAS(a.err, 0, 1);   // 1: an XCD id outside 0..7
        } else {
            const int pos = atomicAdd(a.xcd_count + xcd, 1);
            atomicAdd(a.arrived, 1);
            int spins = 0;
            while (ld_acq(a.arrived) < (int)gridDim.x && spins < a.max_spin) {
                __builtin_amdgcn_s_sleep(1);
                spins++;
            }
            if (spins >= a.max_spin) {
                atomicCAS(a.err, 0, 3);   // 3: not every workgroup arrived
            } else {
                int base = 0, mine = 0;
                for (int q = 0; q < kXcds; q++) {
                    const int teams = ld_acq(a.xcd_count + q) / a.T;
                    if (q < xcd) base += teams;
                    if (q == xcd) mine = teams;
                }
                if (pos < mine * a.T) {
                    s_team = base + pos / a.T;
                    s_member = pos % a.T;
                }
            }
        }
    }
    __syncthreads();
    if (s_team < 0) return;
    TeamCtx c;
    c.T = a.T;
    c.member = s_member;
    c.mem = a.team_mem + (long long)s_team * a.team_bytes;
    c.bars = 0;
    c.max_spin = a.max_spin;
    c.err = a.err;
    c.stop = ASYNC ? &ctrl->stop : nullptr;
    const long long fs = a.face_stride;
    T *faces = reinterpret_cast<T *>(c.mem + kFaceOff);            // [T][2][fs], shared
    int *work = (int *)(c.mem + kWorkOff);
    const long long nx = g.nx, ny = g.ny, nz = g.nz;
    for (int round = 0;; round++) {
        // ---- the next block, chosen by member 0 and passed to the team ----
        if (c.member == 0) {
            int blk;
            if (ASYNC) {
                blk = async_claim<kTeamThreads>(g, as, S, max_sweeps, ctrl, ash);
                if (blk == -1) blk = -3;   // nothing eligible now: the team waits a round
            } else {
                if (tid == 0) s_blk = atomicAdd(a.next, 1);
                __syncthreads();
                blk = s_blk < a.nwork ? s_blk : -2;
                __syncthreads();
            }
            if (tid == 0) work[round & 1] = blk;
        }
        if (!team_sync(c)) return;
        const int blk = ld_acq(work + (round & 1));
        if (blk == -2) return;
        if (blk == -3) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        // async: acquire the x values neighbours published (member 0's claim
        // acquired them for its own caches only)
        if (ASYNC) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const BlockInfo B = g.blocks[blk];
        int lo, hi;
        slab(B.bx, a.T, c.member, lo, hi);
        const int np = hi - lo;
        const int tpr = B.bz / VZ;              // z vectors per row
        const int P = B.by * tpr;               // z vectors per plane
        const int V = np * P;                   // z vectors of this member
        const int PB = B.by * B.bz;             // cells per plane
        // FP64: d in registers (LDS holds p only, so twice the cells fit);
        // FP32: d after p in LDS
        // LDS: the lower halo plane (the previous member's last plane of p,
        // zero at the box's edge), the member's np planes of p, the upper
        // halo plane; d stays in registers with r
        constexpr bool DREG = true;
        T *lp = lds + PB;                         // p of member-local element e at lp[e]
        T *ldd = lp;                              // (d in LDS: unused)
        T *hlo = lds;                             // lower halo plane
        T *hhi = lds + (long long)(np + 1) * PB;  // upper halo plane
        // Vector slot s of this thread is vector tid + s * kTeamThreads of the
        // member; LDS holds the member's cells densely (plane, row, z), so the
        // slot's first element is at vector * VZ = eb + s * 512 * VZ, with
        // eb = tid * VZ taken afresh before each loop over the slots (the
        // empty asm keeps the compiler from hoisting the slots' addresses out
        // of the iteration loop, which would cost registers per slot; inside
        // one loop they are eb plus constants, so the slots' loads can be
        // issued together).  Flags per slot: bit 0..5 the neighbour
        // exists inside the box at -x,+x,-y,+y,-z,+z (x: inside this slab),
        // bit 6/7 the -x/+x neighbour is in a halo plane (another member's
        // slab), bit 8
        // own cells (overlap), bits 9.. cells outside the overlap region.
        const int nE = V * VZ;
        auto E0 = [&]() {
            int e = tid * VZ;
            asm volatile("" : "+v"(e));
            return e;
        };
#define E(s) (eb + (s) * kTeamThreads * VZ)
        int FL[Q];
#pragma unroll
        for (int s = 0; s < Q; s++) {
            const int vi = tid + s * kTeamThreads;
            FL[s] = 0;
            if (vi >= V) continue;
            const int l = vi / P, q = vi % P;
            const int j = q / tpr, k = (q % tpr) * VZ;
            int f = (l > 0) | ((l < np - 1) << 1) | ((j > 0) << 2) | ((j < B.by - 1) << 3) |
                    ((k > 0) << 4) | ((k + VZ < B.bz) << 5);
            if (l == 0 && c.member > 0) f |= 1 << 6;
            if (l == np - 1 && c.member < a.T - 1) f |= 1 << 7;
            if (OVL) {
                if (axes_out(B, lo + l, j, k) == 0) f |= 1 << 8;
#pragma unroll
                for (int v = 0; v < VZ; v++)
                    if (axes_out(B, lo + l, j, k + v) > 1) f |= 1 << (9 + v);
            } else {
                f |= 1 << 8;
            }
            FL[s] = f;
        }
        // ---- residual r = b_eff - A x on the member's cells (FP64); p = r in
        //      LDS, d = 0 ----
        T r[Q][VZ], dr[DREG ? Q : 1][VZ];
#pragma unroll
        for (int s = 0; s < (DREG ? Q : 1); s++)
#pragma unroll
            for (int v = 0; v < VZ; v++) dr[s][v] = T(0);
        double acc64 = 0.0;
        T accT = T(0);
        T *fme = faces + (long long)c.member * 2 * fs;          // this member's r faces
        const int lastoff = (np - 1) * PB;
        const bool has_lo = c.member > 0, has_hi = c.member < a.T - 1;
        // r on the member's face planes to the team (they are p's faces too
        // at the start)
        auto put_faces = [&](int s, const T(&v)[VZ], int es) {
            if (es < PB && has_lo) vstore<T, VZ>(fme + es, v);
            if (es >= lastoff && has_hi) vstore<T, VZ>(fme + fs + es - lastoff, v);
        };
        {
            const int eb = E0();
#pragma unroll
            for (int s = 0; s < Q; s++) {
#pragma unroll
                for (int v = 0; v < VZ; v++) r[s][v] = T(0);
                const int es = E(s);
                if (es >= nE) continue;
                const int l = es / PB, rem = es - l * PB;
                const int i = lo + l, j = rem / B.bz, k = rem - j * B.bz;
                const long long I = B.i0 + i, J = B.j0 + j, K = B.k0 + k;
                const long long cg = (I * ny + J) * nz + K;
                double xc[VZ], xm[VZ], xp[VZ], ym[VZ], yp[VZ], bb[VZ];
#pragma unroll
                for (int v = 0; v < VZ; v++) { xm[v] = 0.0; xp[v] = 0.0; ym[v] = 0.0; yp[v] = 0.0; }
                vload<double, VZ>(a.xa + cg, xc);
                vload<double, VZ>(a.b + cg, bb);
                if (I > 0) vload<double, VZ>(a.xa + cg - ny * nz, xm);
                if (I < nx - 1) vload<double, VZ>(a.xa + cg + ny * nz, xp);
                if (J > 0) vload<double, VZ>(a.xa + cg - nz, ym);
                if (J < ny - 1) vload<double, VZ>(a.xa + cg + nz, yp);
                const double zm = K > 0 ? a.xa[cg - 1] : 0.0;
                const double zp = K + VZ < nz ? a.xa[cg + VZ] : 0.0;
                // Dirichlet lifting: boundary neighbours' g moved to the right
                if (I == 0 && a.F.f[0]) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) bb[v] += a.F.f[0][J * nz + K + v];
                }
                if (I == nx - 1 && a.F.f[1]) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) bb[v] += a.F.f[1][J * nz + K + v];
                }
                if (J == 0 && a.F.f[2]) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) bb[v] += a.F.f[2][I * nz + K + v];
                }
                if (J == ny - 1 && a.F.f[3]) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) bb[v] += a.F.f[3][I * nz + K + v];
                }
                if (K == 0 && a.F.f[4]) bb[0] += a.F.f[4][I * ny + J];
                if (K + VZ == nz && a.F.f[5]) bb[VZ - 1] += a.F.f[5][I * ny + J];
                T zero[VZ];
#pragma unroll
                for (int v = 0; v < VZ; v++) {
                    const double left = v == 0 ? zm : xc[v - 1];
                    const double right = v == VZ - 1 ? zp : xc[v + 1];
                    const double ax = 6.0 * xc[v] - xm[v] - xp[v] - ym[v] - yp[v] - left - right;
                    double rv = bb[v] - ax;
                    if (OVL) {
                        if ((FL[s] >> (9 + v)) & 1) rv = 0.0;
                        // own cells: the vector is wholly own or wholly not
                        if ((FL[s] >> 8) & 1) acc64 += rv * rv;
                    } else {
                        acc64 += rv * rv;
                    }
                    r[s][v] = (T)rv;
                    accT += r[s][v] * r[s][v];
                    zero[v] = T(0);
                }
                vstore<T, VZ>(lp + es, r[s]);    // p = r
                if (!DREG) vstore<T, VZ>(ldd + es, zero);   // d = 0
                put_faces(s, r[s], es);
            }
        }
        // residual sums over the team (the barrier also publishes the faces)
        if (!team_reduce2(c, acc64, accT)) return;
        T rho = accT;
        const T rho0 = rho;
        if (c.member == 0 && tid == 0) {
            if (ASYNC) __hip_atomic_store(&as.board[blk], acc64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else a.p64[blk] = acc64;
        }
        // the neighbours' face planes of p, into the private halo planes:
        // from their r faces scaled by beta plus the old halo (beta = 0 here)
        const T *nlo = faces + (long long)(c.member - 1) * 2 * fs + fs;   // member-1's last plane
        const T *nhi = faces + (long long)(c.member + 1) * 2 * fs;        // member+1's first plane
        // Each element of the member's first (last) plane belongs to one
        // vector slot of one thread; that thread also keeps the matching
        // element of the lower (upper) halo plane (zero at the box's edge).
        auto nbr_face = [&](const T *f, T(&v)[VZ]) {
#pragma unroll
            for (int u = 0; u < VZ; u++) v[u] = ld_sh(f + u);
        };
        {
            const int eb = E0();
#pragma unroll
            for (int s = 0; s < Q; s++) {
                const int es = E(s);
                if (es >= nE) continue;
                T v[VZ];
#pragma unroll
                for (int u = 0; u < VZ; u++) v[u] = T(0);
                if (es < PB) {
                    if (has_lo) nbr_face(nlo + es, v);
                    vstore<T, VZ>(hlo + es, v);
                }
                if (es >= lastoff) {
#pragma unroll
                    for (int u = 0; u < VZ; u++) v[u] = T(0);
                    if (has_hi) nbr_face(nhi + es - lastoff, v);
                    vstore<T, VZ>(hhi + es - lastoff, v);
                }
            }
        }
        __syncthreads();
        int iters = 0;
        // q = A_ii p on vector slot s, with p at the slot returned in pc
        // (zero outside the box; outside an overlap region q is zero too, so
        // r, p and d stay zero there)
        auto apply = [&](int s, int e, T(&pc)[VZ], T(&qv)[VZ]) {
            int f = FL[s];
            asm volatile("" : "+v"(f));   // keep the per-slot offsets from being hoisted
            T xm[VZ], xp[VZ], ym[VZ], yp[VZ];
            // every load is made (an edge reads the cell itself, then
            // drops it), so the slot's loads issue together without branches
            vload<T, VZ>(lp + e, pc);
            vload<T, VZ>(lp + e - PB, xm);   // a halo plane at the slab's faces
            vload<T, VZ>(lp + e + PB, xp);
            vload<T, VZ>(lp + e - ((f & 4) ? B.bz : 0), ym);
            vload<T, VZ>(lp + e + ((f & 8) ? B.bz : 0), yp);
            T zm = lp[e - ((f & 16) ? 1 : 0)];
            T zp = lp[e + ((f & 32) ? VZ : 0)];
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                if (!(f & 4)) ym[v] = T(0);
                if (!(f & 8)) yp[v] = T(0);
            }
            if (!(f & 16)) zm = T(0);
            if (!(f & 32)) zp = T(0);
#pragma unroll
            for (int v = 0; v < VZ; v++) {
                const T left = v == 0 ? zm : pc[v - 1];
                const T right = v == VZ - 1 ? zp : pc[v + 1];
                T qq = T(6) * pc[v] - xm[v] - xp[v] - ym[v] - yp[v] - left - right;
                if (OVL && ((f >> (9 + v)) & 1)) qq = T(0);
                qv[v] = qq;
            }
        };
        bool ok = true;
        // A p of the sigma pass, kept in registers for the update pass on the
        // first QK slots (32 registers, 16 when there are more than 8 slots);
        // later slots apply the stencil again
        constexpr int QK = Q * VZ * (int)sizeof(T) <= 128 ? Q : 64 / (VZ * (int)sizeof(T));
        T qr[QK][VZ];
        // the iterations, with the slot loops free of per-slot branches when
        // every slot of every thread holds a vector (FULL)
        auto cg_loop = [&](auto fullc) {
            constexpr bool FULL = decltype(fullc)::value;
            for (int it = 0; it < a.m; it++) {
                // sigma = p . A p
                T sig = T(0), unused = T(0);
                {
                    const int eb = E0();
#pragma unroll
                    for (int s = 0; s < Q; s++) {
                        if (!FULL && E(s) >= nE) continue;
                        T pc[VZ], qv[VZ];
                        apply(s, E(s), pc, qv);
#pragma unroll
                        for (int v = 0; v < VZ; v++) {
                            sig += pc[v] * qv[v];
                            if (s < QK) qr[s < QK ? s : 0][v] = qv[v];
                        }
                        // slots go in pairs: the loads of two slots in flight
                        // together, without holding all slots' in registers
                        if (s % kSlotGroup == kSlotGroup - 1) __builtin_amdgcn_sched_barrier(0);
                    }
                }
                if (!team_reduce2(c, sig, unused)) { ok = false; break; }
                if (!(sig > T(0))) break;   // breakdown guard: stop this block's inner solve
                const T alpha = rho / sig;
                // d += alpha p; r -= alpha A p; rho' = r . r; r faces out
                T rn = T(0);
                {
                    const int eb = E0();
#pragma unroll
                    for (int s = 0; s < Q; s++) {
                        const int es = E(s);
                        if (!FULL && es >= nE) continue;
                        T pc[VZ], qv[VZ], dd[VZ];
                        if (s < QK) {
                            vload<T, VZ>(lp + es, pc);
#pragma unroll
                            for (int v = 0; v < VZ; v++) qv[v] = qr[s < QK ? s : 0][v];
                        } else {
                            apply(s, es, pc, qv);
                        }
                        if (DREG) {
#pragma unroll
                            for (int v = 0; v < VZ; v++) dd[v] = dr[DREG ? s : 0][v];
                        } else {
                            vload<T, VZ>(ldd + es, dd);
                        }
#pragma unroll
                        for (int v = 0; v < VZ; v++) {
                            dd[v] = dd[v] + alpha * pc[v];
                            r[s][v] = r[s][v] - alpha * qv[v];
                            rn += r[s][v] * r[s][v];
                        }
                        if (DREG) {
#pragma unroll
                            for (int v = 0; v < VZ; v++) dr[DREG ? s : 0][v] = dd[v];
                        } else {
                            vstore<T, VZ>(ldd + es, dd);
                        }
                        if (it < a.m - 1) put_faces(s, r[s], es);
                        if (s % kSlotGroup == kSlotGroup - 1) __builtin_amdgcn_sched_barrier(0);
                    }
                }
                iters = it + 1;
                if (it == a.m - 1) break;
                if (!team_reduce2(c, rn, unused)) { ok = false; break; }
                if (a.inner_tol > 0.0 && sqrt((double)rn) <= a.inner_tol * sqrt((double)rho0)) break;
                const T beta = rn / rho;
                rho = rn;
                // p = r + beta p (every thread is past its reads of p: the
                // team sum synchronised the workgroup)
                {
                    const int eb = E0();
#pragma unroll
                    for (int s = 0; s < Q; s++) {
                        const int es = E(s);
                        if (!FULL && es >= nE) continue;
                        T pv[VZ];
                        vload<T, VZ>(lp + es, pv);
#pragma unroll
                        for (int v = 0; v < VZ; v++) pv[v] = __builtin_fma(beta, pv[v], r[s][v]);
                        vstore<T, VZ>(lp + es, pv);
                        // the neighbours' face planes of p, the same way
                        T nr[VZ], hv[VZ];
                        if (es < PB && has_lo) {
                            nbr_face(nlo + es, nr);
                            vload<T, VZ>(hlo + es, hv);
#pragma unroll
                            for (int v = 0; v < VZ; v++) hv[v] = __builtin_fma(beta, hv[v], nr[v]);
                            vstore<T, VZ>(hlo + es, hv);
                        }
                        if (es >= lastoff && has_hi) {
                            nbr_face(nhi + es - lastoff, nr);
                            vload<T, VZ>(hhi + es - lastoff, hv);
#pragma unroll
                            for (int v = 0; v < VZ; v++) hv[v] = __builtin_fma(beta, hv[v], nr[v]);
                            vstore<T, VZ>(hhi + es - lastoff, hv);
                        }
                    }
                }
                __syncthreads();
            }
        };
        if (rho > T(0)) {
            cg_loop(std::false_type{});
        }
        if (!ok) return;
        // ---- outer update x_new = x_old + d on the block's own cells ----
        {
            const int eb = E0();
#pragma unroll
            for (int s = 0; s < Q; s++) {
                const int es = E(s);
                if (es >= nE || !((FL[s] >> 8) & 1)) continue;
                const int l = es / PB, rem = es - l * PB;
                const int j = rem / B.bz, k = rem - j * B.bz;
                const long long cg = ((long long)(B.i0 + lo + l) * ny + B.j0 + j) * nz + B.k0 + k;
                double xo[VZ];
                T dd[VZ];
                vload<double, VZ>(a.xa + cg, xo);
                if (DREG) {
#pragma unroll
                    for (int v = 0; v < VZ; v++) dd[v] = dr[DREG ? s : 0][v];
                } else {
                    vload<T, VZ>(ldd + es, dd);
                }
#pragma unroll
                for (int v = 0; v < VZ; v++) xo[v] += (double)dd[v];
                vstore<double, VZ>(a.xb + cg, xo);
            }
        }
        if (c.member == 0 && tid == 0 && iters > 0 && !ASYNC)
            atomicAdd(&ctrl->inner_iters, (unsigned long long)iters);
        if (ASYNC) {
            // every member's x is written before the block is published
            if (!team_sync(c)) return;
            if (c.member == 0) async_publish(as, blk, max_sweeps, iters, tol2, ctrl, ash, g.nblocks);
        }
    }
}

#undef E

template <typename T, int VZ, int Q, bool OVL, bool ASYNC>
static hipError_t team_launch(const Geom &g, const TeamArgs &a, AsyncState as, int S,
                              int max_sweeps, double tol2, Ctrl *ctrl, int grid, size_t lds,
                              hipStream_t st) {
    auto kern = k_team<T, VZ, Q, OVL, ASYNC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    Geom gg = g;
    TeamArgs aa = a;
    void *args[] = {&gg, &aa, &as, &S, &max_sweeps, &tol2, &ctrl};
    if (g_launch_events.pending) {
        g_launch_events.pending = false;
        (void)hipEventRecord(g_launch_events.start, st);
        e = hipLaunchCooperativeKernel((const void *)kern, dim3(grid), dim3(kTeamThreads), args,
                                       (unsigned)lds, st);
        (void)hipEventRecord(g_launch_events.stop, st);
        return e;
    }
    return hipLaunchCooperativeKernel((const void *)kern, dim3(grid), dim3(kTeamThreads), args,
                                      (unsigned)lds, st);
}

#define MS_TEAM_Q(T_, VZ_, OVL_, ASYNC_)                                                     \
    switch (q) {                                                                             \
        case 2: return team_launch<T_, VZ_, 2, OVL_, ASYNC_>(g, a, as, S, ms, tol2, c, grid, lds, st); \
        case 4: return team_launch<T_, VZ_, 4, OVL_, ASYNC_>(g, a, as, S, ms, tol2, c, grid, lds, st); \
        case 8: return team_launch<T_, VZ_, 8, OVL_, ASYNC_>(g, a, as, S, ms, tol2, c, grid, lds, st); \
        case 12: return team_launch<T_, VZ_, 12, OVL_, ASYNC_>(g, a, as, S, ms, tol2, c, grid, lds, st); \
        default: return hipErrorInvalidValue;                                                \
    }

template <typename T>
hipError_t launch_team(const Geom &g, int vz, int q, const TeamArgs &a, bool async,
                       AsyncState as, int S, int ms, double tol2, Ctrl *c, int grid,
                       size_t lds, hipStream_t st) {
    const bool ovl = g.ovl != 0;
#define MS_TEAM_VZ(VZ_)                                                                      \
    if (ovl) {                                                                               \
        if (async) { MS_TEAM_Q(T, VZ_, true, true) } else { MS_TEAM_Q(T, VZ_, true, false) } \
    } else {                                                                                 \
        if (async) { MS_TEAM_Q(T, VZ_, false, true) } else { MS_TEAM_Q(T, VZ_, false, false) } \
    }
    // FP64 runs on vectors of at most 2 cells (4 would not leave registers
    // for the slots)
    switch (vz) {
        case 1: MS_TEAM_VZ(1)
        case 2: MS_TEAM_VZ(2)
        case 4:
            if constexpr (sizeof(T) == 4) {
                MS_TEAM_VZ(4)
            }
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
#undef MS_TEAM_VZ
}

int team_threads() { return kTeamThreads; }
int team_face_offset() { return kFaceOff; }

template hipError_t launch_team<double>(const Geom &, int, int, const TeamArgs &, bool,
                                        AsyncState, int, int, double, Ctrl *, int, size_t,
                                        hipStream_t);
template hipError_t launch_team<float>(const Geom &, int, int, const TeamArgs &, bool,
                                       AsyncState, int, int, double, Ctrl *, int, size_t,
                                       hipStream_t);

}  // namespace ms
