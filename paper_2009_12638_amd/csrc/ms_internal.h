// Internal declarations shared by the kernels and the host side of libms.
// Not part of the public ABI (include/ms.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace ms {

constexpr int kThreads = 256;       // threads per workgroup in the tiled kernels
constexpr int kAsyncThreads = 1024;   // threads per persistent asynchronous CG worker
constexpr int kAsyncGmThreads = 512;  // threads per asynchronous GMRES worker (its w tiles
                                      // need more than the 128 registers 1024 threads allow)

// One block of the partition (Section 3: the unknowns X_i of one block).
// The box [i0, i0+bx) x [j0, j0+by) x [k0, k0+bz) is the block's inner-solve
// domain: the block itself, or with overlap the box holding its region (the
// block plus slabs of depth dep across faces that have a neighbour).  The
// box is grown by dep in x and y and by dep rounded up to the widest vector
// width in z, so z vectors stay aligned.  The block's own cells are the
// sub-box at offset (oi, oj, ok) of extents (obx, oby, obz); without overlap
// that is the whole box.
struct BlockInfo {
    int i0, j0, k0;   // origin in the global interior grid
    int bx, by, bz;   // extents
    long long off;    // offset of this block inside the packed inner vectors
    int tile0;        // first tile (workgroup) number of this block
    int ntiles;       // tiles of this block = nplane * nxchunk
    int nplane;       // tiles across one y-z plane
    int oi, oj, ok;   // own cells: offset inside the box
    int obx, oby, obz;  // own cells: extents
    int dep;          // overlap depth (0: none)
};

// Device-side control block: convergence state of one solve.
struct Ctrl {
    int done;          // 1 once the solve has finished (all kernels then exit)
    int status;        // ms_status of the finished solve
    int sweep;         // index of the next residual check
    int final_sweep;   // iterate returned = x^(final_sweep)
    double nbeff;      // ||b_eff||_2
    double res0;       // first relative residual (divergence test)
    double last_res;   // latest relative residual
    unsigned long long inner_iters;  // CG iterations summed over blocks
    unsigned long long inner_snap;   // inner_iters as of the previous check
    // async bookkeeping
    int stop;          // async: set once the residual estimate is below tol
    int max_stale;     // async: largest version gap observed
    unsigned long long work_items;   // async: block sweeps completed
    double pad_[3];
};

// Geometry passed by value to every kernel.
struct Geom {
    long long nx, ny, nz;
    const BlockInfo *blocks;
    const int *tile_block;   // tile -> block
    int tx;                  // x planes per tile
    int rows;                // rows (y) per thread: 1, 2 or 4
    int nblocks;
    int ovl;                 // 1: blocks are overlap regions (mask edges, write own cells)
};

struct Faces {
    const double *f[6];      // -x,+x,-y,+y,-z,+z (nullable)
};

// Several right-hand sides solved by the same launches: workgroup w of a
// launch over nt tiles serves right-hand side w / nt; per-RHS arrays are
// offset by these strides.
struct Batch {
    int nt;          // tiles per right-hand side in this launch (set by the launcher)
    int nrhs;        // right-hand sides
    long long vs;    // element stride between right-hand sides' vectors (b, x)
    long long ps;    // stride of per-tile partial arrays
    long long bs;    // stride of per-block arrays
    long long is;    // element stride between right-hand sides' inner vectors
    int k0, nk;      // CG phase launches: right-hand sides [k0, k0 + nk)
};

inline Batch single_rhs() { return Batch{0, 1, 0, 0, 0, 0, 0, 1}; }

// GMRES inner solves: per (right-hand side, block) records of the
// Hessenberg/Givens state (doubles), per (right-hand side, tile) partial
// sums, and the Krylov vectors (vector i of right-hand side k starts at
// V + i * kvs + k * Batch::is).
struct GmArgs {
    double *gm;          // records, rec_stride doubles each
    double *gpart;       // tile partials, gstride slots each
    long long kvs;       // elements between consecutive Krylov vectors
    int M;               // inner iterations the records are laid out for
    int gstride;         // M + 2: dots with u_0..u_M, then the norm slot
    int nblocks;
    int rec_stride;
};

// Shared state of an asynchronous solve (one entry per block).
struct AsyncState {
    int *version;        // sweeps the block has completed
    int *claim;          // 1 while a worker holds the block
    double *board;       // latest published ||r_i||^2 of the block
    const int *nbr;      // 6 neighbour blocks per block (-1 = none)
    int *finished;       // blocks that reached the sweep limit this launch
    // debugging aids (off when trace is null / slow_sleep is 0)
    int *trace;          // kTraceInts ints per started block sweep: block,
                         // its version, the 6 neighbours' versions (-1 = none)
    int *trace_n;        // block sweeps started (records beyond trace_cap are not written)
    int trace_cap;
    int slow_block;      // block whose worker waits before each of its sweeps
    int slow_sleep;      // ... this many s_sleep(127) instructions
};
constexpr int kTraceInts = 8;

// Resident-team block solves (ms_team.hip): T workgroups of one XCD per
// team, one block per team at a time, the block's inner vectors held in
// registers and LDS.
struct TeamArgs {
    int T;                 // workgroups per team
    int per_xcd;           // workgroups of the launch per XCD expected (grid / 8)
    int nwork;             // sync: blocks swept by the launch (all of them)
    int *next;             // sync: next block to hand out (zeroed before each launch)
    int *err;              // 0, or 1: an XCD id outside 0..7, 2: a team barrier
                           // timed out, 3: the launch's workgroups did not all start
    int *xcd_count;        // [8] workgroups that arrived on each XCD (zeroed per launch)
    int *arrived;          // workgroups that arrived (zeroed per launch)
    char *team_mem;        // team_bytes per team: barrier counter, work
                           // ring, partial sums, slab faces
    long long team_bytes;
    long long face_stride; // elements per slab face (>= the largest box's y*z)
    int m;                 // inner iterations
    double inner_tol;
    const double *b;
    const double *xa;      // x read by the residual
    double *xb;            // x written by the update (== xa in async mode)
    Faces F;
    double *p64;           // sync: own-cell residual^2 per block
    int max_spin;          // polls before a team barrier gives up
};

// ---- kernel launches ------------------------------------------------------
// Profiling: the host sets events that the next launch of this thread
// records its start and end into.  They are attached to the dispatch itself
// (hipExtLaunchKernelGGL), so they time the kernel alone, without the gap
// before it starts.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool pending = false;
};
extern thread_local LaunchEvents g_launch_events;

template <typename F, typename... Args>
inline void launch(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st, Args... args) {
    if (g_launch_events.pending) {
        g_launch_events.pending = false;
        hipExtLaunchKernelGGL(kernel, grid, block, shm, st, g_launch_events.start,
                              g_launch_events.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    }
}

// ---- launchers (ms_kernels.hip) ----------------------------------------
// All launchers enqueue on `st` and return the launch error.

// Outer residual r = b_eff - A x (x == nullptr means x = 0) over tiles
// [t0, t1); stores r packed (relative to group offset goff) when r != null;
// writes per-tile partial sums of r^2 in FP64 (p64) and in the inner type
// (pT, may equal p64 for FP64).
template <typename T>
hipError_t launch_resid(const Geom &g, int vz, int t0, int t1, long long goff,
                        const double *b, const double *x, Faces faces, T *r,
                        double *p64, T *pT, const Ctrl *ctrl, Batch bt, hipStream_t st);

// Inner CG phase 1: p_new = r + beta p_old (beta = 0 at iter 0), per-tile
// partials of sigma = p_new . A_ii p_new.
template <typename T>
hipError_t launch_stencil(const Geom &g, int vz, int t0, int t1, long long goff,
                          const T *r, const T *p_old, T *p_new, T *psig,
                          const T *prho_cur, const T *prho_prev, const T *prho0,
                          int *active, int iter, double inner_tol,
                          Ctrl *ctrl, Batch bt, hipStream_t st);

// Inner CG phase 2: alpha = rho/sigma; d += alpha p; r -= alpha A_ii p;
// partials of r.r.  When last != 0: xb = xa + d + alpha p instead (r and d
// not written).
template <typename T>
hipError_t launch_update(const Geom &g, int vz, int t0, int t1, long long goff,
                         T *r, const T *p, T *d, const T *psig,
                         const T *prho_cur, T *prho_next, int *active, int iter,
                         int last, const double *xa, double *xb, Ctrl *ctrl,
                         Batch bt, hipStream_t st);

// Persistent asynchronous sweep kernel (grid = workers).
template <typename T>
hipError_t launch_async(const Geom &g, int vz, int grid, const double *b, double *x, Faces faces,
                        T *r, T *p0, T *p1, T *d, AsyncState as, int m, int S, int max_sweeps,
                        double tol2, double inner_tol, Ctrl *ctrl, hipStream_t st);
template <typename T>
hipError_t async_occupancy(int vz, int rows, int ovl, int *per_cu);

// Global CG on the single-block geometry g (device scalars scal[3]).
hipError_t launch_gcg_stencil(const Geom &g, int vz, int ntiles, const double *r,
                              const double *pold, double *pnew, double *psig, const double *scal,
                              int iter, const Ctrl *ctrl, hipStream_t st);
hipError_t launch_gcg_update(const Geom &g, int vz, int ntiles, double *r, const double *p,
                             double *x, double *prho, const double *scal, const Ctrl *ctrl,
                             hipStream_t st);
hipError_t launch_gcg_reduce(const double *part, int ntiles, int which, double tol, int max_iters,
                             double *history, int history_cap, double *scal, Ctrl *ctrl,
                             hipStream_t st);

// Residual check after a sweep's residual kernels: fixed-order sum of the
// FP64 partials of tiles [0, ntiles), convergence/divergence decision.
hipError_t launch_check(const double *p64, int ntiles, double tol, int final_check,
                        double *history, int history_cap, Ctrl *ctrl, Batch bt,
                        hipStream_t st);

// ||b_eff||: fixed-order sum of partials into ctrl->nbeff.
hipError_t launch_norm(const double *p64, int ntiles, Ctrl *ctrl, hipStream_t st);

// y = A u on the global grid (zero outside the interior).
hipError_t launch_apply(long long nx, long long ny, long long nz, const double *u,
                        double *y, hipStream_t st);

// out = s f + boundary values of the faces F (the lifted right-hand side).
hipError_t launch_lift(long long nx, long long ny, long long nz, const double *f, double s,
                       Faces F, double *out, hipStream_t st);
// Transpose of launch_lift: gf = s lam (when gf != null) and, for every
// non-null gfaces[t], lam at the interior cells next to face t.
hipError_t launch_lift_adjoint(long long nx, long long ny, long long nz, const double *lam,
                               double s, double *gf, double *const gfaces[6], hipStream_t st);

// Fixed-order sum of n doubles into *out (device).
hipError_t launch_sum(const double *v, int n, double *out, hipStream_t st);

// ---- GMRES inner solves (ms_gmres.hip) ----------------------------------
// Tiles must be one row per thread and at most gm_max_planes() x planes.
// init: beta = ||r|| per block of [b0, b1) from the residual's region
// partials pT.  step part 0..2 of Arnoldi step j: apply + dots,
// coefficients + orthogonalisation + norm partials, per-block norm and
// Givens rotation.  finish part 0: per-block triangular solve; part 1:
// x_new = x_old + correction on own cells.
template <typename T>
hipError_t launch_gm_init(const Geom &g, int b0, int b1, const T *pT, Batch bt, GmArgs a,
                          Ctrl *ctrl, hipStream_t st);
template <typename T>
hipError_t launch_gm_step(const Geom &g, int vz, int t0, int t1, int b0, int b1, long long goff,
                          T *V, int j, double inner_tol, Batch bt, GmArgs a, Ctrl *ctrl,
                          hipStream_t st, int part);
template <typename T>
hipError_t launch_gm_finish(const Geom &g, int vz, int t0, int t1, int b0, int b1,
                            long long goff, const T *V, const double *xa, double *xb, Batch bt,
                            GmArgs a, Ctrl *ctrl, hipStream_t st, int part);
int gm_record_doubles(int M);
int gm_max_planes();

// Resident-team sweep (sync: every block from a.xa into a.xb; async: claimed
// blocks in place) on grid = 8 * a.per_xcd workgroups of team_threads()
// threads, launched cooperatively; vz: z cells per vector, q: vectors per
// thread (1, 2, 4 or 8), lds: bytes of dynamic LDS (the largest slab).
template <typename T>
hipError_t launch_team(const Geom &g, int vz, int q, const TeamArgs &a, bool async,
                       AsyncState as, int S, int max_sweeps, double tol2, Ctrl *ctrl, int grid,
                       size_t lds, hipStream_t st);
int team_threads();
int team_face_offset();

// Asynchronous sweeps with GMRES inner solves (persistent workers, as
// launch_async; Krylov vectors and records of right-hand side 0).
template <typename T>
hipError_t launch_async_gmres(const Geom &g, int vz, int grid, const double *b, double *x,
                              Faces faces, T *V, AsyncState as, int m, int S, int max_sweeps,
                              double tol2, double inner_tol, GmArgs a, Ctrl *ctrl,
                              hipStream_t st);
template <typename T>
hipError_t async_gmres_occupancy(int vz, int ovl, int *per_cu);

}  // namespace ms
