/*
 * ms.h - C ABI of libms, a two-stage multisplitting solver (synchronous or
 * asynchronous block Jacobi outer sweep, conjugate-gradient inner solves on
 * each block) for the 3D 7-point Laplace/Poisson system A x = b on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Brown, Bull and Bethune, "A highly scalable approach to solving
 * linear systems using two-stage multisplitting".  Section 2.1 defines the
 * operator (7-point Laplace stencil, Dirichlet boundaries) and the stopping
 * rule on ||Ax - b||_2; Section 3 gives the block Jacobi update
 *     X_i^(k) = A_ii^{-1} (B_i - sum_{j != i} A_ij X_j^(k-1)),
 * its loop (Listing 1: inner Krylov solve per block, halo exchange, global
 * residual) and the global residual as the root-sum-square of the block
 * residuals; Section 3.2 fixes a maximum number of inner iterations;
 * Sections 2.1 and 2.3 describe the asynchronous variant in which a block
 * uses the latest neighbour values it has.
 *
 * Conventions shared by every entry point
 *   - Unknowns live on the interior points of an nx*ny*nz grid, C order,
 *     element (i,j,k) at offset (i*ny + j)*nz + k (z fastest).
 *   - (A u)(i,j,k) = 6 u(i,j,k) - sum of the six axis neighbours; a
 *     neighbour outside the interior is a Dirichlet node whose value comes
 *     from the boundary faces held by the handle and is moved to the
 *     right-hand side: b_eff = b + sum over boundary neighbours of g.
 *   - All vector arguments are FP64 DEVICE pointers (for instance the
 *     data_ptr() of a contiguous torch tensor on the GPU), 16-byte aligned,
 *     length nx*ny*nz, owned by the caller.  Nothing is retained after a
 *     call returns.  A pointer that is not device memory, or whose
 *     allocation ends before nx*ny*nz doubles, is rejected (MS_ERR_ARG);
 *     a piece of a larger allocation (a caching allocator's block) cannot
 *     be told apart from a whole buffer, so its size is the caller's duty.
 *   - Relative residual = ||b_eff - A x||_2 / ||b_eff||_2 in FP64.
 *   - Every call returns an ms_status; nothing aborts or prints.  After a
 *     failure ms_last_error(handle) describes it.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef MS_H
#define MS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MS_OK = 0,
    MS_ERR_ARG = 1,           /* invalid argument; nothing was run          */
    MS_ERR_HIP = 2,           /* a HIP runtime call failed                  */
    MS_ERR_NOMEM = 3,         /* device allocation failed                   */
    MS_ERR_NOT_CONVERGED = 4, /* max_sweeps reached above tol; x = last iterate */
    MS_ERR_NONFINITE = 5,     /* residual became NaN/Inf; x unspecified     */
    MS_ERR_DIVERGED = 6,      /* residual grew 1e6x over its start; x unspecified */
    MS_ERR_UNSUPPORTED = 7    /* valid but not supported by the library     */
} ms_status;

typedef enum { MS_SYNC = 0, MS_ASYNC = 1 } ms_mode;
/* Inner solver of every block (Section 3.1: the framework takes CG or
 * GMRES; the paper's experiments used GMRES). */
typedef enum { MS_INNER_CG = 0, MS_INNER_GMRES = 1 } ms_inner;
typedef enum { MS_FP64 = 0, MS_MIXED = 1 } ms_precision;

/* Interior grid size (points per axis, each >= 1). */
typedef struct {
    int64_t nx, ny, nz;
} ms_grid;

/* Block partition (Section 3: the unknowns split into blocks X_i): a tensor
 * product of per-axis cuts.  gx,gy,gz = blocks per axis.  cuts_x is a HOST
 * array of gx+1 increasing offsets 0 = c[0] < ... < c[gx] = nx (likewise y,
 * z); NULL means a uniform split, which requires nx % gx == 0.  Block
 * edges may be any size >= 1 (kernels use wider z accesses when nz and every
 * z cut are multiples of 8, 4 or 2); block (bi,bj,bk) has number
 * (bi*gy + bj)*gz + bk. */
typedef struct {
    int32_t gx, gy, gz;
    const int32_t *cuts_x, *cuts_y, *cuts_z;
} ms_blocks;

/* Dirichlet data g on the six faces, DEVICE pointers in the order
 * -x,+x,-y,+y,-z,+z.  The x faces are [ny][nz], the y faces [nx][nz], the z
 * faces [nx][ny] (C order).  NULL means a zero face.  Copied at ms_create /
 * ms_set_bc; the caller may free them afterwards. */
typedef struct {
    const double *face[6];
} ms_bc;

/* Solver options.  Fill with ms_default_opts() and change what is needed. */
typedef struct {
    int32_t max_sweeps;   /* outer sweeps before MS_ERR_NOT_CONVERGED (default 100000) */
    double inner_tol;     /* > 0: also stop a block's CG once ||r_i|| <= inner_tol*||r_i^0|| */
    int32_t staleness;    /* async (>= 1, default 2): a block starts sweep v+1
                             only when every face neighbour has finished at
                             least v+1-staleness sweeps, so the neighbour data
                             it starts from is at most staleness-1 sweeps
                             older than its own (sync ignores it) */
    int32_t precision;    /* ms_precision (default MS_FP64) */
    void *stream;         /* hipStream_t used for all work; NULL = null stream */
    int32_t check_every;  /* sync: sweeps enqueued between host reads of the
                             convergence flag; async: sweeps per block per
                             launch, after which the host verifies the true
                             residual and relaunches if needed (0 =
                             automatic: about 2^33 cell-iterations per launch
                             for the phase engine, 2^38 for teams, 8 to 1000
                             sweeps) */
    int32_t group_blocks; /* sync: blocks per launch.  0 = automatic: groups
                             whose inner vectors fill the 256 MB on-package
                             cache (with several right-hand sides and CG, each
                             launch covers as many right-hand sides of its
                             blocks as fit); -1 = all blocks at once; > 0 =
                             that many (every right-hand side in each launch) */
    int32_t x_chunk;      /* x planes marched per workgroup (0 = automatic) */
    int32_t profile;      /* 1: time every launch with HIP events attached to
                             its dispatch (kernel time alone), summed per
                             kernel class into ms_stats; sweeps are then
                             launched one by one instead of from a graph */
    int32_t use_graph;    /* sync: 1 = replay sweeps from a captured HIP graph
                             (default 1) */
    int32_t rows;         /* y rows each thread owns: 1, 2 or 4 (0 = automatic);
                             asynchronous CG workers take at most 2 (1 with
                             4-cell z vectors) */
    int32_t workers;      /* async: persistent workgroups, each sweeping one block
                             at a time (0 = automatic) */
    int32_t inner_solver; /* ms_inner (default MS_INNER_CG).  MS_INNER_GMRES
                             needs ms_reserve_krylov */
    int32_t z_vector;     /* sync: z cells each thread accesses at once, 1, 2, 4
                             or 8 (0 = automatic: 16 bytes; at most 32 bytes,
                             16 with GMRES, 4 cells with overlap; nz and every
                             z cut must be multiples of it) */
    /* Debugging aids of asynchronous mode (Section 5: tolerance of slow
     * processes; Section 2.3: bounded delays). */
    int32_t slow_block;   /* block whose worker waits before each of its sweeps
                             (< 0: none; default -1) */
    int32_t slow_sleep;   /* that wait: this many s_sleep(127) instructions,
                             about 8000 cycles each (0: off; at most 100000) */
    int32_t *trace;       /* DEVICE buffer (or NULL) of trace_cap records of 8
                             int32, one per block sweep started, in start
                             order: block, the block's version (sweeps it had
                             finished), then the versions of its -x,+x,-y,+y,
                             -z,+z neighbours read when it started (-1: no
                             neighbour).  Sweeps beyond trace_cap are counted
                             in ms_stats.trace_len but not written */
    int32_t trace_cap;
    int32_t engine;       /* how CG inner solves run (ms_engine, default
                             MS_ENGINE_AUTO) */
    int32_t team_spin;    /* debugging: polls a team-engine wait (the launch's
                             start, a team barrier) makes before it gives up
                             and the solve fails with MS_ERR_HIP; 0 (default)
                             = 2^24.  A tiny value forces that failure path;
                             every kernel still exits.  >= 0 */
} ms_opts;

/* Kernels that carry out the CG inner solves.
 *   MS_ENGINE_PHASE: each CG phase is a launch over a group of blocks whose
 *     inner vectors stay in the 256 MB on-package cache (synchronous mode);
 *     one persistent workgroup per block being swept (asynchronous mode).
 *   MS_ENGINE_TEAM: a team of workgroups of one XCD solves one block at a
 *     time with the block's inner vectors held in registers and LDS for all
 *     inner iterations (synchronous and asynchronous mode, single
 *     right-hand side).  Needs every block's box to fit: with 512-thread
 *     workgroups of 160 KB LDS, about 20K cells per workgroup (FP32 inner)
 *     or 10K (FP64), a team being at most 32 workgroups.  Each sweep is one
 *     cooperative launch that occupies every compute unit: work on other
 *     streams of the device delays it, and if its workgroups do not all
 *     start within the wait bound, or a team barrier does not complete, the
 *     solve returns MS_ERR_HIP (x unspecified).  Team sums add per-member
 *     partials in member order, so results are deterministic; they differ
 *     from the phase engine's in rounding only.
 *   MS_ENGINE_AUTO: TEAM when it fits, else PHASE; setting any tiling
 *     option of the phase engine (group_blocks, x_chunk, rows, z_vector,
 *     workers) selects PHASE.
 * GMRES inner solves and several right-hand sides always use PHASE. */
typedef enum { MS_ENGINE_AUTO = 0, MS_ENGINE_PHASE = 1, MS_ENGINE_TEAM = 2 } ms_engine;

/* Kernel classes reported by the profile counters of ms_stats. */
enum {
    MS_K_RESID = 0,   /* outer residual r = b_eff - A x with halo reads   */
    MS_K_STENCIL = 1, /* inner CG: p = r + beta p; sigma = p.A_ii p.
                         GMRES: w = A_ii v_j and its dots with the basis */
    MS_K_UPDATE = 2,  /* inner CG: d += alpha p; r -= alpha A_ii p; r.r   */
    MS_K_FINAL = 3,   /* last inner step fused with x_new = x + d
                         (GMRES: x_new = x + V y)                        */
    MS_K_CHECK = 4,   /* global residual sum and convergence test          */
    MS_K_OTHER = 5,   /* persistent asynchronous workers; resident-team
                         sweeps (MS_ENGINE_TEAM)                           */
    MS_K_ORTH = 6,    /* GMRES: Hessenberg column, Gram-Schmidt
                         orthogonalisation and norm                        */
    MS_K_HESS = 7,    /* GMRES: per-block start, Givens rotations, solve   */
    MS_K_COUNT = 8
};

typedef struct {
    int32_t sweeps;            /* outer updates applied to x                 */
    int64_t inner_iters;       /* CG iterations summed over blocks and sweeps */
    double rel_residual;       /* true FP64 relative residual of returned x  */
    double seconds;            /* wall time of the call                      */
    int32_t max_staleness_seen;/* async: largest version gap to a neighbour
                                  a block sweep started from (<= staleness-1) */
    int32_t relaunches;        /* async: relaunches after a failed verification */
    int32_t history_len;       /* entries written to history                 */
    double *history;           /* HOST buffer supplied by the caller (or NULL):
                                  relative residual at the top of each sweep */
    int32_t history_cap;       /* its capacity                               */
    double kernel_ms[MS_K_COUNT];       /* profile=1: summed event time      */
    int64_t kernel_launches[MS_K_COUNT];/* profile=1: launches timed         */
    int32_t trace_len;         /* async with opts->trace: block sweeps started  */
    int32_t *block_sweeps;     /* HOST buffer supplied by the caller (or NULL)
                                  of block_sweeps_cap entries: sweeps applied
                                  to each block, in block order (sync: all
                                  equal to sweeps) */
    int32_t block_sweeps_cap;
    int32_t engine_used;       /* MS_ENGINE_PHASE or MS_ENGINE_TEAM: the engine
                                  that ran the solve (0 before one ran)     */
} ms_stats;

typedef struct ms_handle ms_handle;

/* Fill *o with the defaults listed above. */
void ms_default_opts(ms_opts *o);

/* Create a solver for one grid, partition and boundary data (Section 3:
 * blocks X_i; Section 2.1: Laplace operator with Dirichlet boundaries).
 * Allocates every device buffer a solve needs, so ms_solve never allocates.
 * Errors: MS_ERR_ARG (bad sizes or cuts), MS_ERR_NOMEM, MS_ERR_HIP.  On
 * error *out is NULL. */
ms_status ms_create(const ms_grid *grid, const ms_blocks *blocks,
                    const ms_bc *bc, ms_handle **out);

/* Replace the boundary data (same layout as ms_create). */
ms_status ms_set_bc(ms_handle *h, const ms_bc *bc);

/* Overlapping blocks (Section 3.2: the block overlap parameter; Section 2.3:
 * the weights D_i of the multisplitting B = sum_i D_i M_i^-1 N_i).  With
 * overlap o >= 1 the inner solve of block i runs on its region: the block's
 * own cells plus, across each face that has a neighbouring block, the slab
 * of depth o beyond that face (clipped to the grid) -- o(2xy+2yz+2zx) extra
 * unknowns for an x*y*z block with neighbours on all sides.  Edge and corner
 * cells next to the block are not in the region.  The inner CG solves the
 * region's principal submatrix of A (zero correction outside the region)
 * from the residual b_eff - A x at the region's cells, and every cell takes
 * the correction of the block that owns it (D_i = indicator of block i's
 * own cells).  The global residual counts each cell once.  o = 0 restores
 * plain block Jacobi.
 * Applies to later ms_solve (sync and async) and ms_solve_batch calls.  In
 * async mode the overlap values, like the halo, are whatever the neighbours
 * last wrote; the staleness bound applies to face neighbours, and cells of
 * the region's halo in edge-adjacent blocks (two face steps away) are at
 * most twice as stale.  Allocates when
 * the regions need larger inner buffers than the handle holds (never
 * shrinks them).  The inner box of a block is grown in z by o rounded up
 * to the vector width (the cells beyond depth o are masked), so z accesses
 * keep their full width for any o.
 * Errors: MS_ERR_ARG (o < 0 or larger than the grid), MS_ERR_NOMEM (the
 * handle keeps its previous overlap), MS_ERR_HIP. */
ms_status ms_set_overlap(ms_handle *h, int32_t overlap);

/* Solve A x = b_eff by two-stage multisplitting (Section 3, Listing 1):
 * each outer sweep computes r = b_eff - A x with neighbour-block values read
 * straight from x (the halo exchange), tests ||r|| / ||b_eff|| <= tol, runs
 * at most inner_iters CG iterations on A_ii d_i = r_i in every block from
 * d_i = 0, then sets x_i += d_i.
 *   b      device, FP64: interior right-hand side before boundary lifting
 *          (for -lap u = f with spacing h this is h*h*f).  Never written.
 *   x      device, FP64, in/out: initial guess in, iterate out.  Must not
 *          alias b.
 *   tol    stop at the first iterate with relative residual <= tol; tol <= 0
 *          runs exactly opts->max_sweeps sweeps and returns MS_OK.
 *   inner_iters  maximum CG iterations per block per sweep (>= 1).
 *   mode   MS_SYNC: every block of sweep k reads sweep k-1 values (Jacobi).
 *          MS_ASYNC: blocks advance independently and read whatever
 *          neighbour values are in memory, a block running at most
 *          opts->staleness sweeps ahead of a neighbour; the stop is decided
 *          from published block residuals and then verified in FP64.
 *   opts   NULL for defaults.  stats: NULL or filled on return.
 * Precision MS_MIXED runs the inner CG in FP32 (storage and accumulation)
 * while residual, convergence test and x stay FP64 (iterative refinement).
 * Blocking: returns once the work on opts->stream is finished.
 * Errors: MS_ERR_ARG, MS_ERR_NOT_CONVERGED (x = last iterate, stats valid),
 * MS_ERR_NONFINITE / MS_ERR_DIVERGED (x unspecified), MS_ERR_HIP.
 * If ||b_eff|| = 0 the result is x = 0 with MS_OK. */
ms_status ms_solve(ms_handle *h, const double *b, double *x, double tol,
                   int32_t inner_iters, ms_mode mode, const ms_opts *opts,
                   ms_stats *stats);

/* Make room for solving nrhs right-hand sides at once with ms_solve_batch
 * (allocates per-right-hand-side device buffers; every other call keeps
 * working).  Errors: MS_ERR_ARG (nrhs outside [1, 4096]), MS_ERR_NOMEM (the
 * handle keeps its previous capacity). */
ms_status ms_reserve(ms_handle *h, int32_t nrhs);

/* GMRES inner solves (Sections 3.1 and 4: the experiments' inner solver;
 * Section 3.2: a maximum number of inner iterations).  With
 * opts->inner_solver = MS_INNER_GMRES each block runs one GMRES(m) cycle
 * per sweep, m = inner_iters, from a zero correction on its residual: an
 * Arnoldi basis built with classical Gram-Schmidt, the correction that
 * minimises the block residual over the Krylov space (Givens rotations of
 * the Hessenberg matrix), early stop when that least-squares residual is
 * <= inner_tol * ||r_i|| or the space becomes invariant.  Works with
 * overlap, with several right-hand sides (synchronous) and in asynchronous
 * mode (each worker runs the whole cycle of the block it took).
 * This call allocates the m+1 basis vectors and per-block state for
 * inner_iters up to max_inner (1..128) for the handle's current right-hand
 * side capacity and overlap; call it again after ms_reserve or
 * ms_set_overlap enlarge those (a GMRES solve otherwise returns
 * MS_ERR_ARG).  Memory: (max_inner+1) * 8 bytes per unknown and
 * right-hand side.  Errors: MS_ERR_ARG, MS_ERR_NOMEM. */
ms_status ms_reserve_krylov(ms_handle *h, int32_t max_inner);

/* Synchronous solve of nrhs independent right-hand sides with the same grid,
 * blocks and boundary data in the same kernel launches (each launch covers
 * every block of every right-hand side; Section 3's sweep applied to each).
 * b and x hold the right-hand sides and iterates one after another
 * ([nrhs][nx][ny][nz], device, FP64).  Each right-hand side stops on its own
 * test (the others keep going).  stats: NULL or an array of nrhs entries.
 * Needs ms_reserve(h, n >= nrhs) first.  Returns MS_OK when every right-hand
 * side converged, else the first failure status.  mode must be MS_SYNC
 * (MS_ERR_UNSUPPORTED otherwise). */
ms_status ms_solve_batch(ms_handle *h, int32_t nrhs, const double *b, double *x, double tol,
                         int32_t inner_iters, ms_mode mode, const ms_opts *opts,
                         ms_stats *stats);

/* True FP64 relative residual ||b_eff - A x||_2 / ||b_eff||_2 (Section 2.1
 * stopping quantity; Section 3 root-sum-square of block residuals).  b, x:
 * device FP64.  *rel_out (host) receives the value (0 if ||b_eff|| = 0);
 * abs_out (host, nullable) receives ||b_eff - A x||_2.  stream: hipStream_t
 * or NULL.  Blocking. */
ms_status ms_residual(ms_handle *h, const double *b, const double *x,
                      double *rel_out, double *abs_out, void *stream);

/* ms_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * it allocates nothing and uses no work buffer of the handle.  Its tile
 * partials and sums live in a static device array of the library (one per
 * GPU, 1 MiB, held until the process ends) that holds the partials of at
 * most 65536 tiles; a handle whose current tiling has more tiles is
 * rejected (MS_ERR_ARG).  Every call on a GPU shares that GPU's array: calls
 * that overlap in time on one GPU (other threads, other streams) race and
 * may return wrong values.  Nothing in the array needs clearing between
 * calls (every slot a call reads, it writes first).  The current device
 * must be the handle's (MS_ERR_ARG otherwise).  Arguments, result and
 * blocking as ms_residual. */
ms_status ms_residual_noalloc(ms_handle *h, const double *b, const double *x,
                              double *rel_out, double *abs_out, void *stream);

/* Right-hand side assembly (Section 2.1: the Dirichlet data of boundary
 * neighbours moved to the right-hand side): b_eff = s * f + sum over each
 * cell's boundary neighbours of the handle's face values.  For -lap u = f
 * with spacing h, s = h*h gives the system the solver works on.  f, b_eff:
 * device FP64, nx*ny*nz; they may be the same buffer (in place) but must not
 * otherwise overlap.  Enqueued on stream (hipStream_t or NULL); not
 * blocking.  Errors: MS_ERR_ARG, MS_ERR_HIP. */
ms_status ms_lift(ms_handle *h, const double *f, double s, double *b_eff, void *stream);

/* Transpose of ms_lift, the last step of an adjoint (backward) solve: with
 * lambda = A^-1 g for an incoming gradient g (A is symmetric), the gradient
 * of a loss with respect to f is s * lambda and with respect to face t it is
 * lambda at the interior cells next to that face (edge and corner nodes do
 * not enter the 7-point stencil).  grad_f: device FP64 nx*ny*nz or NULL (may
 * be lambda itself); grad_face: NULL, or six device pointers (each NULL or a
 * buffer of the face's size, layout as ms_bc).  Enqueued on stream; not
 * blocking.  Errors: MS_ERR_ARG, MS_ERR_HIP. */
ms_status ms_lift_adjoint(ms_handle *h, const double *lambda, double s, double *grad_f,
                          double *const grad_face[6], void *stream);

/* y = A u with zero values outside the interior (the Section 2.1 stencil,
 * boundary data not applied).  u, y device FP64, must not alias.  Enqueued on
 * stream (hipStream_t or NULL); not blocking. */
ms_status ms_apply(ms_handle *h, const double *u, double *y, void *stream);

/* Conventional global solver (Section 4's baseline, here unpreconditioned CG
 * on the whole grid) with the same kernels and data layout.  Stops at the
 * first iteration whose recurrence residual is <= tol * ||b_eff|| (tol <= 0:
 * run exactly max_iters iterations) and reports the true residual in stats.
 * Same argument rules as ms_solve. */
ms_status ms_cg(ms_handle *h, const double *b, double *x, double tol,
                int32_t max_iters, const ms_opts *opts, ms_stats *stats);

/* Free the handle and its device memory (NULL is ignored). */
void ms_destroy(ms_handle *h);

/* Static text for a status code. */
const char *ms_status_string(ms_status s);

/* Text of the last error on this handle (or of the last failed ms_create
 * when h is NULL).  Valid until the next call on the handle. */
const char *ms_last_error(const ms_handle *h);

/* Library version string. */
const char *ms_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MS_H */
