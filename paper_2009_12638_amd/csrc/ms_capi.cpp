// Host side of libms: handle, argument checks, device buffers and the sweep
// scheduler for the synchronous two-stage multisplitting solve.
//
// Sweep schedule (synchronous mode).  Blocks are processed in groups of
// consecutive blocks whose inner vectors (r, d and two p buffers) fill the
// 256 MB on-package cache, so the inner iterations of a group re-read them
// from the cache; every group reuses the same inner buffers.  For one
// group: residual (halo reads from x_old), then m x {stencil, update}; the
// last update writes x_new = x_old + d into the second outer buffer, so all
// groups of a sweep read only x_old (Section 3: X_i^(k) uses only sweep k-1
// values).  After all groups a one-workgroup kernel adds the residual
// partials of x_old in a fixed order and decides convergence on the device.
// Because the test is on x_old, a converged solve returns x_old and the
// sweep just computed is discarded (the two outer buffers make that free).
// The host reads the device flag once per batch of sweeps; kernels enqueued
// after convergence exit at once.
#include "ms.h"
#include "ms_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using ms::BlockInfo;
using ms::Ctrl;
using ms::Faces;
using ms::Geom;
using ms::AsyncState;
using ms::Batch;

namespace {

constexpr int kTxMin = 4;             // smallest x chunk a tiling may use
constexpr int kHistoryCap = 1 << 20;  // device residual history entries
constexpr int kMaxEvents = 4096;      // profile: event pairs per batch

std::string g_create_error;

struct Group {
    int b0, b1;     // blocks [b0, b1)
    int t0, t1;     // tiles [t0, t1)
    long long off;  // packed offset of block b0
    int k0, k1;     // right-hand sides [k0, k1)
};

}  // namespace

struct ms_handle {
    long long nx = 0, ny = 0, nz = 0, N = 0;
    int gx = 0, gy = 0, gz = 0, nblocks = 0;
    std::vector<int> cx, cy, cz;
    int vzmax = 1;              // widest z vector (cells) the z cuts and nz allow, <= 8
    int vzbase = 1;             // min(vzmax, 4): the width overlap boxes are aligned to in z
    int overlap = 0;            // block overlap depth (0: plain block Jacobi)
    long long inner_n = 0;      // inner-vector elements per right-hand side
    long long inner_cap = 0;    // ... that the inner buffers hold (>= inner_n)
    // current tiling
    int cur_vz = 0, cur_tx = 0, cur_rows = 0, ntiles = 0;
    std::vector<BlockInfo> blocks_h;
    int tiles_cap = 0;
    // device memory
    BlockInfo *blocks_d = nullptr;
    int *tile_block_d = nullptr;
    double *x1 = nullptr;
    void *r = nullptr, *d = nullptr, *p0 = nullptr, *p1 = nullptr;
    double *part64 = nullptr;
    void *partT = nullptr, *psig = nullptr, *prhoA = nullptr, *prhoB = nullptr;
    int *active = nullptr;
    Ctrl *ctrl = nullptr;
    double *history_d = nullptr;
    double *faces_d[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double *scal_d = nullptr;
    double *scratch_d = nullptr;    // static scratch of the handle's device (ms_residual_noalloc)
    // resident-team solves: team memory (sized by team_alloc for the
    // current geometry) and counters ([0] next block, [1] error code)
    char *team_mem = nullptr;
    size_t team_mem_bytes = 0;
    int *team_ctr = nullptr;
    // global CG: the whole grid as a single block
    BlockInfo *cg_block_d = nullptr;
    int *cg_tiles_d = nullptr;
    int cg_cap = 0, cg_ntiles = 0, cg_vz = 0, cg_tx = 0, cg_rows = 0;
    // asynchronous sweeps
    int *version_d = nullptr, *claim_d = nullptr, *nbr_d = nullptr;
    int *finished_d = nullptr;  // [0]: blocks at the launch's sweep limit; [1]: sweeps started
    double *board_d = nullptr;
    int num_cu = 0;
    // right-hand sides the per-RHS buffers hold (ms_reserve grows it)
    int rhs_cap = 1;
    // GMRES inner solves (ms_reserve_krylov): basis vectors, tile partials
    // and per-block records, sized for kry_M steps, kry_inner inner
    // elements, kry_rhs right-hand sides and kry_tiles tiles
    int kry_M = 0, kry_rhs = 0;
    long long kry_inner = 0, kry_tiles = 0;
    void *V = nullptr;
    double *gpart = nullptr, *gm = nullptr;
    // replayed sweep pairs
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    unsigned char graph_key[256] = {0};
    // profiling
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_class;
    int ev_used = 0;
    bool profiling = false;
    double prof_ms[8] = {0};        // timed launches drained from the event pool
    long long prof_n[8] = {0};
    std::string err;
};

namespace ms {
thread_local LaunchEvents g_launch_events;
}

namespace {

ms_status fail(ms_handle *h, ms_status s, const std::string &msg) {
    if (h) h->err = msg;
    else g_create_error = msg;
    if (getenv("MS_LOG")) fprintf(stderr, "[libms] %s: %s\n", ms_status_string(s), msg.c_str());
    return s;
}

ms_status hip_fail(ms_handle *h, hipError_t e, const char *what) {
    return fail(h, e == hipErrorOutOfMemory ? MS_ERR_NOMEM : MS_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

bool valid_cuts(const std::vector<int> &c, long long n) {
    if (c.size() < 2 || c.front() != 0 || c.back() != n) return false;
    for (size_t t = 0; t + 1 < c.size(); t++)
        if (c[t + 1] <= c[t]) return false;
    return true;
}

// A device allocation that covers [p, p + bytes).
bool dev_range_ok(const void *p, size_t bytes) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) return false;
    void *base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (const char *)p + bytes <= (const char *)base + size;
}

// Inner-solve box of block b: the block, grown across every face that has
// a neighbour (clipped to the grid) by the overlap depth in x and y and by
// the depth rounded up to the widest vector width in z (so every vector
// width the handle uses divides the box's z offset and extent), with the
// block's own cells recorded inside it.  The region proper is the box minus
// its edge and corner parts and minus the z cells beyond the depth.
void region_box(const ms_handle *h, int b, BlockInfo &B) {
    const int bi = b / (h->gy * h->gz), bj = (b / h->gz) % h->gy, bk = b % h->gz;
    const int o = h->overlap;
    const int oz = (o + h->vzbase - 1) / h->vzbase * h->vzbase;
    const int grow[3] = {o, o, oz};
    const int c0[3] = {h->cx[bi], h->cy[bj], h->cz[bk]};
    const int c1[3] = {h->cx[bi + 1], h->cy[bj + 1], h->cz[bk + 1]};
    const long long n[3] = {h->nx, h->ny, h->nz};
    int lo[3], ext[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = std::min(grow[a], c0[a]);
        const int hi = (int)std::min<long long>(grow[a], n[a] - c1[a]);
        ext[a] = c1[a] - c0[a] + lo[a] + hi;
    }
    B.i0 = c0[0] - lo[0]; B.j0 = c0[1] - lo[1]; B.k0 = c0[2] - lo[2];
    B.bx = ext[0]; B.by = ext[1]; B.bz = ext[2];
    B.oi = lo[0]; B.oj = lo[1]; B.ok = lo[2];
    B.obx = c1[0] - c0[0]; B.oby = c1[1] - c0[1]; B.obz = c1[2] - c0[2];
    B.dep = o;
}

// Build the tile table for vector width vz, x chunk tx and rows per thread.
ms_status set_tiling(ms_handle *h, int vz, int tx, int rows, hipStream_t st) {
    if (h->cur_vz == vz && h->cur_tx == tx && h->cur_rows == rows) return MS_OK;
    std::vector<int> tb;
    h->blocks_h.resize(h->nblocks);
    long long off = 0;
    int tile = 0;
    for (int bi = 0; bi < h->gx; bi++)
        for (int bj = 0; bj < h->gy; bj++)
            for (int bk = 0; bk < h->gz; bk++) {
                const int b = (bi * h->gy + bj) * h->gz + bk;
                BlockInfo &B = h->blocks_h[b];
                region_box(h, b, B);
                B.off = off;
                const long long P = (long long)B.by * B.bz;
                const long long slots = (long long)((B.by + rows - 1) / rows) * (B.bz / vz);
                B.nplane = (int)((slots + ms::kThreads - 1) / ms::kThreads);
                const int nxc = (B.bx + tx - 1) / tx;
                B.ntiles = B.nplane * nxc;
                B.tile0 = tile;
                for (int t = 0; t < B.ntiles; t++) tb.push_back(b);
                tile += B.ntiles;
                off += (long long)B.bx * P;
            }
    if (tile > h->tiles_cap) return fail(h, MS_ERR_ARG, "tiling exceeds its table");
    HIPCHK(h, hipMemcpyAsync(h->blocks_d, h->blocks_h.data(), sizeof(BlockInfo) * h->nblocks,
                             hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(h->tile_block_d, tb.data(), sizeof(int) * tb.size(),
                             hipMemcpyHostToDevice, st));
    HIPCHK(h, hipStreamSynchronize(st));
    h->ntiles = tile;
    h->cur_vz = vz;
    h->cur_tx = tx;
    h->cur_rows = rows;
    return MS_OK;
}

Geom geom(const ms_handle *h) {
    Geom g;
    g.nx = h->nx; g.ny = h->ny; g.nz = h->nz;
    g.blocks = h->blocks_d;
    g.tile_block = h->tile_block_d;
    g.tx = h->cur_tx;
    g.rows = h->cur_rows;
    g.nblocks = h->nblocks;
    g.ovl = h->overlap > 0 ? 1 : 0;
    return g;
}

Faces faces(const ms_handle *h) {
    Faces f;
    for (int t = 0; t < 6; t++) f.f[t] = h->faces_d[t];
    return f;
}

void drop_graph(ms_handle *h);

// Copies the boundary faces into handle-owned buffers (a NULL face frees its
// buffer).  Faces whose buffer stays put are overwritten in place, which a
// captured sweep graph sees on its next replay; a face buffer that is
// allocated or freed invalidates the graph.
ms_status copy_bc(ms_handle *h, const ms_bc *bc) {
    const long long sz[6] = {h->ny * h->nz, h->ny * h->nz, h->nx * h->nz,
                             h->nx * h->nz, h->nx * h->ny, h->nx * h->ny};
    for (int t = 0; t < 6; t++) {
        const double *src = bc ? bc->face[t] : nullptr;
        if (src && !dev_range_ok(src, sizeof(double) * sz[t]))
            return fail(h, MS_ERR_ARG, "boundary face " + std::to_string(t) +
                                           " is not a device buffer of the face's size");
    }
    for (int t = 0; t < 6; t++) {
        const double *src = bc ? bc->face[t] : nullptr;
        if (!src) {
            if (h->faces_d[t]) {
                // a captured sweep graph holds this face pointer: drop it
                // before the buffer goes
                drop_graph(h);
                (void)hipFree(h->faces_d[t]);
                h->faces_d[t] = nullptr;
            }
            continue;
        }
        if (!h->faces_d[t]) {
            drop_graph(h);   // the graph was captured with this face absent
            HIPCHK(h, hipMalloc(&h->faces_d[t], sizeof(double) * sz[t]));
        }
        HIPCHK(h, hipMemcpy(h->faces_d[t], src, sizeof(double) * sz[t], hipMemcpyDeviceToDevice));
    }
    return MS_OK;
}

void free_all(ms_handle *h) {
    void *ps[] = {h->blocks_d, h->tile_block_d, h->x1, h->r, h->d, h->p0, h->p1, h->part64,
                  h->partT, h->psig, h->prhoA, h->prhoB, h->active, h->ctrl, h->history_d,
                  h->scal_d, h->cg_block_d, h->cg_tiles_d, h->version_d, h->claim_d,
                  h->nbr_d, h->finished_d, h->board_d, h->V, h->gpart, h->gm, h->team_mem,
                  h->team_ctr};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    for (int t = 0; t < 6; t++)
        if (h->faces_d[t]) (void)hipFree(h->faces_d[t]);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
}

// ---- profiling -------------------------------------------------------

// Moves the timings of the recorded launches into the per-class totals and
// empties the event pool (waits for those launches).
void prof_drain(ms_handle *h) {
    for (int s = 0; s + 1 < h->ev_used; s += 2) {
        float ms_ = 0.f;
        if (h->ev_class[s] >= 0 && hipEventSynchronize(h->ev[s + 1]) == hipSuccess &&
            hipEventElapsedTime(&ms_, h->ev[s], h->ev[s + 1]) == hipSuccess) {
            h->prof_ms[h->ev_class[s]] += ms_;
            h->prof_n[h->ev_class[s]] += 1;
        }
    }
    h->ev_used = 0;
}

// Times the one launch in its scope with a pair of events attached to that
// dispatch (kernel time alone).  A full pool is drained first, so every
// launch of a profiled solve is timed; a scope that launched nothing leaves
// its slot out.
struct Prof {
    ms_handle *h;
    int slot;
    Prof(ms_handle *h_, hipStream_t, int c) : h(h_), slot(-1) {
        if (!h->profiling) return;
        if (h->ev_used + 2 > (int)h->ev.size()) prof_drain(h);
        slot = h->ev_used;
        h->ev_used += 2;
        h->ev_class[slot] = c;
        ms::g_launch_events = {h->ev[slot], h->ev[slot + 1], true};
    }
    ~Prof() {
        if (slot >= 0 && ms::g_launch_events.pending) {
            ms::g_launch_events.pending = false;
            h->ev_class[slot] = -1;
        }
    }
};

void prof_collect(ms_handle *h, ms_stats *stats) {
    if (!h->profiling) return;
    prof_drain(h);
    for (int c = 0; c < 8; c++) {
        if (stats) {
            stats->kernel_ms[c] += h->prof_ms[c];
            stats->kernel_launches[c] += h->prof_n[c];
        }
        h->prof_ms[c] = 0.0;
        h->prof_n[c] = 0;
    }
}

ms_status prof_begin(ms_handle *h, bool on) {
    h->profiling = on;
    h->ev_used = 0;
    for (int c = 0; c < 8; c++) { h->prof_ms[c] = 0.0; h->prof_n[c] = 0; }
    if (on && h->ev.empty()) {
        h->ev.resize(2 * kMaxEvents);
        h->ev_class.assign(2 * kMaxEvents, 0);
        for (auto &e : h->ev) HIPCHK(h, hipEventCreate(&e));
    }
    return MS_OK;
}

// ---- solve pieces -------------------------------------------------------

// Inner-vector cells of block b (its region's box).
long long block_cells(const ms_handle *h, int b) {
    BlockInfo B;
    region_box(h, b, B);
    return (long long)B.bx * B.by * B.bz;
}

template <typename T>
struct Bufs {
    T *r, *d, *p[2];
    T *pT, *psig, *prA, *prB;
};

template <typename T>
Bufs<T> bufs(ms_handle *h) {
    Bufs<T> B;
    B.r = (T *)h->r;
    B.d = (T *)h->d;
    B.p[0] = (T *)h->p0;
    B.p[1] = (T *)h->p1;
    // FP64 without overlap shares the FP64 partials; with overlap the
    // region sums (inner CG) and own-cell sums (global residual) differ
    B.pT = sizeof(T) == sizeof(double) && h->overlap == 0 ? (T *)h->part64 : (T *)h->partT;
    B.psig = (T *)h->psig;
    B.prA = (T *)h->prhoA;
    B.prB = (T *)h->prhoB;
    return B;
}

// Strides of the per-right-hand-side arrays (a right-hand side owns N
// elements of b, x and the second outer buffer, inner_n of every inner
// vector, tiles_cap partial slots and nblocks flags).
Batch batch_of(const ms_handle *h, int nrhs) {
    Batch bt;
    bt.nt = 0;
    bt.nrhs = nrhs;
    bt.vs = h->N;
    bt.ps = h->tiles_cap;
    bt.bs = h->nblocks;
    bt.is = h->inner_n;
    bt.k0 = 0;
    bt.nk = nrhs;
    return bt;
}

// Consecutive blocks whose volume stays within cap_cells (at least one
// block each).  Returns block ranges; tile ranges are filled by fill_tiles.
std::vector<Group> make_groups(const ms_handle *h, long long cap_cells) {
    std::vector<Group> gs;
    int b = 0;
    while (b < h->nblocks) {
        Group g;
        g.b0 = b;
        long long cells = 0;
        do {
            cells += block_cells(h, b);
            b++;
        } while (b < h->nblocks && cells + block_cells(h, b) <= cap_cells);
        g.b1 = b;
        g.t0 = g.t1 = 0;
        g.off = 0;
        g.k0 = 0;
        g.k1 = 1;
        gs.push_back(g);
    }
    return gs;
}

// (right-hand side, block) work items: every block group of `gs` is split
// into launches of as many right-hand sides as keep the launch's inner
// vectors within cap_cells (at least one), so a group's m inner iterations
// re-read them from the on-package cache.  Returns the largest number of
// right-hand sides in one launch.
int split_rhs(const ms_handle *h, std::vector<Group> &gs, int nrhs, long long cap_cells) {
    std::vector<Group> out;
    int qmax = 1;
    for (const Group &g : gs) {
        long long cells = 0;
        for (int b = g.b0; b < g.b1; b++) cells += block_cells(h, b);
        const int q = (int)std::max(1ll, std::min<long long>(nrhs, cap_cells / std::max(1ll, cells)));
        qmax = std::max(qmax, q);
        for (int k = 0; k < nrhs; k += q) {
            Group c = g;
            c.k0 = k;
            c.k1 = std::min(nrhs, k + q);
            out.push_back(c);
        }
    }
    gs.swap(out);
    return qmax;
}

void fill_tiles(const ms_handle *h, std::vector<Group> &gs) {
    for (Group &g : gs) {
        g.off = h->blocks_h[g.b0].off;
        g.t0 = h->blocks_h[g.b0].tile0;
        g.t1 = h->blocks_h[g.b1 - 1].tile0 + h->blocks_h[g.b1 - 1].ntiles;
    }
}

ms::GmArgs gm_args(const ms_handle *h) {
    ms::GmArgs a;
    a.gm = h->gm;
    a.gpart = h->gpart;
    a.kvs = h->kry_inner * h->kry_rhs;
    a.M = h->kry_M;
    a.gstride = h->kry_M + 2;
    a.nblocks = h->nblocks;
    a.rec_stride = ms::gm_record_doubles(h->kry_M);
    return a;
}

// One sweep with GMRES(m) inner solves: per group, the residual (written as
// the first, unscaled Krylov vector), m Arnoldi steps of three launches, the
// per-block triangular solves and x_new = x_old + V y on own cells.
template <typename T>
ms_status enqueue_sweep_gmres(ms_handle *h, const std::vector<Group> &groups, const double *b,
                              const double *xa, double *xb, double tol, int m, double inner_tol,
                              bool final_only, Batch bt, hipStream_t st) {
    const Geom g = geom(h);
    const int vz = h->cur_vz;
    Bufs<T> B = bufs<T>(h);
    const Faces F = faces(h);
    T *V = (T *)h->V;
    const ms::GmArgs a = gm_args(h);
    for (const Group &G : groups) {
        {
            Prof p(h, st, MS_K_RESID);
            HIPCHK(h, ms::launch_resid<T>(g, vz, G.t0, G.t1, G.off, b, xa, F,
                                          final_only ? nullptr : V, h->part64, B.pT, h->ctrl,
                                          bt, st));
        }
        if (final_only) continue;
        {
            Prof p(h, st, MS_K_HESS);
            HIPCHK(h, ms::launch_gm_init<T>(g, G.b0, G.b1, B.pT, bt, a, h->ctrl, st));
        }
        static const int cls[3] = {MS_K_STENCIL, MS_K_ORTH, MS_K_HESS};
        for (int j = 0; j < m; j++)
            for (int part = 0; part < 3; part++) {
                Prof p(h, st, cls[part]);
                HIPCHK(h, ms::launch_gm_step<T>(g, vz, G.t0, G.t1, G.b0, G.b1, G.off, V, j,
                                                inner_tol, bt, a, h->ctrl, st, part));
            }
        for (int part = 0; part < 2; part++) {
            Prof p(h, st, part ? MS_K_FINAL : MS_K_HESS);
            HIPCHK(h, ms::launch_gm_finish<T>(g, vz, G.t0, G.t1, G.b0, G.b1, G.off, V, xa, xb, bt,
                                              a, h->ctrl, st, part));
        }
    }
    {
        Prof p(h, st, MS_K_CHECK);
        HIPCHK(h, ms::launch_check(h->part64, h->ntiles, tol, final_only ? 1 : 0, h->history_d,
                                   kHistoryCap, h->ctrl, bt, st));
    }
    return MS_OK;
}

// Enqueue one sweep of every right-hand side from xa into xb (or, final_only,
// just the residual check of xa).  inner: ms_inner.
template <typename T>
ms_status enqueue_sweep(ms_handle *h, const std::vector<Group> &groups, const double *b,
                        const double *xa, double *xb, double tol, int m, double inner_tol,
                        int inner, bool final_only, Batch bt, hipStream_t st) {
    if (inner == MS_INNER_GMRES)
        return enqueue_sweep_gmres<T>(h, groups, b, xa, xb, tol, m, inner_tol, final_only, bt, st);
    const Geom g = geom(h);
    const int vz = h->cur_vz;
    Bufs<T> B = bufs<T>(h);
    const Faces F = faces(h);
    for (const Group &G : groups) {
        bt.k0 = G.k0;          // this launch's right-hand sides
        bt.nk = G.k1 - G.k0;
        {
            Prof p(h, st, MS_K_RESID);
            HIPCHK(h, ms::launch_resid<T>(g, vz, G.t0, G.t1, G.off, b, xa, F,
                                          final_only ? nullptr : B.r, h->part64, B.pT, h->ctrl,
                                          bt, st));
        }
        if (final_only) continue;
        T *prho[3] = {B.pT, B.prA, B.prB};
        for (int j = 0; j < m; j++) {
            T *cur = j == 0 ? prho[0] : (j % 2 ? prho[1] : prho[2]);
            T *prev = j == 0 ? prho[0] : (j == 1 ? prho[0] : (j % 2 ? prho[2] : prho[1]));
            T *next = (j + 1) % 2 ? prho[1] : prho[2];
            T *pold = B.p[(j + 1) % 2];
            T *pnew = B.p[j % 2];
            const bool last = j == m - 1;
            {
                Prof p(h, st, MS_K_STENCIL);
                HIPCHK(h, ms::launch_stencil<T>(g, vz, G.t0, G.t1, G.off, B.r, pold, pnew,
                                                B.psig, cur, prev, prho[0], h->active, j,
                                                inner_tol, h->ctrl, bt, st));
            }
            {
                Prof p(h, st, last ? MS_K_FINAL : MS_K_UPDATE);
                HIPCHK(h, ms::launch_update<T>(g, vz, G.t0, G.t1, G.off, B.r, pnew, B.d,
                                               B.psig, cur, next, h->active, j, last ? 1 : 0,
                                               xa, xb, h->ctrl, bt, st));
            }
        }
    }
    bt.k0 = 0;
    bt.nk = bt.nrhs;
    {
        Prof p(h, st, MS_K_CHECK);
        HIPCHK(h, ms::launch_check(h->part64, h->ntiles, tol, final_only ? 1 : 0, h->history_d,
                                   kHistoryCap, h->ctrl, bt, st));
    }
    return MS_OK;
}

__global__ void k_ctrl_init(Ctrl *c, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        c[k].done = 0; c[k].status = 0; c[k].sweep = 0; c[k].final_sweep = 0;
        c[k].nbeff = 0.0; c[k].res0 = 0.0; c[k].last_res = 0.0;
        c[k].inner_iters = 0ull; c[k].inner_snap = 0ull;
        c[k].stop = 0; c[k].max_stale = 0; c[k].work_items = 0ull;
    }
}

// A right-hand side with b_eff = 0 is solved by x = 0 before any sweep.
__global__ void k_mark_zero_rhs(Ctrl *c, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && c[k].nbeff == 0.0) { c[k].done = 1; c[k].status = 0; c[k].final_sweep = 0; }
}

__global__ void k_fill_zero(double *x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

ms_status zero_vec(ms_handle *h, double *x, long long n, hipStream_t st) {
    long long grid = std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::max<long long>(grid, 1)), dim3(256), 0,
                       st, x, n);
    HIPCHK(h, hipGetLastError());
    return MS_OK;
}

// ||b_eff|| of every right-hand side into ctrl[k].nbeff and out[k] (host);
// resets the control blocks.
template <typename T>
ms_status beff_norms(ms_handle *h, const double *b, int nrhs, hipStream_t st, double *out) {
    hipLaunchKernelGGL(k_ctrl_init, dim3((nrhs + 63) / 64), dim3(64), 0, st, h->ctrl, nrhs);
    HIPCHK(h, hipGetLastError());
    const Geom g = geom(h);
    Bufs<T> B = bufs<T>(h);
    const Batch bt = batch_of(h, nrhs);
    HIPCHK(h, ms::launch_resid<T>(g, h->cur_vz, 0, h->ntiles, 0, b, nullptr, faces(h), nullptr,
                                  h->part64, B.pT, nullptr, bt, st));
    for (int k = 0; k < nrhs; k++)
        HIPCHK(h, ms::launch_norm(h->part64 + (long long)k * h->tiles_cap, h->ntiles, h->ctrl + k, st));
    std::vector<Ctrl> c(nrhs);
    HIPCHK(h, hipMemcpyAsync(c.data(), h->ctrl, sizeof(Ctrl) * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    for (int k = 0; k < nrhs; k++) out[k] = c[k].nbeff;
    return MS_OK;
}

template <typename T>
ms_status beff_norm(ms_handle *h, const double *b, hipStream_t st, double *out) {
    return beff_norms<T>(h, b, 1, st, out);
}

// Tile choice when the caller leaves it open, for launches over blocks
// [b0, b1): the longest x chunk, then the most rows per thread, that still
// give at least kMinTiles workgroups per launch (per right-hand side count
// nrhs).  Measured on 512^3 with 64^3 blocks in cache-sized groups: about
// 1024 workgroups per launch and chunks of 8-16 planes are best.
constexpr long long kMinTiles = 1024;

long long count_tiles(const ms_handle *h, int vz, int tx, int rows, int b0, int b1) {
    long long n = 0;
    for (int b = b0; b < b1; b++) {
        BlockInfo B;
        region_box(h, b, B);
        const long long slots = (long long)((B.by + rows - 1) / rows) * (B.bz / vz);
        n += ((slots + ms::kThreads - 1) / ms::kThreads) * ((B.bx + tx - 1) / tx);
    }
    return n;
}

// Tile-table capacity: the narrowest vector, one row per thread and the
// smallest x chunk give the most tiles.
long long tile_capacity(const ms_handle *h) {
    return count_tiles(h, 1, kTxMin, 1, 0, h->nblocks);
}

// Rows per thread the asynchronous CG worker fits in the 128 registers a
// 1024-thread workgroup allows: 2 with 2-cell z vectors, 1 with wider ones.
int async_max_rows(int vz) { return vz >= 4 ? 1 : 2; }

// Tiling of the asynchronous CG workers (one workgroup sweeps a whole
// block): the largest tiles within async_max_rows that still give
// kMinTiles tiles in all.
void async_tiling(const ms_handle *h, int vz, int nrhs, int b0, int b1, int *tx, int *rows) {
    for (int t : {32, 16, 8, 4})
        for (int r : {2, 1})
            if (r <= async_max_rows(vz) && count_tiles(h, vz, t, r, b0, b1) * nrhs >= kMinTiles) {
                *tx = t;
                *rows = r;
                return;
            }
    *tx = kTxMin;
    *rows = 1;
}

// Tiling of the synchronous phase kernels: one row per thread and the
// longest x march of 16, 8 or 4 planes that still gives kMinTiles
// workgroups per launch.  Measured: rows 1 with 16 planes is the fastest
// tile at 512^3 (mixed and FP64, with and without overlap), and larger
// tiles (32 planes, 2 or 4 rows) were never faster, by up to 3.5x slower
// on the uneven 16-right-hand-side workload where launches hold many tiles.
void sync_tiling(const ms_handle *h, int vz, int nrhs, int b0, int b1, int *tx, int *rows) {
    *rows = 1;
    *tx = kTxMin;
    for (int t : {16, 8, 4})
        if (count_tiles(h, vz, t, 1, b0, b1) * nrhs >= kMinTiles) { *tx = t; return; }
}

// Inner-vector working set of one launch group: the on-package cache
// (256 MB) holds r, d and both p buffers of the group, so the m inner
// iterations re-read them from the cache rather than from HBM (measured:
// 64 blocks of 64^3 in FP32, 32 in FP64 are the fastest groups).
constexpr long long kGroupBytes = 256ll << 20;

// A HIP graph holding two sweeps (even then odd parity) of one solve
// configuration, replayed instead of launching the kernels one by one.
struct GraphKey {
    const double *b;
    double *x;
    const double *faces[6];   // boundary buffers the captured kernels read
    double tol, inner_tol;
    long long cap_cells;
    int m, tsize, vz, tx, rows, nrhs, overlap, inner;
};
static_assert(sizeof(GraphKey) <= sizeof(ms_handle::graph_key), "graph key storage");

void drop_graph(ms_handle *h) {
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
}

template <typename T>
ms_status sweep_pair_graph(ms_handle *h, const GraphKey &key, const std::vector<Group> &groups,
                           const double *b, double *const X[2], double tol, int m,
                           double inner_tol, int inner, Batch bt) {
    if (h->graph_exec && memcmp(&h->graph_key, &key, sizeof(GraphKey)) == 0) return MS_OK;
    drop_graph(h);
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    ms_status s = enqueue_sweep<T>(h, groups, b, X[0], X[1], tol, m, inner_tol, inner, false, bt,
                                   h->cap_stream);
    if (s == MS_OK)
        s = enqueue_sweep<T>(h, groups, b, X[1], X[0], tol, m, inner_tol, inner, false, bt,
                             h->cap_stream);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &gr);
    if (s != MS_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return s;
    }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    h->graph = gr;
    HIPCHK(h, hipGraphInstantiate(&h->graph_exec, gr, nullptr, nullptr, 0));
    memcpy(&h->graph_key, &key, sizeof(GraphKey));
    return MS_OK;
}

// ---- resident-team solves ------------------------------------------------------

// LDS a team workgroup may use (160 KB per compute unit, less its static
// shared variables) and the vector slots per thread the kernels exist for.
constexpr size_t kTeamLds = 163840 - 1024;
constexpr int kTeamMaxSpin = 1 << 24;   // polls before a team barrier gives up (seconds)

struct TeamPlan {
    bool ok = false;
    int T = 0, q = 0, vz = 0, per_xcd = 0;
    size_t lds = 0;
    long long face_stride = 0, team_bytes = 0;
    std::string why;
};

// Team shape for the handle's blocks (their overlap boxes when overlap is
// on) with inner type size tsize: the smallest team (most teams at once)
// whose members' slabs fit in LDS (p and d) and in the vector slots a
// thread has.
TeamPlan team_plan(const ms_handle *h, int tsize) {
    TeamPlan P;
    if (h->num_cu < 8 || h->num_cu % 8) { P.why = "compute units not a multiple of 8"; return P; }
    P.per_xcd = h->num_cu / 8;
    int vz = std::min(h->vzmax, tsize == 4 ? 4 : 2);
    if (h->overlap > 0) vz = std::min(vz, h->vzbase);
    P.vz = vz;
    int minbx = 1 << 30, maxbx = 0;
    long long maxplane = 0;
    for (int b = 0; b < h->nblocks; b++) {
        BlockInfo B;
        region_box(h, b, B);
        minbx = std::min(minbx, B.bx);
        maxbx = std::max(maxbx, B.bx);
        maxplane = std::max(maxplane, (long long)B.by * B.bz);
    }
    P.face_stride = maxplane;
    const int nthreads = ms::team_threads();
    for (int T : {1, 2, 4, 8, 16, 32}) {
        if (T > P.per_xcd || P.per_xcd % T || T > minbx) continue;
        long long cells = 0;
        for (int b = 0; b < h->nblocks; b++) {
            BlockInfo B;
            region_box(h, b, B);
            const long long planes = (B.bx + T - 1) / T;
            cells = std::max(cells, planes * B.by * B.bz);
        }
        // p in LDS with a halo plane on each side (r and d in registers)
        long long pb = 0;
        for (int b = 0; b < h->nblocks; b++) {
            BlockInfo B;
            region_box(h, b, B);
            pb = std::max(pb, (long long)((B.bx + T - 1) / T + 2) * B.by * B.bz);
        }
        const size_t lds = (size_t)pb * tsize;
        if (lds > kTeamLds) continue;
        const long long need = (cells / vz + nthreads - 1) / nthreads;
        int q = 0;
        for (int c : {2, 4, 8, 12})   // (16 slots spill registers in FP64)
            if (c >= need) { q = c; break; }
        if (!q) continue;
        P.ok = true;
        P.T = T;
        P.q = q;
        P.lds = std::max<size_t>(lds, 16);
        // each member's two r face planes
        P.team_bytes = ((ms::team_face_offset() + 2ll * T * P.face_stride * tsize) + 255) / 256 * 256;
        return P;
    }
    P.why = "a block's slab does not fit a team workgroup";
    return P;
}

// Team memory for the current geometry, for both inner types (never shrinks).
ms_status team_alloc(ms_handle *h) {
    size_t need = 0;
    for (int tsize : {4, 8}) {
        const TeamPlan P = team_plan(h, tsize);
        if (P.ok) need = std::max(need, (size_t)(8 * P.per_xcd / P.T) * (size_t)P.team_bytes);
    }
    if (need <= h->team_mem_bytes) return MS_OK;
    char *fresh = nullptr;
    const hipError_t e = hipMalloc(&fresh, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return MS_OK;   // the team engine stays unavailable for this geometry
    }
    if (h->team_mem) (void)hipFree(h->team_mem);
    h->team_mem = fresh;
    h->team_mem_bytes = need;
    return MS_OK;
}

// ctr: [0] next block, [1] error code (kept), [2..9] workgroups per XCD,
// [10] workgroups arrived
// Every team's header (barrier counter, work ring, partial-sum slots: the
// first clear_ints ints of its memory) to zero.
__global__ void k_team_reset(char *mem, long long team_bytes, int nteams, int clear_ints,
                             int *ctr) {
    const long long n = (long long)nteams * clear_ints;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        ((int *)(mem + (i / clear_ints) * team_bytes))[i % clear_ints] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 11 && threadIdx.x != 1) ctr[threadIdx.x] = 0;
}

// The plan to use for a solve, or !ok (with the reason) for the phase engine.
TeamPlan team_for_solve(ms_handle *h, int tsize, const ms_opts &o, int nrhs) {
    TeamPlan P;
    if (o.engine == MS_ENGINE_PHASE) { P.why = "phase engine requested"; return P; }
    if (o.engine == MS_ENGINE_AUTO &&
        (o.group_blocks != 0 || o.x_chunk > 0 || o.rows > 0 || o.z_vector > 0 || o.workers > 0)) {
        P.why = "a tiling option of the phase engine was set";
        return P;
    }
    if (o.inner_solver != MS_INNER_CG) { P.why = "GMRES inner solves"; return P; }
    if (nrhs != 1) { P.why = "several right-hand sides"; return P; }
    P = team_plan(h, tsize);
    if (P.ok && (size_t)(8 * P.per_xcd / P.T) * (size_t)P.team_bytes > h->team_mem_bytes) {
        P.ok = false;
        P.why = "team memory not allocated";
    }
    return P;
}

template <typename T>
ms_status enqueue_team(ms_handle *h, const TeamPlan &P, const double *b, const double *xa,
                       double *xb, int m, double inner_tol, bool async, AsyncState as, int S,
                       int limit, double tol2, int spin, hipStream_t st) {
    const int nteams = 8 * P.per_xcd / P.T;
    const int clear_ints = ms::team_face_offset() / (int)sizeof(int);
    const int rgrid = (int)std::min<long long>(256, ((long long)nteams * clear_ints + 255) / 256);
    hipLaunchKernelGGL(k_team_reset, dim3(rgrid), dim3(256), 0, st, h->team_mem,
                       (long long)P.team_bytes, nteams, clear_ints, h->team_ctr);
    HIPCHK(h, hipGetLastError());
    ms::TeamArgs a;
    a.T = P.T;
    a.per_xcd = P.per_xcd;
    a.nwork = h->nblocks;
    a.next = h->team_ctr;
    a.err = h->team_ctr + 1;
    a.xcd_count = h->team_ctr + 2;
    a.arrived = h->team_ctr + 10;
    a.team_mem = h->team_mem;
    a.team_bytes = P.team_bytes;
    a.face_stride = P.face_stride;
    a.m = m;
    a.inner_tol = inner_tol;
    a.b = b;
    a.xa = xa;
    a.xb = xb;
    a.F = faces(h);
    a.p64 = h->part64;
    a.max_spin = spin > 0 ? spin : kTeamMaxSpin;
    Prof p(h, st, MS_K_OTHER);
    HIPCHK(h, ms::launch_team<T>(geom(h), P.vz, P.q, a, async, as, S, limit, tol2, h->ctrl,
                                 8 * P.per_xcd, P.lds, st));
    return MS_OK;
}

// Error code the team kernels left (0: none); clears it.  Under MS_LOG
// prints how the last launch's workgroups fell on the XCDs.
ms_status team_error(ms_handle *h, hipStream_t st) {
    int ctr[11] = {0};
    HIPCHK(h, hipMemcpyAsync(ctr, h->team_ctr, sizeof(ctr), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    const int err = ctr[1];
    if (getenv("MS_LOG")) {
        fprintf(stderr, "[libms] team launch: workgroups per XCD");
        for (int q = 0; q < 8; q++) fprintf(stderr, " %d", ctr[2 + q]);
        fprintf(stderr, ", arrived %d, error %d\n", ctr[10], err);
    }
    if (err == 0) return MS_OK;
    const int zero = 0;
    HIPCHK(h, hipMemcpy(h->team_ctr + 1, &zero, sizeof(int), hipMemcpyHostToDevice));
    return fail(h, MS_ERR_HIP, err == 1   ? "team engine: an XCD id outside 0..7"
                               : err == 2 ? "team engine: a team barrier timed out"
                                          : "team engine: the launch's workgroups did not all start");
}

// Synchronous solve of one right-hand side on the resident-team engine: per
// sweep one cooperative launch sweeps every block from one outer buffer into
// the other (team kernels compute each block's residual, CG and update) and
// writes each block's own-cell residual of the old iterate; a one-workgroup
// kernel then sums those in block order and tests convergence.
template <typename T>
ms_status solve_sync_team(ms_handle *h, const TeamPlan &P, const double *b, double *x,
                          double tol, int m, const ms_opts &o, ms_stats *stats, hipStream_t st) {
    double nbeff = 0.0;
    ms_status s = beff_norms<T>(h, b, 1, st, &nbeff);
    if (s != MS_OK) return s;
    if (!std::isfinite(nbeff)) return fail(h, MS_ERR_NONFINITE, "b_eff is not finite");
    if (nbeff == 0.0) {
        s = zero_vec(h, x, h->N, st);
        if (s != MS_OK) return s;
    }
    hipLaunchKernelGGL(k_mark_zero_rhs, dim3(1), dim3(64), 0, st, h->ctrl, 1);
    HIPCHK(h, hipGetLastError());
    const long long cells_per_sweep = h->N * (long long)m;
    const int batch = o.check_every > 0
                          ? o.check_every
                          : (int)std::max(2ll, std::min(256ll, (1ll << 31) / std::max(1ll, cells_per_sweep)));
    s = prof_begin(h, o.profile != 0);
    if (s != MS_OK) return s;
    double *X[2] = {x, h->x1};
    // the final check of x^(max_sweeps) uses the residual kernels over all tiles
    std::vector<Group> all(1);
    all[0].b0 = 0; all[0].b1 = h->nblocks; all[0].k0 = 0; all[0].k1 = 1;
    fill_tiles(h, all);
    const Batch bt = batch_of(h, 1);
    AsyncState none{};
    Ctrl c;
    int next = 0;
    for (;;) {
        const int nb = std::min(batch, o.max_sweeps - next);
        for (int q = 0; q < nb; q++, next++) {
            s = enqueue_team<T>(h, P, b, X[next % 2], X[(next + 1) % 2], m, o.inner_tol, false,
                                none, 0, 0, 0.0, o.team_spin, st);
            if (s != MS_OK) return s;
            Prof p(h, st, MS_K_CHECK);
            HIPCHK(h, ms::launch_check(h->part64, h->nblocks, tol, 0, h->history_d, kHistoryCap,
                                       h->ctrl, bt, st));
        }
        if (next == o.max_sweeps) {
            s = enqueue_sweep<T>(h, all, b, X[next % 2], nullptr, tol, m, o.inner_tol,
                                 MS_INNER_CG, true, bt, st);
            if (s != MS_OK) return s;
        }
        HIPCHK(h, hipMemcpyAsync(&c, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        s = team_error(h, st);
        if (s != MS_OK) return s;
        prof_collect(h, stats);
        if (c.done) break;
        if (next >= o.max_sweeps) return fail(h, MS_ERR_HIP, "device did not finish the solve");
    }
    if (c.final_sweep % 2 == 1)
        HIPCHK(h, hipMemcpyAsync(x, h->x1, sizeof(double) * h->N, hipMemcpyDeviceToDevice, st));
    HIPCHK(h, hipStreamSynchronize(st));
    if (stats) {
        stats->sweeps = c.final_sweep;
        stats->inner_iters = (int64_t)c.inner_snap;
        stats->rel_residual = nbeff == 0.0 ? 0.0 : c.last_res;
        if (stats->block_sweeps)
            for (int q = 0; q < std::min(h->nblocks, stats->block_sweeps_cap); q++)
                stats->block_sweeps[q] = c.final_sweep;
        if (stats->history && stats->history_cap > 0) {
            const int n = std::min(std::min(stats->history_cap, kHistoryCap), c.final_sweep + 1);
            if (nbeff == 0.0) {
                stats->history[0] = 0.0;
                stats->history_len = 1;
            } else {
                HIPCHK(h, hipMemcpy(stats->history, h->history_d, sizeof(double) * n,
                                    hipMemcpyDeviceToHost));
                stats->history_len = n;
            }
        }
    }
    switch (c.status) {
        case 0: return MS_OK;
        case 4: return fail(h, MS_ERR_NOT_CONVERGED, "max_sweeps reached above tol");
        case 5: return fail(h, MS_ERR_NONFINITE, "residual became non-finite");
        case 6: return fail(h, MS_ERR_DIVERGED, "residual grew by 1e6");
        default: return fail(h, MS_ERR_HIP, "unknown device status");
    }
}

// Synchronous solve of nrhs right-hand sides stored one after another in b
// and x (each nx*ny*nz).  stats: nrhs entries or NULL.
template <typename T>
ms_status solve_sync(ms_handle *h, const double *b, double *x, int nrhs, double tol, int m,
                     const ms_opts &o, ms_stats *stats, hipStream_t st) {
    if (nrhs > h->rhs_cap) return fail(h, MS_ERR_ARG, "more right-hand sides than reserved");
    {
        const TeamPlan P = team_for_solve(h, (int)sizeof(T), o, nrhs);
        if (P.ok) {
            if (stats) stats->engine_used = MS_ENGINE_TEAM;
            return solve_sync_team<T>(h, P, b, x, tol, m, o, stats, st);
        }
        if (o.engine == MS_ENGINE_TEAM)
            return fail(h, MS_ERR_UNSUPPORTED, "team engine unavailable: " + P.why);
        if (stats)
            for (int k = 0; k < nrhs; k++) stats[k].engine_used = MS_ENGINE_PHASE;
    }
    const bool gmres = o.inner_solver == MS_INNER_GMRES;
    if (gmres && (m > h->kry_M || nrhs > h->kry_rhs || h->inner_n > h->kry_inner ||
                  h->tiles_cap > h->kry_tiles))
        return fail(h, MS_ERR_ARG,
                    "GMRES inner solves need ms_reserve_krylov(h, >= inner_iters) after the "
                    "last ms_reserve / ms_set_overlap");
    // z cells per thread access: 16 bytes of the inner type by default; up
    // to 32 bytes on request (a wavefront then spans more y rows, but the
    // FP64 x and b accesses of the residual and final kernels double too:
    // measured slower at 512^3).  GMRES kernels take at most 16 bytes;
    // overlap boxes are aligned to vzbase.
    int vzlim = std::min(h->vzmax, (int)((gmres ? 16 : 32) / sizeof(T)));
    if (h->overlap > 0) vzlim = std::min(vzlim, h->vzbase);
    int vz = std::min(vzlim, (int)(16 / sizeof(T)));
    if (o.z_vector > 0) {
        if ((o.z_vector & (o.z_vector - 1)) || o.z_vector > vzlim)
            return fail(h, MS_ERR_ARG, "z_vector must be a power of two the z cuts, nz, the "
                                       "precision and the inner solver allow");
        vz = o.z_vector;
    }
    // blocks per launch: cache-sized groups by default (-1: all blocks at
    // once, > 0: that many blocks).  CG keeps four inner vectors per block;
    // GMRES re-reads its basis at every step, and groups half the CG size
    // were measured fastest for GMRES(10) at 512^3 (32 blocks of 64^3 in
    // FP32, 16 in FP64)
    long long cap_cells = kGroupBytes / ((gmres ? 8 : 4) * (long long)sizeof(T) * nrhs);
    if (o.group_blocks < 0) {
        cap_cells = h->inner_n;
    } else if (o.group_blocks > 0) {
        long long mx = 0;
        for (int bb = 0; bb < h->nblocks; bb++) mx = std::max(mx, block_cells(h, bb));
        cap_cells = mx * o.group_blocks;
    }
    // several right-hand sides with CG inner solves and automatic groups:
    // (right-hand side, block) launches, each within the cache budget
    const bool rhs_items = nrhs > 1 && !gmres && o.group_blocks == 0;
    if (rhs_items) cap_cells *= nrhs;
    std::vector<Group> groups = make_groups(h, cap_cells);
    int per_launch = nrhs;   // right-hand sides in the largest launch
    if (rhs_items) {
        per_launch = split_rhs(h, groups, nrhs, cap_cells);
    } else {
        for (Group &G : groups) { G.k0 = 0; G.k1 = nrhs; }
    }
    int gmax = 0;
    for (size_t q = 0; q < groups.size(); q++)
        if (groups[q].b1 - groups[q].b0 > groups[gmax].b1 - groups[gmax].b0) gmax = (int)q;
    int tx = 0, rows = 0;
    sync_tiling(h, vz, per_launch, groups[gmax].b0, groups[gmax].b1, &tx, &rows);
    if (o.x_chunk > 0) tx = std::max(kTxMin, o.x_chunk);
    if (o.rows == 1 || o.rows == 2 || o.rows == 4) rows = o.rows;
    if (gmres) {
        // GMRES kernels keep a tile's w in registers: one row per thread and
        // at most gm_max_planes() planes
        rows = 1;
        if (o.x_chunk <= 0) {
            tx = kTxMin;
            for (int t = ms::gm_max_planes(); t > kTxMin; t /= 2)
                if (count_tiles(h, vz, t, 1, groups[gmax].b0, groups[gmax].b1) * nrhs >= kMinTiles) {
                    tx = t;
                    break;
                }
        }
        tx = std::min(tx, ms::gm_max_planes());
    }
    ms_status s = set_tiling(h, vz, tx, rows, st);
    if (s != MS_OK) return s;
    fill_tiles(h, groups);
    std::vector<double> nbeff(nrhs, 0.0);
    s = beff_norms<T>(h, b, nrhs, st, nbeff.data());
    if (s != MS_OK) return s;
    for (int k = 0; k < nrhs; k++) {
        if (!std::isfinite(nbeff[k])) return fail(h, MS_ERR_NONFINITE, "b_eff is not finite");
        if (nbeff[k] == 0.0) {
            s = zero_vec(h, x + (long long)k * h->N, h->N, st);
            if (s != MS_OK) return s;
        }
    }
    hipLaunchKernelGGL(k_mark_zero_rhs, dim3((nrhs + 63) / 64), dim3(64), 0, st, h->ctrl, nrhs);
    HIPCHK(h, hipGetLastError());
    const Batch bt = batch_of(h, nrhs);
    const long long cells_per_sweep = h->N * (long long)m * nrhs;
    int batch = o.check_every > 0 ? o.check_every
                                  : (int)std::max(2ll, std::min(256ll, (1ll << 31) / std::max(1ll, cells_per_sweep)));
    const bool graph = o.use_graph != 0 && o.profile == 0;
    if (graph) batch += batch % 2;   // whole sweep pairs
    s = prof_begin(h, o.profile != 0);
    if (s != MS_OK) return s;
    double *X[2] = {x, h->x1};
    if (graph) {
        GraphKey key;
        memset(&key, 0, sizeof(key));
        key.b = b; key.x = x; key.tol = tol;
        for (int t = 0; t < 6; t++) key.faces[t] = h->faces_d[t]; key.inner_tol = o.inner_tol; key.cap_cells = cap_cells;
        key.m = m; key.tsize = (int)sizeof(T); key.vz = vz; key.tx = tx; key.rows = rows;
        key.nrhs = nrhs;
        key.overlap = h->overlap;
        key.inner = o.inner_solver;
        s = sweep_pair_graph<T>(h, key, groups, b, X, tol, m, o.inner_tol, o.inner_solver, bt);
        if (s != MS_OK) return s;
    }
    std::vector<Ctrl> c(nrhs);
    int next = 0;   // next sweep to enqueue
    for (;;) {
        const int nb = std::min(batch, o.max_sweeps - next);
        int q = 0;
        if (graph) {
            for (; q + 2 <= nb; q += 2, next += 2) HIPCHK(h, hipGraphLaunch(h->graph_exec, st));
        }
        for (; q < nb; q++, next++) {
            s = enqueue_sweep<T>(h, groups, b, X[next % 2], X[(next + 1) % 2], tol, m, o.inner_tol,
                                 o.inner_solver, false, bt, st);
            if (s != MS_OK) return s;
        }
        if (next == o.max_sweeps) {
            s = enqueue_sweep<T>(h, groups, b, X[next % 2], nullptr, tol, m, o.inner_tol,
                                 o.inner_solver, true, bt, st);
            if (s != MS_OK) return s;
        }
        HIPCHK(h, hipMemcpyAsync(c.data(), h->ctrl, sizeof(Ctrl) * nrhs, hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        prof_collect(h, stats);
        bool all = true;
        for (int k = 0; k < nrhs; k++) all = all && c[k].done;
        if (all) break;
        if (next >= o.max_sweeps) return fail(h, MS_ERR_HIP, "device did not finish the solve");
    }
    ms_status result = MS_OK;
    for (int k = 0; k < nrhs; k++) {
        if (c[k].final_sweep % 2 == 1)
            HIPCHK(h, hipMemcpyAsync(x + (long long)k * h->N, h->x1 + (long long)k * h->N,
                                     sizeof(double) * h->N, hipMemcpyDeviceToDevice, st));
        ms_status sk = MS_OK;
        switch (c[k].status) {
            case 0: break;
            case 4: sk = MS_ERR_NOT_CONVERGED; break;
            case 5: sk = MS_ERR_NONFINITE; break;
            case 6: sk = MS_ERR_DIVERGED; break;
            default: sk = MS_ERR_HIP; break;
        }
        if (sk != MS_OK && (result == MS_OK || result == MS_ERR_NOT_CONVERGED)) result = sk;
    }
    HIPCHK(h, hipStreamSynchronize(st));
    if (stats) {
        for (int k = 0; k < nrhs; k++) {
            ms_stats &S = stats[k];
            S.sweeps = c[k].final_sweep;
            if (S.block_sweeps)
                for (int q = 0; q < std::min(h->nblocks, S.block_sweeps_cap); q++)
                    S.block_sweeps[q] = c[k].final_sweep;
            S.inner_iters = (int64_t)c[k].inner_snap;
            S.rel_residual = nbeff[k] == 0.0 ? 0.0 : c[k].last_res;
            if (S.history && S.history_cap > 0) {
                const int n = std::min(std::min(S.history_cap, kHistoryCap), c[k].final_sweep + 1);
                if (nbeff[k] == 0.0) {
                    S.history[0] = 0.0;
                    S.history_len = 1;
                } else {
                    HIPCHK(h, hipMemcpy(S.history, h->history_d + (long long)k * kHistoryCap,
                                        sizeof(double) * n, hipMemcpyDeviceToHost));
                    S.history_len = n;
                }
            }
        }
    }
    switch (result) {
        case MS_OK: return MS_OK;
        case MS_ERR_NOT_CONVERGED: return fail(h, result, "max_sweeps reached above tol");
        case MS_ERR_NONFINITE: return fail(h, result, "residual became non-finite");
        case MS_ERR_DIVERGED: return fail(h, result, "residual grew by 1e6");
        default: return fail(h, MS_ERR_HIP, "unknown device status");
    }
}

// ---- residual of an iterate, FP64, without touching the control block ----

// p64 / pT: per-tile partials (ntiles each; pT takes the region sums of
// overlap tiles, unused here); sums: two doubles.  Every tile writes its
// slots, so nothing needs clearing first.
ms_status residual_norms_in(ms_handle *h, const double *b, const double *x, hipStream_t st,
                            double *p64, double *pT, double *sums, double *nbeff,
                            double *absres) {
    const Geom g = geom(h);
    HIPCHK(h, ms::launch_resid<double>(g, h->cur_vz, 0, h->ntiles, 0, b, nullptr, faces(h),
                                       nullptr, p64, pT, nullptr, ms::single_rhs(), st));
    HIPCHK(h, ms::launch_sum(p64, h->ntiles, sums, st));
    HIPCHK(h, ms::launch_resid<double>(g, h->cur_vz, 0, h->ntiles, 0, b, x, faces(h), nullptr,
                                       p64, pT, nullptr, ms::single_rhs(), st));
    HIPCHK(h, ms::launch_sum(p64, h->ntiles, sums + 1, st));
    double ss[2] = {0.0, 0.0};
    HIPCHK(h, hipMemcpyAsync(ss, sums, sizeof(ss), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    *nbeff = std::sqrt(ss[0]);
    *absres = std::sqrt(ss[1]);
    return MS_OK;
}

ms_status residual_norms(ms_handle *h, const double *b, const double *x, hipStream_t st,
                         double *nbeff, double *absres) {
    return residual_norms_in(h, b, x, st, h->part64, (double *)h->partT, h->scal_d, nbeff,
                             absres);
}

// ---- static scratch of the allocation-free residual ------------------------
// Tile partials (two arrays of kScratchTiles) and two sums.  Each GPU the
// library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, recorded once per device by ms_create.
constexpr int kScratchTiles = 1 << 16;
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[2 * kScratchTiles + 32];
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The scratch address on device dev (which must be current).
ms_status scratch_setup(int dev, double **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return MS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return MS_ERR_HIP;
        }
        g_scratch[dev] = (double *)ptr;
    }
    *out = g_scratch[dev];
    return MS_OK;
}

// ---- asynchronous solve ----------------------------------------------------

// counters[0]: blocks at the launch's sweep limit; counters[1]: block sweeps
// started (trace records)
__global__ void k_async_reset(int *version, int *claim, double *board, int nb, int *counters,
                              int already, Ctrl *c, int full) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        if (full) { version[i] = 0; claim[i] = 0; }
        board[i] = INFINITY;   // a block counts as unconverged until it publishes
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counters[0] = already;   // blocks already at the sweep limit of this launch
        c->stop = 0;
        if (full) {
            c->work_items = 0ull; c->inner_iters = 0ull; c->max_stale = 0;
            counters[1] = 0;
        }
    }
}

template <typename T>
ms_status solve_async(ms_handle *h, const double *b, double *x, double tol, int m,
                      const ms_opts &o, ms_stats *stats, hipStream_t st) {
    if (o.staleness < 1)
        return fail(h, MS_ERR_ARG, "asynchronous mode needs staleness >= 1");
    const bool gmres = o.inner_solver == MS_INNER_GMRES;
    if (gmres && (m > h->kry_M || h->kry_rhs < 1 || h->inner_n > h->kry_inner ||
                  h->tiles_cap > h->kry_tiles))
        return fail(h, MS_ERR_ARG,
                    "GMRES inner solves need ms_reserve_krylov(h, >= inner_iters) after the "
                    "last ms_reserve / ms_set_overlap");
    const int vz = std::min(h->vzmax, (int)(16 / sizeof(T)));
    int tx = 0, rows = 0;
    async_tiling(h, vz, 1, 0, h->nblocks, &tx, &rows);
    if (o.x_chunk > 0) tx = std::max(kTxMin, o.x_chunk);
    if (o.rows == 1 || o.rows == 2 || o.rows == 4) rows = std::min(o.rows, async_max_rows(vz));
    if (gmres) {   // GMRES tiles: one row per thread, at most gm_max_planes() planes
        rows = 1;
        tx = std::min(tx, ms::gm_max_planes());
    }
    ms_status s = set_tiling(h, vz, tx, rows, st);
    if (s != MS_OK) return s;
    double nbeff = 0.0, absres = 0.0;
    s = beff_norm<T>(h, b, st, &nbeff);    // also resets the control block
    if (s != MS_OK) return s;
    if (!std::isfinite(nbeff)) return fail(h, MS_ERR_NONFINITE, "b_eff is not finite");
    if (nbeff == 0.0) {
        s = zero_vec(h, x, h->N, st);
        if (s != MS_OK) return s;
        HIPCHK(h, hipStreamSynchronize(st));
        return MS_OK;
    }
    const TeamPlan TP = team_for_solve(h, (int)sizeof(T), o, 1);
    if (!TP.ok && o.engine == MS_ENGINE_TEAM)
        return fail(h, MS_ERR_UNSUPPORTED, "team engine unavailable: " + TP.why);
    if (stats) stats->engine_used = TP.ok ? MS_ENGINE_TEAM : MS_ENGINE_PHASE;
    int per_cu = 0;
    if (gmres)
        HIPCHK(h, ms::async_gmres_occupancy<T>(vz, h->overlap > 0 ? 1 : 0, &per_cu));
    else
        HIPCHK(h, ms::async_occupancy<T>(vz, rows, h->overlap > 0 ? 1 : 0, &per_cu));
    if (per_cu < 1 && !TP.ok) return fail(h, MS_ERR_HIP, "asynchronous kernel cannot be resident");
    int grid = (int)std::min<long long>(h->nblocks, (long long)per_cu * h->num_cu);
    if (o.workers > 0) grid = std::min(grid, o.workers);
    const int nbk = h->nblocks;
    hipLaunchKernelGGL(k_async_reset, dim3((nbk + 255) / 256), dim3(256), 0, st, h->version_d,
                       h->claim_d, h->board_d, nbk, h->finished_d, 0, h->ctrl, 1);
    HIPCHK(h, hipGetLastError());
    const double tol2 = tol > 0.0 ? (tol * nbeff) * (tol * nbeff) : 0.0;
    const long long per_sweep = std::max(1ll, h->N * (long long)m);
    // sweeps per launch: about 2^33 cell-iterations for the phase engine's
    // workers, 2^38 for teams (a team launch ends with its blocks at
    // different sweep counts, and the teams idle through that tail, so it
    // pays to relaunch rarely; the launch still ends as soon as the residual
    // estimate is below tol)
    const long long budget = TP.ok ? (256ll << 30) : (8ll << 30);
    const int chunk = o.check_every > 0
                          ? o.check_every
                          : (int)std::max(8ll, std::min(1000ll, budget / per_sweep));
    AsyncState as;
    as.version = h->version_d;
    as.claim = h->claim_d;
    as.board = h->board_d;
    as.nbr = h->nbr_d;
    as.finished = h->finished_d;
    as.trace = o.trace_cap > 0 ? o.trace : nullptr;
    as.trace_n = h->finished_d + 1;
    as.trace_cap = o.trace_cap;
    as.slow_block = o.slow_sleep > 0 ? o.slow_block : -1;
    as.slow_sleep = o.slow_sleep;
    Bufs<T> B = bufs<T>(h);
    std::vector<int> ver(nbk, 0);
    int maxv = 0, minv = 0, relaunches = 0;
    int hist_n = 0;
    ms_status result = MS_OK;
    s = prof_begin(h, o.profile != 0);
    if (s != MS_OK) return s;
    // the test comes first, as in the synchronous loop
    s = residual_norms(h, b, x, st, &nbeff, &absres);
    if (s != MS_OK) return s;
    double rel = absres / nbeff;
    const double rel0 = rel;
    if (stats && stats->history && hist_n < stats->history_cap) stats->history[hist_n++] = rel;
    bool first = true;
    for (;;) {
        if (!std::isfinite(rel)) { result = fail(h, MS_ERR_NONFINITE, "residual became non-finite"); break; }
        if (tol > 0.0 && rel <= tol) break;
        if (rel0 > 0.0 && rel > 1e6 * rel0) { result = fail(h, MS_ERR_DIVERGED, "residual grew by 1e6"); break; }
        if (minv >= o.max_sweeps) {
            if (tol > 0.0) result = fail(h, MS_ERR_NOT_CONVERGED, "max_sweeps reached above tol");
            break;
        }
        // this launch runs until the estimate drops below tol or every block
        // has reached `limit` sweeps (limit > minv, so some block can move)
        const int limit = (int)std::min<long long>(o.max_sweeps, (long long)maxv + chunk);
        int already = 0;
        for (int v : ver) already += v >= limit;
        if (!first) {
            Ctrl c;
            HIPCHK(h, hipMemcpy(&c, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
            if (c.stop) relaunches++;   // the estimate said converged, the check did not
        }
        hipLaunchKernelGGL(k_async_reset, dim3((nbk + 255) / 256), dim3(256), 0, st, h->version_d,
                           h->claim_d, h->board_d, nbk, h->finished_d, already, h->ctrl, 0);
        HIPCHK(h, hipGetLastError());
        first = false;
        if (TP.ok) {
            s = enqueue_team<T>(h, TP, b, x, x, m, o.inner_tol, true, as, o.staleness, limit, tol2,
                                o.team_spin, st);
            if (s != MS_OK) return s;
        } else {
            Prof p(h, st, MS_K_OTHER);
            if (gmres)
                HIPCHK(h, ms::launch_async_gmres<T>(geom(h), vz, grid, b, x, faces(h), (T *)h->V,
                                                    as, m, o.staleness, limit, tol2, o.inner_tol,
                                                    gm_args(h), h->ctrl, st));
            else
                HIPCHK(h, ms::launch_async<T>(geom(h), vz, grid, b, x, faces(h), B.r, B.p[0],
                                              B.p[1], B.d, as, m, o.staleness, limit, tol2,
                                              o.inner_tol, h->ctrl, st));
        }
        HIPCHK(h, hipMemcpyAsync(ver.data(), h->version_d, sizeof(int) * nbk,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        if (TP.ok) {
            s = team_error(h, st);
            if (s != MS_OK) return s;
        }
        prof_collect(h, stats);
        minv = *std::min_element(ver.begin(), ver.end());
        maxv = *std::max_element(ver.begin(), ver.end());
        // verify on the true FP64 residual (the estimate may be sweeps old)
        s = residual_norms(h, b, x, st, &nbeff, &absres);
        if (s != MS_OK) return s;
        rel = absres / nbeff;
        if (stats && stats->history && hist_n < stats->history_cap) stats->history[hist_n++] = rel;
    }
    Ctrl c;
    HIPCHK(h, hipMemcpy(&c, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    int started = 0;
    HIPCHK(h, hipMemcpy(&started, h->finished_d + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (stats) {
        stats->trace_len = as.trace ? started : 0;
        if (stats->block_sweeps)
            for (int q = 0; q < std::min(nbk, stats->block_sweeps_cap); q++)
                stats->block_sweeps[q] = ver[q];
        stats->sweeps = (int)((c.work_items + nbk / 2) / nbk);
        stats->inner_iters = (int64_t)c.inner_iters;
        stats->rel_residual = rel;
        stats->max_staleness_seen = c.max_stale;
        stats->relaunches = relaunches;
        stats->history_len = hist_n;
    }
    return result;
}

// ---- global CG baseline ------------------------------------------------------

ms_status set_cg_tiling(ms_handle *h, int vz, hipStream_t st) {
    int tx = kTxMin, rows = 1;
    bool found = false;
    const long long slots_base = h->ny;  // rows
    for (int r : {4, 2, 1}) {
        for (int t : {32, 16, 8, 4}) {
            const long long slots = ((slots_base + r - 1) / r) * (h->nz / vz);
            const long long n = ((slots + ms::kThreads - 1) / ms::kThreads) * ((h->nx + t - 1) / t);
            if (n >= kMinTiles) { tx = t; rows = r; found = true; break; }
        }
        if (found) break;
    }
    if (h->cg_vz == vz && h->cg_tx == tx && h->cg_rows == rows) return MS_OK;
    BlockInfo B;
    B.i0 = B.j0 = B.k0 = 0;
    B.bx = (int)h->nx; B.by = (int)h->ny; B.bz = (int)h->nz;
    B.off = 0;
    B.tile0 = 0;
    const long long slots = ((h->ny + rows - 1) / rows) * (h->nz / vz);
    B.nplane = (int)((slots + ms::kThreads - 1) / ms::kThreads);
    B.ntiles = B.nplane * (int)((h->nx + tx - 1) / tx);
    B.oi = B.oj = B.ok = 0;
    B.obx = B.bx; B.oby = B.by; B.obz = B.bz;
    B.dep = 0;
    if (B.ntiles > h->cg_cap) return fail(h, MS_ERR_ARG, "global CG tiling exceeds its table");
    std::vector<int> tb(B.ntiles, 0);
    HIPCHK(h, hipMemcpyAsync(h->cg_block_d, &B, sizeof(B), hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(h->cg_tiles_d, tb.data(), sizeof(int) * tb.size(),
                             hipMemcpyHostToDevice, st));
    HIPCHK(h, hipStreamSynchronize(st));
    h->cg_vz = vz; h->cg_tx = tx; h->cg_rows = rows; h->cg_ntiles = B.ntiles;
    return MS_OK;
}

ms_status solve_cg(ms_handle *h, const double *b, double *x, double tol, int max_iters,
                   const ms_opts &o, ms_stats *stats, hipStream_t st) {
    if (h->nx > (1 << 30) || h->ny > (1 << 30) || h->nz > (1 << 30))
        return fail(h, MS_ERR_ARG, "grid too large for the single-block tiling");
    const int vz = h->nz % 2 == 0 ? 2 : 1;
    ms_status s = set_cg_tiling(h, vz, st);
    if (s != MS_OK) return s;
    // block tiling for the b_eff norm (any valid tiling will do)
    if (h->cur_vz == 0) {
        s = set_tiling(h, std::min(h->vzmax, 2), 16, 1, st);
        if (s != MS_OK) return s;
    }
    double nbeff = 0.0;
    s = beff_norm<double>(h, b, st, &nbeff);
    if (s != MS_OK) return s;
    if (!std::isfinite(nbeff)) return fail(h, MS_ERR_NONFINITE, "b_eff is not finite");
    if (nbeff == 0.0) {
        s = zero_vec(h, x, h->N, st);
        if (s != MS_OK) return s;
        HIPCHK(h, hipStreamSynchronize(st));
        return MS_OK;
    }
    Geom g1;
    g1.nx = h->nx; g1.ny = h->ny; g1.nz = h->nz;
    g1.blocks = h->cg_block_d;
    g1.tile_block = h->cg_tiles_d;
    g1.tx = h->cg_tx;
    g1.rows = h->cg_rows;
    g1.nblocks = 1;
    g1.ovl = 0;
    const int nt = h->cg_ntiles;
    double *r = (double *)h->r, *P[2] = {(double *)h->p0, (double *)h->p1};
    double *psig = (double *)h->psig, *prho = (double *)h->prhoA, *scal = h->scal_d;
    s = prof_begin(h, o.profile != 0);
    if (s != MS_OK) return s;
    {
        Prof p(h, st, MS_K_RESID);
        HIPCHK(h, ms::launch_resid<double>(g1, vz, 0, nt, 0, b, x, faces(h), r, h->part64,
                                           h->part64, h->ctrl, ms::single_rhs(), st));
    }
    HIPCHK(h, ms::launch_gcg_reduce(h->part64, nt, 0, tol, max_iters, h->history_d, kHistoryCap,
                                    scal, h->ctrl, st));
    const int batch = o.check_every > 0 ? o.check_every : 64;
    Ctrl c;
    int j = 0;
    for (;;) {
        const int nb = std::min(batch, max_iters - j);
        for (int q = 0; q < nb; q++, j++) {
            {
                Prof p(h, st, MS_K_STENCIL);
                HIPCHK(h, ms::launch_gcg_stencil(g1, vz, nt, r, P[(j + 1) % 2], P[j % 2], psig,
                                                 scal, j, h->ctrl, st));
            }
            HIPCHK(h, ms::launch_gcg_reduce(psig, nt, 1, tol, max_iters, h->history_d, kHistoryCap,
                                            scal, h->ctrl, st));
            {
                Prof p(h, st, MS_K_UPDATE);
                HIPCHK(h, ms::launch_gcg_update(g1, vz, nt, r, P[j % 2], x, prho, scal, h->ctrl, st));
            }
            HIPCHK(h, ms::launch_gcg_reduce(prho, nt, 2, tol, max_iters, h->history_d, kHistoryCap,
                                            scal, h->ctrl, st));
        }
        HIPCHK(h, hipMemcpyAsync(&c, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        prof_collect(h, stats);
        if (c.done) break;
        if (j >= max_iters) return fail(h, MS_ERR_HIP, "device did not finish the CG solve");
    }
    double absres = 0.0;
    s = residual_norms(h, b, x, st, &nbeff, &absres);
    if (s != MS_OK) return s;
    if (stats) {
        stats->sweeps = c.final_sweep;
        stats->inner_iters = c.final_sweep;
        stats->rel_residual = absres / nbeff;
        if (stats->history && stats->history_cap > 0) {
            const int n = std::min(std::min(stats->history_cap, kHistoryCap), c.final_sweep + 1);
            HIPCHK(h, hipMemcpy(stats->history, h->history_d, sizeof(double) * n,
                                hipMemcpyDeviceToHost));
            stats->history_len = n;
        }
    }
    switch (c.status) {
        case 0: return MS_OK;
        case 4: return fail(h, MS_ERR_NOT_CONVERGED, "max_iters reached above tol");
        case 5: return fail(h, MS_ERR_NONFINITE, "residual became non-finite");
        default: return fail(h, MS_ERR_HIP, "unknown device status");
    }
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================

extern "C" {

void ms_default_opts(ms_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->max_sweeps = 100000;
    o->inner_tol = 0.0;
    o->staleness = 2;
    o->precision = MS_FP64;
    o->stream = nullptr;
    o->check_every = 0;
    o->group_blocks = 0;
    o->x_chunk = 0;
    o->profile = 0;
    o->use_graph = 1;
    o->rows = 0;
    o->workers = 0;
    o->inner_solver = MS_INNER_CG;
    o->z_vector = 0;
    o->slow_block = -1;
    o->slow_sleep = 0;
    o->trace = nullptr;
    o->trace_cap = 0;
    o->engine = MS_ENGINE_AUTO;
}

const char *ms_status_string(ms_status s) {
    switch (s) {
        case MS_OK: return "MS_OK";
        case MS_ERR_ARG: return "MS_ERR_ARG";
        case MS_ERR_HIP: return "MS_ERR_HIP";
        case MS_ERR_NOMEM: return "MS_ERR_NOMEM";
        case MS_ERR_NOT_CONVERGED: return "MS_ERR_NOT_CONVERGED";
        case MS_ERR_NONFINITE: return "MS_ERR_NONFINITE";
        case MS_ERR_DIVERGED: return "MS_ERR_DIVERGED";
        case MS_ERR_UNSUPPORTED: return "MS_ERR_UNSUPPORTED";
    }
    return "MS_ERR_UNKNOWN";
}

const char *ms_last_error(const ms_handle *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

const char *ms_version(void) { return "libms 0.1.0 (gfx950)"; }

ms_status ms_create(const ms_grid *grid, const ms_blocks *blocks, const ms_bc *bc,
                    ms_handle **out) {
    if (!out) return fail(nullptr, MS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !blocks) return fail(nullptr, MS_ERR_ARG, "grid or blocks is NULL");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1)
        return fail(nullptr, MS_ERR_ARG, "grid sizes must be >= 1");
    if (grid->nx > (1 << 20) || grid->ny > (1 << 20) || grid->nz > (1 << 20) ||
        (double)grid->nx * grid->ny * grid->nz > 4.0e10)
        return fail(nullptr, MS_ERR_ARG, "grid too large");
    if (blocks->gx < 1 || blocks->gy < 1 || blocks->gz < 1)
        return fail(nullptr, MS_ERR_ARG, "block counts must be >= 1");
    ms_handle tmp;
    tmp.nx = grid->nx; tmp.ny = grid->ny; tmp.nz = grid->nz;
    tmp.N = tmp.nx * tmp.ny * tmp.nz;
    tmp.gx = blocks->gx; tmp.gy = blocks->gy; tmp.gz = blocks->gz;
    const int32_t *cuts[3] = {blocks->cuts_x, blocks->cuts_y, blocks->cuts_z};
    const long long ns[3] = {tmp.nx, tmp.ny, tmp.nz};
    const int gs[3] = {tmp.gx, tmp.gy, tmp.gz};
    std::vector<int> *dst[3] = {&tmp.cx, &tmp.cy, &tmp.cz};
    for (int a = 0; a < 3; a++) {
        if (gs[a] > ns[a]) return fail(nullptr, MS_ERR_ARG, "more blocks than points on an axis");
        dst[a]->resize(gs[a] + 1);
        if (cuts[a]) {
            for (int t = 0; t <= gs[a]; t++) (*dst[a])[t] = cuts[a][t];
        } else {
            if (ns[a] % gs[a]) return fail(nullptr, MS_ERR_ARG, "uniform split needs n % g == 0");
            for (int t = 0; t <= gs[a]; t++) (*dst[a])[t] = (int)(ns[a] / gs[a] * t);
        }
        if (!valid_cuts(*dst[a], ns[a]))
            return fail(nullptr, MS_ERR_ARG, "cuts must increase strictly from 0 to n");
    }
    if ((long long)tmp.gx * tmp.gy * tmp.gz > (1 << 22))
        return fail(nullptr, MS_ERR_ARG, "too many blocks");
    tmp.nblocks = tmp.gx * tmp.gy * tmp.gz;
    // vector width: every z cut and nz divisible
    tmp.vzmax = 1;
    for (int w : {8, 4, 2}) {
        bool ok = tmp.nz % w == 0;
        for (int c : tmp.cz) ok = ok && (c % w == 0);
        if (ok) { tmp.vzmax = w; break; }
    }
    tmp.vzbase = std::min(tmp.vzmax, 4);
    tmp.inner_n = tmp.inner_cap = tmp.N;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, MS_ERR_HIP, std::string("no HIP device: ") + hipGetErrorString(e));
    ms_handle *h = new ms_handle(std::move(tmp));
    // tile table capacity: narrowest vector, smallest x chunk
    const long long cap = tile_capacity(h);
    // the global-CG tiling (one block = the grid) needs at most as many tiles
    const long long cg_cap = ((h->ny * h->nz + ms::kThreads - 1) / ms::kThreads) *
                             ((h->nx + kTxMin - 1) / kTxMin);
    if (cap > (1ll << 30) || cg_cap > (1ll << 30)) {
        delete h;
        return fail(nullptr, MS_ERR_ARG, "too many tiles");
    }
    h->cg_cap = (int)cg_cap;
    h->tiles_cap = (int)std::max(cap, cg_cap);
    const size_t vb = sizeof(double) * (size_t)h->N;
    const size_t tb = sizeof(double) * (size_t)h->tiles_cap;
    struct A { void **p; size_t n; } allocs[] = {
        {(void **)&h->blocks_d, sizeof(BlockInfo) * (size_t)h->nblocks},
        {(void **)&h->tile_block_d, sizeof(int) * (size_t)h->tiles_cap},
        {(void **)&h->x1, vb}, {&h->r, vb}, {&h->d, vb}, {&h->p0, vb}, {&h->p1, vb},
        {(void **)&h->part64, tb}, {&h->partT, tb}, {&h->psig, tb}, {&h->prhoA, tb},
        {&h->prhoB, tb},
        {(void **)&h->active, sizeof(int) * (size_t)h->nblocks},
        {(void **)&h->ctrl, sizeof(Ctrl)},
        {(void **)&h->history_d, sizeof(double) * (size_t)kHistoryCap},
        {(void **)&h->scal_d, 64},
        {(void **)&h->cg_block_d, sizeof(BlockInfo)},
        {(void **)&h->cg_tiles_d, sizeof(int) * (size_t)h->cg_cap},
        {(void **)&h->version_d, sizeof(int) * (size_t)h->nblocks},
        {(void **)&h->claim_d, sizeof(int) * (size_t)h->nblocks},
        {(void **)&h->nbr_d, sizeof(int) * 6 * (size_t)h->nblocks},
        {(void **)&h->finished_d, 64},
        {(void **)&h->board_d, sizeof(double) * (size_t)h->nblocks},
        {(void **)&h->team_ctr, 64},
    };
    for (auto &a : allocs) {
        e = hipMalloc(a.p, a.n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_all(h);
            delete h;
            return fail(nullptr, e == hipErrorOutOfMemory ? MS_ERR_NOMEM : MS_ERR_HIP,
                        std::string("device allocation failed: ") + hipGetErrorString(e));
        }
    }
    ms_status s = copy_bc(h, bc);
    if (s == MS_OK) s = set_tiling(h, h->vzmax >= 2 ? 2 : 1, 16, 1, nullptr);
    if (s == MS_OK) {
        // neighbour table of the block grid, faces -x,+x,-y,+y,-z,+z
        std::vector<int> nbr(6 * (size_t)h->nblocks, -1);
        for (int bi = 0; bi < h->gx; bi++)
            for (int bj = 0; bj < h->gy; bj++)
                for (int bk = 0; bk < h->gz; bk++) {
                    const int b = (bi * h->gy + bj) * h->gz + bk;
                    if (bi > 0) nbr[6 * b + 0] = b - h->gy * h->gz;
                    if (bi < h->gx - 1) nbr[6 * b + 1] = b + h->gy * h->gz;
                    if (bj > 0) nbr[6 * b + 2] = b - h->gz;
                    if (bj < h->gy - 1) nbr[6 * b + 3] = b + h->gz;
                    if (bk > 0) nbr[6 * b + 4] = b - 1;
                    if (bk < h->gz - 1) nbr[6 * b + 5] = b + 1;
                }
        e = hipMemcpy(h->nbr_d, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) s = hip_fail(h, e, "ms_create setup");
    }
    if (s == MS_OK) {
        s = scratch_setup(dev, &h->scratch_d);
        if (s != MS_OK) s = fail(h, s, "hipGetSymbolAddress of the static scratch failed");
    }
    if (s == MS_OK) {
        e = hipMemset(h->team_ctr, 0, 64);
        if (e != hipSuccess) s = hip_fail(h, e, "ms_create setup");
    }
    if (s == MS_OK) s = team_alloc(h);
    if (s != MS_OK) {
        g_create_error = h->err;
        free_all(h);
        delete h;
        return s;
    }
    *out = h;
    return MS_OK;
}

ms_status ms_set_bc(ms_handle *h, const ms_bc *bc) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    return copy_bc(h, bc);
}

void ms_destroy(ms_handle *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
}

static ms_status check_vec(ms_handle *h, const void *p, const char *name, long long n = 0) {
    if (n <= 0) n = h->N;
    if (!p) return fail(h, MS_ERR_ARG, std::string(name) + " is NULL");
    if ((uintptr_t)p % 16) return fail(h, MS_ERR_ARG, std::string(name) + " must be 16-byte aligned");
    if (!dev_range_ok(p, sizeof(double) * (size_t)n))
        return fail(h, MS_ERR_ARG, std::string(name) + " is not a device buffer of the right size");
    return MS_OK;
}

// Argument checks shared by ms_solve and ms_solve_batch.
static ms_status check_solve(ms_handle *h, const double *b, double *x, long long n,
                             int32_t inner_iters, const ms_opts &o, double tol) {
    ms_status s = check_vec(h, b, "b", n);
    if (s != MS_OK) return s;
    s = check_vec(h, x, "x", n);
    if (s != MS_OK) return s;
    const char *bb = (const char *)b, *xx = (const char *)x;
    const size_t bytes = sizeof(double) * (size_t)n;
    if (bb < xx + bytes && xx < bb + bytes) return fail(h, MS_ERR_ARG, "b and x overlap");
    if (inner_iters < 1) return fail(h, MS_ERR_ARG, "inner_iters must be >= 1");
    if (o.max_sweeps < 0) return fail(h, MS_ERR_ARG, "max_sweeps must be >= 0");
    if (o.staleness < 0) return fail(h, MS_ERR_ARG, "staleness must be >= 0");
    if (std::isnan(tol) || !(o.inner_tol >= 0.0) || !std::isfinite(o.inner_tol))
        return fail(h, MS_ERR_ARG, "tol or inner_tol invalid");
    if (o.precision != MS_FP64 && o.precision != MS_MIXED)
        return fail(h, MS_ERR_ARG, "unknown precision");
    if (o.inner_solver != MS_INNER_CG && o.inner_solver != MS_INNER_GMRES)
        return fail(h, MS_ERR_ARG, "unknown inner solver");
    if (o.z_vector < 0) return fail(h, MS_ERR_ARG, "z_vector must be >= 0");
    if (o.team_spin < 0) return fail(h, MS_ERR_ARG, "team_spin must be >= 0");
    if (o.slow_sleep < 0 || o.slow_sleep > 100000)
        return fail(h, MS_ERR_ARG, "slow_sleep must be in [0, 100000]");
    if (o.slow_sleep > 0 && o.slow_block >= h->nblocks)
        return fail(h, MS_ERR_ARG, "slow_block is not a block of the partition");
    if (o.trace_cap < 0) return fail(h, MS_ERR_ARG, "trace_cap must be >= 0");
    if (o.engine != MS_ENGINE_AUTO && o.engine != MS_ENGINE_PHASE && o.engine != MS_ENGINE_TEAM)
        return fail(h, MS_ERR_ARG, "unknown engine");
    if (o.trace_cap > 0 && (!o.trace || !dev_range_ok(o.trace, sizeof(int32_t) * 8 * (size_t)o.trace_cap)))
        return fail(h, MS_ERR_ARG, "trace is not a device buffer of trace_cap records");
    return MS_OK;
}

static void reset_stats(ms_stats *stats, int n) {
    for (int k = 0; stats && k < n; k++) {
        double *hist = stats[k].history;
        const int cap = stats[k].history_cap;
        int32_t *bsw = stats[k].block_sweeps;
        const int bcap = stats[k].block_sweeps_cap;
        memset(&stats[k], 0, sizeof(ms_stats));
        stats[k].history = hist;
        stats[k].history_cap = cap;
        stats[k].block_sweeps = bsw;
        stats[k].block_sweeps_cap = bcap;
    }
}

ms_status ms_solve(ms_handle *h, const double *b, double *x, double tol, int32_t inner_iters,
                   ms_mode mode, const ms_opts *opts, ms_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    ms_opts o;
    ms_default_opts(&o);
    if (opts) o = *opts;
    ms_status s = check_solve(h, b, x, h->N, inner_iters, o, tol);
    if (s != MS_OK) return s;
    if (mode != MS_SYNC && mode != MS_ASYNC) return fail(h, MS_ERR_ARG, "unknown mode");
    reset_stats(stats, 1);
    hipStream_t st = (hipStream_t)o.stream;
    if (mode == MS_ASYNC)
        s = o.precision == MS_FP64 ? solve_async<double>(h, b, x, tol, inner_iters, o, stats, st)
                                   : solve_async<float>(h, b, x, tol, inner_iters, o, stats, st);
    else
        s = o.precision == MS_FP64 ? solve_sync<double>(h, b, x, 1, tol, inner_iters, o, stats, st)
                                   : solve_sync<float>(h, b, x, 1, tol, inner_iters, o, stats, st);
    if (stats)
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return s;
}

ms_status ms_reserve(ms_handle *h, int32_t nrhs) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    if (nrhs < 1 || nrhs > 4096) return fail(h, MS_ERR_ARG, "nrhs must be in [1, 4096]");
    if (nrhs <= h->rhs_cap) return MS_OK;
    const size_t vb = sizeof(double) * (size_t)h->N * nrhs;
    const size_t ib = sizeof(double) * (size_t)h->inner_cap * nrhs;
    const size_t tb = sizeof(double) * (size_t)h->tiles_cap * nrhs;
    void **slots[] = {(void **)&h->x1, &h->r, &h->d, &h->p0, &h->p1, (void **)&h->part64,
                      &h->partT, &h->psig, &h->prhoA, &h->prhoB, (void **)&h->active,
                      (void **)&h->ctrl, (void **)&h->history_d};
    const size_t sizes[] = {vb, ib, ib, ib, ib, tb, tb, tb, tb, tb,
                            sizeof(int) * (size_t)h->nblocks * nrhs, sizeof(Ctrl) * (size_t)nrhs,
                            sizeof(double) * (size_t)kHistoryCap * nrhs};
    constexpr int n = sizeof(sizes) / sizeof(sizes[0]);
    void *fresh[n] = {};
    for (int i = 0; i < n; i++) {
        const hipError_t e = hipMalloc(&fresh[i], sizes[i]);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; j++) (void)hipFree(fresh[j]);
            return fail(h, e == hipErrorOutOfMemory ? MS_ERR_NOMEM : MS_ERR_HIP,
                        std::string("ms_reserve: ") + hipGetErrorString(e));
        }
    }
    drop_graph(h);
    for (int i = 0; i < n; i++) {
        (void)hipFree(*slots[i]);
        *slots[i] = fresh[i];
    }
    h->rhs_cap = nrhs;
    return MS_OK;
}

ms_status ms_set_overlap(ms_handle *h, int32_t overlap) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    if (overlap < 0) return fail(h, MS_ERR_ARG, "overlap must be >= 0");
    if (overlap > std::max(h->nx, std::max(h->ny, h->nz)))
        return fail(h, MS_ERR_ARG, "overlap exceeds the grid");
    if (overlap == h->overlap) return MS_OK;
    // sizes under the new overlap
    const int old = h->overlap;
    h->overlap = overlap;
    long long inner = 0;
    for (int b = 0; b < h->nblocks; b++) inner += block_cells(h, b);
    const long long cap = std::max(tile_capacity(h), (long long)h->cg_cap);
    h->overlap = old;
    if (cap > (1ll << 30)) return fail(h, MS_ERR_ARG, "too many tiles");
    // grow the inner vectors and the per-tile arrays when they are too small
    const size_t R = (size_t)h->rhs_cap;
    const bool gi = inner > h->inner_cap, gt = cap > h->tiles_cap;
    void **slots[] = {&h->r, &h->d, &h->p0, &h->p1, (void **)&h->tile_block_d,
                      (void **)&h->part64, &h->partT, &h->psig, &h->prhoA, &h->prhoB};
    const size_t ib = sizeof(double) * (size_t)inner * R, tb = sizeof(double) * (size_t)cap * R;
    const size_t sizes[] = {ib, ib, ib, ib, sizeof(int) * (size_t)cap, tb, tb, tb, tb, tb};
    const bool grow[] = {gi, gi, gi, gi, gt, gt, gt, gt, gt, gt};
    constexpr int n = sizeof(sizes) / sizeof(sizes[0]);
    void *fresh[n] = {};
    for (int i = 0; i < n; i++) {
        if (!grow[i]) continue;
        const hipError_t e = hipMalloc(&fresh[i], sizes[i]);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; j++)
                if (fresh[j]) (void)hipFree(fresh[j]);
            return fail(h, e == hipErrorOutOfMemory ? MS_ERR_NOMEM : MS_ERR_HIP,
                        std::string("ms_set_overlap: ") + hipGetErrorString(e));
        }
    }
    drop_graph(h);
    for (int i = 0; i < n; i++) {
        if (!grow[i]) continue;
        (void)hipFree(*slots[i]);
        *slots[i] = fresh[i];
    }
    if (gi) h->inner_cap = inner;
    if (gt) h->tiles_cap = (int)cap;
    h->overlap = overlap;
    h->inner_n = inner;
    h->cur_vz = 0;
    ms_status st = set_tiling(h, std::min(h->vzmax, 2), 16, 1, nullptr);
    if (st == MS_OK) st = team_alloc(h);
    return st;
}

ms_status ms_reserve_krylov(ms_handle *h, int32_t max_inner) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    if (max_inner < 1 || max_inner > 128) return fail(h, MS_ERR_ARG, "max_inner must be in [1, 128]");
    const int M = std::max((int)max_inner, h->kry_M);
    if (M == h->kry_M && h->kry_inner >= h->inner_cap && h->kry_rhs >= h->rhs_cap &&
        h->kry_tiles >= h->tiles_cap)
        return MS_OK;
    const size_t R = (size_t)h->rhs_cap;
    const size_t sizes[3] = {
        sizeof(double) * (size_t)(M + 1) * (size_t)h->inner_cap * R,
        sizeof(double) * (size_t)h->tiles_cap * R * (size_t)(M + 2),
        sizeof(double) * (size_t)h->nblocks * R * (size_t)ms::gm_record_doubles(M)};
    void *fresh[3] = {};
    for (int i = 0; i < 3; i++) {
        const hipError_t e = hipMalloc(&fresh[i], sizes[i]);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; j++) (void)hipFree(fresh[j]);
            return fail(h, e == hipErrorOutOfMemory ? MS_ERR_NOMEM : MS_ERR_HIP,
                        std::string("ms_reserve_krylov: ") + hipGetErrorString(e));
        }
    }
    drop_graph(h);
    if (h->V) (void)hipFree(h->V);
    if (h->gpart) (void)hipFree(h->gpart);
    if (h->gm) (void)hipFree(h->gm);
    h->V = fresh[0];
    h->gpart = (double *)fresh[1];
    h->gm = (double *)fresh[2];
    h->kry_M = M;
    h->kry_inner = h->inner_cap;
    h->kry_rhs = h->rhs_cap;
    h->kry_tiles = h->tiles_cap;
    return MS_OK;
}

ms_status ms_solve_batch(ms_handle *h, int32_t nrhs, const double *b, double *x, double tol,
                         int32_t inner_iters, ms_mode mode, const ms_opts *opts,
                         ms_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    if (nrhs < 1) return fail(h, MS_ERR_ARG, "nrhs must be >= 1");
    if (nrhs > h->rhs_cap) return fail(h, MS_ERR_ARG, "nrhs exceeds the capacity set by ms_reserve");
    if (mode != MS_SYNC) return fail(h, MS_ERR_UNSUPPORTED, "batched solves are synchronous only");
    ms_opts o;
    ms_default_opts(&o);
    if (opts) o = *opts;
    ms_status s = check_solve(h, b, x, h->N * nrhs, inner_iters, o, tol);
    if (s != MS_OK) return s;
    reset_stats(stats, nrhs);
    hipStream_t st = (hipStream_t)o.stream;
    s = o.precision == MS_FP64 ? solve_sync<double>(h, b, x, nrhs, tol, inner_iters, o, stats, st)
                               : solve_sync<float>(h, b, x, nrhs, tol, inner_iters, o, stats, st);
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int k = 0; stats && k < nrhs; k++) stats[k].seconds = sec;
    return s;
}

ms_status ms_residual(ms_handle *h, const double *b, const double *x, double *rel_out,
                      double *abs_out, void *stream) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    if (!rel_out) return fail(h, MS_ERR_ARG, "rel_out is NULL");
    ms_status s = check_vec(h, b, "b");
    if (s != MS_OK) return s;
    s = check_vec(h, x, "x");
    if (s != MS_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    double nbeff = 0.0, a = 0.0;
    s = residual_norms(h, b, x, st, &nbeff, &a);
    if (s != MS_OK) return s;
    if (abs_out) *abs_out = a;
    *rel_out = nbeff > 0.0 ? a / nbeff : 0.0;
    return MS_OK;
}

ms_status ms_residual_noalloc(ms_handle *h, const double *b, const double *x, double *rel_out,
                              double *abs_out, void *stream) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    if (!rel_out) return fail(h, MS_ERR_ARG, "rel_out is NULL");
    ms_status s = check_vec(h, b, "b");
    if (s != MS_OK) return s;
    s = check_vec(h, x, "x");
    if (s != MS_OK) return s;
    if (h->ntiles > kScratchTiles)
        return fail(h, MS_ERR_ARG, "the handle's tiling has " + std::to_string(h->ntiles) +
                                       " tiles; the static scratch holds " +
                                       std::to_string(kScratchTiles));
    if (!h->scratch_d) return fail(h, MS_ERR_HIP, "static scratch not set up");
    int dev = -1;
    HIPCHK(h, hipGetDevice(&dev));
    bool same = false;
    if (dev >= 0 && dev < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        same = g_scratch[dev] == h->scratch_d;
    }
    if (!same) return fail(h, MS_ERR_ARG, "the current device is not the handle's device");
    double *p64 = h->scratch_d, *pT = p64 + kScratchTiles, *sums = p64 + 2 * kScratchTiles;
    double nbeff = 0.0, a = 0.0;
    s = residual_norms_in(h, b, x, (hipStream_t)stream, p64, pT, sums, &nbeff, &a);
    if (s != MS_OK) return s;
    if (abs_out) *abs_out = a;
    *rel_out = nbeff > 0.0 ? a / nbeff : 0.0;
    return MS_OK;
}

ms_status ms_lift(ms_handle *h, const double *f, double s, double *b_eff, void *stream) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    ms_status st = check_vec(h, f, "f");
    if (st != MS_OK) return st;
    st = check_vec(h, b_eff, "b_eff");
    if (st != MS_OK) return st;
    if (!std::isfinite(s)) return fail(h, MS_ERR_ARG, "scale is not finite");
    const char *ff = (const char *)f, *bb = (const char *)b_eff;
    const size_t bytes = sizeof(double) * (size_t)h->N;
    if (ff != bb && ff < bb + bytes && bb < ff + bytes)
        return fail(h, MS_ERR_ARG, "f and b_eff overlap without being the same buffer");
    HIPCHK(h, ms::launch_lift(h->nx, h->ny, h->nz, f, s, faces(h), b_eff, (hipStream_t)stream));
    return MS_OK;
}

ms_status ms_lift_adjoint(ms_handle *h, const double *lambda, double s, double *grad_f,
                          double *const grad_face[6], void *stream) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    ms_status st = check_vec(h, lambda, "lambda");
    if (st != MS_OK) return st;
    if (grad_f) {
        st = check_vec(h, grad_f, "grad_f");
        if (st != MS_OK) return st;
        const char *ll = (const char *)lambda, *gg = (const char *)grad_f;
        const size_t bytes = sizeof(double) * (size_t)h->N;
        if (ll != gg && ll < gg + bytes && gg < ll + bytes)
            return fail(h, MS_ERR_ARG, "lambda and grad_f overlap without being the same buffer");
    }
    if (!std::isfinite(s)) return fail(h, MS_ERR_ARG, "scale is not finite");
    const long long sz[6] = {h->ny * h->nz, h->ny * h->nz, h->nx * h->nz,
                             h->nx * h->nz, h->nx * h->ny, h->nx * h->ny};
    double *gfaces[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int t = 0; grad_face && t < 6; t++) {
        gfaces[t] = grad_face[t];
        if (gfaces[t] && !dev_range_ok(gfaces[t], sizeof(double) * (size_t)sz[t]))
            return fail(h, MS_ERR_ARG, "grad_face " + std::to_string(t) +
                                           " is not a device buffer of the face's size");
    }
    HIPCHK(h, ms::launch_lift_adjoint(h->nx, h->ny, h->nz, lambda, s, grad_f, gfaces,
                                      (hipStream_t)stream));
    return MS_OK;
}

ms_status ms_apply(ms_handle *h, const double *u, double *y, void *stream) {
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    ms_status s = check_vec(h, u, "u");
    if (s != MS_OK) return s;
    s = check_vec(h, y, "y");
    if (s != MS_OK) return s;
    const char *uu = (const char *)u, *yy = (const char *)y;
    const size_t bytes = sizeof(double) * (size_t)h->N;
    if (uu < yy + bytes && yy < uu + bytes) return fail(h, MS_ERR_ARG, "u and y overlap");
    HIPCHK(h, ms::launch_apply(h->nx, h->ny, h->nz, u, y, (hipStream_t)stream));
    return MS_OK;
}

ms_status ms_cg(ms_handle *h, const double *b, double *x, double tol, int32_t max_iters,
                const ms_opts *opts, ms_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!h) return fail(nullptr, MS_ERR_ARG, "handle is NULL");
    ms_opts o;
    ms_default_opts(&o);
    if (opts) o = *opts;
    ms_status s = check_vec(h, b, "b");
    if (s != MS_OK) return s;
    s = check_vec(h, x, "x");
    if (s != MS_OK) return s;
    const char *bb = (const char *)b, *xx = (const char *)x;
    const size_t bytes = sizeof(double) * (size_t)h->N;
    if (bb < xx + bytes && xx < bb + bytes) return fail(h, MS_ERR_ARG, "b and x overlap");
    if (max_iters < 0) return fail(h, MS_ERR_ARG, "max_iters must be >= 0");
    if (std::isnan(tol)) return fail(h, MS_ERR_ARG, "tol is NaN");
    reset_stats(stats, 1);
    s = solve_cg(h, b, x, tol, max_iters, o, stats, (hipStream_t)o.stream);
    if (stats)
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return s;
}

}  // extern "C"
