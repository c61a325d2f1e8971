/*
 * Plain FP64 CPU oracle for two-stage multisplitting (block Jacobi outer
 * sweep, conjugate-gradient inner solves) on the 3D 7-point Laplace/Poisson
 * system, after Brown, Bull and Bethune, "A highly scalable approach to
 * solving linear systems using two-stage multisplitting".
 *
 * THIS IS TEST INFRASTRUCTURE.  It exists only to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with
 * the GPU library, and it is written to be read against the paper, not to
 * be fast: every loop is the plain definition.  OpenMP is used only where
 * each output element is computed independently, and every sum is taken in
 * a fixed serial order, so results do not depend on the thread count.
 *
 * Conventions (the same ones the GPU library documents, restated here):
 *   - interior grid nx*ny*nz, C order, index (i*ny + j)*nz + k, z fastest;
 *   - (A u)(i,j,k) = 6 u(i,j,k) - sum of the 6 axis neighbours, the
 *     7-point Laplacian of Section 2.1 (diagonal 6, off-diagonal -1);
 *   - neighbours outside the interior are Dirichlet nodes; their values g
 *     are moved to the right-hand side (b_eff = b + sum of boundary g);
 *   - six boundary faces in the order -x,+x,-y,+y,-z,+z; the x faces are
 *     [ny][nz], the y faces [nx][nz], the z faces [nx][ny]; NULL means 0;
 *   - blocks are a tensor product of per-axis cut lists
 *     cx[0]=0 < cx[1] < ... < cx[gx]=nx (likewise y, z); block (bi,bj,bk)
 *     has linear number (bi*gy + bj)*gz + bk.
 *
 * Readings of the paper where it is silent (each is also listed in the
 * design notes):
 *   - inner solver: unpreconditioned CG (every diagonal block is SPD);
 *   - inner start: residual-correction form, d = 0 on r_i, which equals CG
 *     on A_ii X_i = B_i - sum_j A_ij X_j started from the current X_i;
 *   - inner stop: at most m iterations, or earlier when
 *     ||r_i|| <= inner_tol * ||r_i at entry|| (inner_tol > 0 only), or on
 *     breakdown (p.Ap not > 0);
 *   - residual: the true residual ||b_eff - A x|| / ||b_eff||, tested with
 *     "<=" at the top of every sweep;
 *   - tol <= 0 means: run exactly max_sweeps sweeps.
 *
 * ORACLE_MUTANT (compile-time, test use only) plants one known mistake so
 * that the test suite can show each pin catches something.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* status codes returned by the solvers */
#define OR_OK 0
#define OR_NOT_CONVERGED 4
#define OR_NONFINITE 5
#define OR_DIVERGED 6
#define OR_ARG 1

#define IDX(i, j, k) (((long)(i) * ny + (j)) * nz + (k))

/* threads an OpenMP region of the oracle uses (1 without OpenMP) */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Operator and right-hand side (Section 2.1: 7-point Laplace stencil) */
/* ------------------------------------------------------------------ */

/* y = A u with u = 0 outside the interior. */
void or_apply(long nx, long ny, long nz, const double *u, double *y)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nx; i++)
        for (long j = 0; j < ny; j++)
            for (long k = 0; k < nz; k++) {
                double s = 6.0 * u[IDX(i, j, k)];
                if (i > 0) s -= u[IDX(i - 1, j, k)];
                if (i < nx - 1) s -= u[IDX(i + 1, j, k)];
                if (j > 0) s -= u[IDX(i, j - 1, k)];
                if (j < ny - 1) s -= u[IDX(i, j + 1, k)];
                if (k > 0) s -= u[IDX(i, j, k - 1)];
#if ORACLE_MUTANT != 1
                if (k < nz - 1) s -= u[IDX(i, j, k + 1)];
#endif
                y[IDX(i, j, k)] = s;
            }
}

/* b_eff = b + g at every boundary neighbour (Dirichlet lifting). */
void or_lift_bc(long nx, long ny, long nz, const double *b,
                const double *fxm, const double *fxp, const double *fym,
                const double *fyp, const double *fzm, const double *fzp,
                double *beff)
{
#if ORACLE_MUTANT == 8
    /* planted mistake: -x and -y faces exchanged (only meaningful on cubes) */
    const double *t = fxm; fxm = fym; fym = t;
#endif
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nx; i++)
        for (long j = 0; j < ny; j++)
            for (long k = 0; k < nz; k++) {
                double s = b ? b[IDX(i, j, k)] : 0.0;
                if (i == 0 && fxm) s += fxm[j * nz + k];
                if (i == nx - 1 && fxp) s += fxp[j * nz + k];
                if (j == 0 && fym) s += fym[i * nz + k];
                if (j == ny - 1 && fyp) s += fyp[i * nz + k];
                if (k == 0 && fzm) s += fzm[i * ny + j];
#if ORACLE_MUTANT == 2
                if (k == nz - 1 && fzp) s -= fzp[i * ny + j];
#else
                if (k == nz - 1 && fzp) s += fzp[i * ny + j];
#endif
                beff[IDX(i, j, k)] = s;
            }
}

/* r = b_eff - A x; returns ||r||_2 summed in index order. r may be NULL. */
double or_residual(long nx, long ny, long nz, const double *beff,
                   const double *x, double *r)
{
    long n = nx * ny * nz;
    double *rr = r ? r : (double *)malloc(sizeof(double) * (size_t)n);
    or_apply(nx, ny, nz, x, rr);
#pragma omp parallel for schedule(static)
    for (long t = 0; t < n; t++) rr[t] = beff[t] - rr[t];
    double s = 0.0;
    for (long t = 0; t < n; t++) s += rr[t] * rr[t];
    if (!r) free(rr);
    return sqrt(s);
}

double or_norm2(long n, const double *v)
{
    double s = 0.0;
#if ORACLE_MUTANT == 18
    n += 1;   /* planted mistake: reads one element past the end */
#endif
    for (long t = 0; t < n; t++) s += v[t] * v[t];
    return sqrt(s);
}

/* ------------------------------------------------------------------ */
/* Inner stage: CG on one diagonal block A_ii (Section 3, the inner    */
/* Krylov solve of each block; Section 3.2, maximum inner iterations)  */
/* ------------------------------------------------------------------ */

/* q = A_ii p on a bx*by*bz block: the 7-point stencil with every
 * neighbour outside the block taken as zero. */
static void block_apply(int bx, int by, int bz, const double *p, double *q)
{
    for (int i = 0; i < bx; i++)
        for (int j = 0; j < by; j++)
            for (int k = 0; k < bz; k++) {
                long c = ((long)i * by + j) * bz + k;
                double s = 6.0 * p[c];
#if ORACLE_MUTANT == 6
                /* planted mistake: periodic wrap instead of zero at the block faces */
                s -= p[(((long)((i + bx - 1) % bx)) * by + j) * bz + k];
#else
                if (i > 0) s -= p[c - (long)by * bz];
#endif
                if (i < bx - 1) s -= p[c + (long)by * bz];
                if (j > 0) s -= p[c - bz];
                if (j < by - 1) s -= p[c + bz];
                if (k > 0) s -= p[c - 1];
                if (k < bz - 1) s -= p[c + 1];
                q[c] = s;
            }
}

static double dot(long n, const double *a, const double *b)
{
    double s = 0.0;
    for (long t = 0; t < n; t++) s += a[t] * b[t];
    return s;
}

/* CG on A_ii d = r from d = 0, at most m iterations.
 * In: r = block residual.  Out: d = correction, r = final inner residual.
 * p, q: scratch of the block's size.  Returns the iterations taken. */
static int block_cg(int bx, int by, int bz, double *r, double *d, double *p,
                    double *q, int m, double inner_tol)
{
    long n = (long)bx * by * bz;
    for (long t = 0; t < n; t++) { d[t] = 0.0; p[t] = r[t]; }
    double rho = dot(n, r, r);
    double rho0 = rho;
    if (rho == 0.0) return 0;
    int it = 0;
    while (it < m) {
        block_apply(bx, by, bz, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0)) break;             /* breakdown guard */
#if ORACLE_MUTANT == 10
        double alpha = sigma / rho;
#else
        double alpha = rho / sigma;
#endif
        for (long t = 0; t < n; t++) {
            d[t] += alpha * p[t];
#if ORACLE_MUTANT == 4
            r[t] += alpha * q[t];
#else
            r[t] -= alpha * q[t];
#endif
        }
        it++;
        double rho_new = dot(n, r, r);
        if (inner_tol > 0.0 && sqrt(rho_new) <= inner_tol * sqrt(rho0)) break;
#if ORACLE_MUTANT == 3
        double beta = rho / rho_new;
#else
        double beta = rho_new / rho;
#endif
        for (long t = 0; t < n; t++) p[t] = r[t] + beta * p[t];
        rho = rho_new;
    }
    return it;
}

/* Same inner stage carried out entirely in single precision (storage and
 * accumulation), used only to attribute the error of mixed precision. */
static void block_apply_f(int bx, int by, int bz, const float *p, float *q)
{
    for (int i = 0; i < bx; i++)
        for (int j = 0; j < by; j++)
            for (int k = 0; k < bz; k++) {
                long c = ((long)i * by + j) * bz + k;
                float s = 6.0f * p[c];
                if (i > 0) s -= p[c - (long)by * bz];
                if (i < bx - 1) s -= p[c + (long)by * bz];
                if (j > 0) s -= p[c - bz];
                if (j < by - 1) s -= p[c + bz];
                if (k > 0) s -= p[c - 1];
                if (k < bz - 1) s -= p[c + 1];
                q[c] = s;
            }
}

static float dot_f(long n, const float *a, const float *b)
{
    float s = 0.0f;
    for (long t = 0; t < n; t++) s += a[t] * b[t];
    return s;
}

static int block_cg_f(int bx, int by, int bz, float *r, float *d, float *p,
                      float *q, int m, double inner_tol)
{
    long n = (long)bx * by * bz;
    for (long t = 0; t < n; t++) { d[t] = 0.0f; p[t] = r[t]; }
    float rho = dot_f(n, r, r);
    float rho0 = rho;
    if (rho == 0.0f) return 0;
    int it = 0;
    while (it < m) {
        block_apply_f(bx, by, bz, p, q);
        float sigma = dot_f(n, p, q);
        if (!(sigma > 0.0f)) break;
        float alpha = rho / sigma;
        for (long t = 0; t < n; t++) { d[t] += alpha * p[t]; r[t] -= alpha * q[t]; }
        it++;
        float rho_new = dot_f(n, r, r);
        if (inner_tol > 0.0 && sqrtf(rho_new) <= (float)inner_tol * sqrtf(rho0)) break;
#if ORACLE_MUTANT == 16
        float beta = rho / rho_new;   /* planted mistake: FP32 beta inverted */
#else
        float beta = rho_new / rho;
#endif
        for (long t = 0; t < n; t++) p[t] = r[t] + beta * p[t];
        rho = rho_new;
    }
    return it;
}

/* ------------------------------------------------------------------ */
/* Block bookkeeping                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    long nx, ny, nz;
    int gx, gy, gz;
    const int *cx, *cy, *cz;
} part_t;

static int check_cuts(const int *c, int g, long n)
{
    if (g < 1 || c[0] != 0 || c[g] != n) return 0;
    for (int t = 0; t < g; t++)
        if (c[t + 1] <= c[t]) return 0;
    return 1;
}

static void block_range(const part_t *P, int b, int *i0, int *j0, int *k0,
                        int *bx, int *by, int *bz)
{
    int bk = b % P->gz, bj = (b / P->gz) % P->gy, bi = b / (P->gz * P->gy);
    *i0 = P->cx[bi]; *j0 = P->cy[bj]; *k0 = P->cz[bk];
    *bx = P->cx[bi + 1] - P->cx[bi];
    *by = P->cy[bj + 1] - P->cy[bj];
    *bz = P->cz[bk + 1] - P->cz[bk];
}

/* copy a block of a global array into a packed buffer, and back */
static void gather(const part_t *P, int b, const double *g, double *loc)
{
    long nx = P->nx, ny = P->ny, nz = P->nz; (void)nx;
    int i0, j0, k0, bx, by, bz;
    block_range(P, b, &i0, &j0, &k0, &bx, &by, &bz);
    for (int i = 0; i < bx; i++)
        for (int j = 0; j < by; j++)
            for (int k = 0; k < bz; k++)
                loc[((long)i * by + j) * bz + k] = g[IDX(i0 + i, j0 + j, k0 + k)];
}

static void scatter(const part_t *P, int b, const double *loc, double *g)
{
    long nx = P->nx, ny = P->ny, nz = P->nz; (void)nx;
    int i0, j0, k0, bx, by, bz;
    block_range(P, b, &i0, &j0, &k0, &bx, &by, &bz);
    for (int i = 0; i < bx; i++)
        for (int j = 0; j < by; j++)
            for (int k = 0; k < bz; k++)
                g[IDX(i0 + i, j0 + j, k0 + k)] = loc[((long)i * by + j) * bz + k];
}

static long max_block_volume(const part_t *P)
{
    long mx = 0;
    for (int a = 0; a < P->gx; a++)
        for (int c = 0; c < P->gy; c++)
            for (int e = 0; e < P->gz; e++) {
                long v = (long)(P->cx[a + 1] - P->cx[a]) * (P->cy[c + 1] - P->cy[c]) *
                         (P->cz[e + 1] - P->cz[e]);
                if (v > mx) mx = v;
            }
    return mx;
}

/* Residual of the current iterate, as the sum over blocks of the squared
 * block residual norms (Section 3: the global residual is the square root
 * of the sum of squares of the block-local residues).  Fills r. */
static double blocked_residual_norm(const part_t *P, const double *beff,
                                    const double *x, double *r)
{
    long nx = P->nx, ny = P->ny, nz = P->nz;
    int nb = P->gx * P->gy * P->gz;
#if ORACLE_MUTANT == 7
    /* planted mistake: residual taken with the block-diagonal operator only
     * (neighbour blocks' values never read) */
    {
        long vmax = max_block_volume(P);
        double *loc = (double *)malloc(sizeof(double) * (size_t)vmax);
        double *out = (double *)malloc(sizeof(double) * (size_t)vmax);
        for (int b = 0; b < nb; b++) {
            int i0, j0, k0, bx, by, bz;
            block_range(P, b, &i0, &j0, &k0, &bx, &by, &bz);
            gather(P, b, x, loc);
            block_apply(bx, by, bz, loc, out);
            scatter(P, b, out, r);
        }
        free(loc); free(out);
#pragma omp parallel for schedule(static)
        for (long t = 0; t < nx * ny * nz; t++) r[t] = beff[t] - r[t];
    }
#else
    or_apply(nx, ny, nz, x, r);
#pragma omp parallel for schedule(static)
    for (long t = 0; t < nx * ny * nz; t++) r[t] = beff[t] - r[t];
#endif
    double total = 0.0;
    for (int b = 0; b < nb; b++) {
        int i0, j0, k0, bx, by, bz;
        block_range(P, b, &i0, &j0, &k0, &bx, &by, &bz);
        double s = 0.0;
        for (int i = 0; i < bx; i++)
            for (int j = 0; j < by; j++)
                for (int k = 0; k < bz; k++) {
                    double v = r[IDX(i0 + i, j0 + j, k0 + k)];
                    s += v * v;
                }
        total += s;
    }
    return sqrt(total);
}

/* ------------------------------------------------------------------ */
/* Outer stage: synchronous block Jacobi (Section 3 block formula and   */
/* Listing 1: test the global residual, inner solve each block, halo    */
/* exchange, repeat)                                                    */
/* ------------------------------------------------------------------ */

/*
 * x (in/out): initial guess on entry, final iterate on exit.
 * history (nullable, length max_sweeps+1): relative residual at the top of
 *   each sweep, history[s] for s = 0..sweeps.
 * precision: 0 = FP64 inner CG; 1 = FP32 inner CG (attribution only).
 * Returns a status; *sweeps_out = number of updates applied.
 */
int or_block_jacobi(long nx, long ny, long nz, int gx, int gy, int gz,
                    const int *cx, const int *cy, const int *cz,
                    const double *beff, double *x, double tol, int m,
                    double inner_tol, int max_sweeps, int precision,
                    double *history, int *sweeps_out, long *inner_out)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (sweeps_out) *sweeps_out = 0;
    if (inner_out) *inner_out = 0;
    if (nx < 1 || ny < 1 || nz < 1 || m < 1 || max_sweeps < 0) return OR_ARG;
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return OR_ARG;
    long n = nx * ny * nz;
    int nb = gx * gy * gz;
    double nbeff = or_norm2(n, beff);
    if (!isfinite(nbeff)) return OR_NONFINITE;
    if (nbeff == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (history) history[0] = 0.0;
        return OR_OK;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *dg = (double *)malloc(sizeof(double) * (size_t)n);
    long vmax = max_block_volume(&P);
    long inner_total = 0;
    int status = OR_OK;
    double res0 = -1.0;
    int s = 0;
    for (;;) {
        double res = blocked_residual_norm(&P, beff, x, r) / nbeff;
        if (history) history[s] = res;
        if (!isfinite(res)) { status = OR_NONFINITE; break; }
        if (res0 < 0.0) res0 = res;
        if (tol > 0.0 && res <= tol) break;
        if (res > 1e6 * res0 && res0 > 0.0) { status = OR_DIVERGED; break; }
        if (s == max_sweeps) { status = tol > 0.0 ? OR_NOT_CONVERGED : OR_OK; break; }
        /* inner solves: each block reads only this sweep's residual */
#pragma omp parallel
        {
            double *lr = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *ld = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *lp = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *lq = (double *)malloc(sizeof(double) * (size_t)vmax);
            float *fr = NULL, *fd = NULL, *fp = NULL, *fq = NULL;
            if (precision == 1) {
                fr = (float *)malloc(sizeof(float) * (size_t)vmax);
                fd = (float *)malloc(sizeof(float) * (size_t)vmax);
                fp = (float *)malloc(sizeof(float) * (size_t)vmax);
                fq = (float *)malloc(sizeof(float) * (size_t)vmax);
            }
#pragma omp for schedule(dynamic, 1) reduction(+ : inner_total)
            for (int b = 0; b < nb; b++) {
                int i0, j0, k0, bx, by, bz;
                block_range(&P, b, &i0, &j0, &k0, &bx, &by, &bz);
                long v = (long)bx * by * bz;
                gather(&P, b, r, lr);
                int it;
                if (precision == 1) {
                    for (long t = 0; t < v; t++) fr[t] = (float)lr[t];
                    it = block_cg_f(bx, by, bz, fr, fd, fp, fq, m, inner_tol);
                    for (long t = 0; t < v; t++) ld[t] = (double)fd[t];
                } else {
                    it = block_cg(bx, by, bz, lr, ld, lp, lq, m, inner_tol);
                }
                inner_total += it;
                scatter(&P, b, ld, dg);
            }
            free(lr); free(ld); free(lp); free(lq);
            free(fr); free(fd); free(fp); free(fq);
        }
        /* Jacobi update, after every block has read the old iterate */
#pragma omp parallel for schedule(static)
        for (long t = 0; t < n; t++) {
#if ORACLE_MUTANT == 5
            x[t] = dg[t];
#else
            x[t] += dg[t];
#endif
        }
        s++;
    }
    free(r); free(dg);
    if (sweeps_out) *sweeps_out = s;
    if (inner_out) *inner_out = inner_total;
    return status;
}

/*
 * One synchronous sweep restricted to a list of blocks: for each listed
 * block b, x_new_b = x_b + d_b with d_b from m inner CG iterations on the
 * residual of x.  Writes the new values of listed blocks into xout (a full
 * array; other entries untouched).  Used to check a GPU sweep one block at a
 * time at sizes where a whole-grid oracle run would take too long.
 */
int or_block_sweep_some(long nx, long ny, long nz, int gx, int gy, int gz,
                        const int *cx, const int *cy, const int *cz,
                        const double *beff, const double *x, int nlist,
                        const int *blocks, int m, double inner_tol,
                        double *xout)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return OR_ARG;
    long vmax = max_block_volume(&P);
    int nb = gx * gy * gz;
    for (int t = 0; t < nlist; t++)
        if (blocks[t] < 0 || blocks[t] >= nb) return OR_ARG;
#pragma omp parallel
    {
        double *lr = (double *)malloc(sizeof(double) * (size_t)vmax);
        double *ld = (double *)malloc(sizeof(double) * (size_t)vmax);
        double *lp = (double *)malloc(sizeof(double) * (size_t)vmax);
        double *lq = (double *)malloc(sizeof(double) * (size_t)vmax);
#pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < nlist; t++) {
            int b = blocks[t];
            int i0, j0, k0, bx, by, bz;
            block_range(&P, b, &i0, &j0, &k0, &bx, &by, &bz);
            /* block residual b_eff - A x, read cell by cell with the global
             * operator (neighbour-block values are the halo) */
            for (int i = 0; i < bx; i++)
                for (int j = 0; j < by; j++)
                    for (int k = 0; k < bz; k++) {
                        long I = i0 + i, J = j0 + j, K = k0 + k;
                        double s = 6.0 * x[IDX(I, J, K)];
                        if (I > 0) s -= x[IDX(I - 1, J, K)];
                        if (I < nx - 1) s -= x[IDX(I + 1, J, K)];
                        if (J > 0) s -= x[IDX(I, J - 1, K)];
                        if (J < ny - 1) s -= x[IDX(I, J + 1, K)];
                        if (K > 0) s -= x[IDX(I, J, K - 1)];
                        if (K < nz - 1) s -= x[IDX(I, J, K + 1)];
                        lr[((long)i * by + j) * bz + k] = beff[IDX(I, J, K)] - s;
                    }
            block_cg(bx, by, bz, lr, ld, lp, lq, m, inner_tol);
            for (int i = 0; i < bx; i++)
                for (int j = 0; j < by; j++)
                    for (int k = 0; k < bz; k++) {
                        long c = ((long)i * by + j) * bz + k;
                        xout[IDX(i0 + i, j0 + j, k0 + k)] = x[IDX(i0 + i, j0 + j, k0 + k)] + ld[c];
                    }
        }
        free(lr); free(ld); free(lp); free(lq);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Asynchronous outer iterations, bounded-delay model (Section 2.3: the */
/* latest received values are used; Section 2.1: whatever halo values   */
/* a process has).  Deterministic given the delay table.                */
/* ------------------------------------------------------------------ */

/*
 * Every block advances one sweep at a time, but in sweep s the value of
 * neighbour block j seen by block i is x_j from sweep s - delay, with
 * delay = delays[(s * nb + i) * 6 + f] (f = the face -x,+x,-y,+y,-z,+z
 * across which j lies), clipped to [0, min(S, s)].  Delays are supplied
 * by the caller (seeded), so the run is reproducible.  The stopping test
 * uses the true residual of the current iterate.  With all delays 0 this
 * is the synchronous method exactly.
 */
int or_block_jacobi_async(long nx, long ny, long nz, int gx, int gy, int gz,
                          const int *cx, const int *cy, const int *cz,
                          const double *beff, double *x, double tol, int m,
                          int max_sweeps, int S, const int *delays,
                          double *history, int *sweeps_out)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (sweeps_out) *sweeps_out = 0;
    if (nx < 1 || ny < 1 || nz < 1 || m < 1 || S < 0 || max_sweeps < 0) return OR_ARG;
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return OR_ARG;
    long n = nx * ny * nz;
    int nb = gx * gy * gz;
    double nbeff = or_norm2(n, beff);
    if (nbeff == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (history) history[0] = 0.0;
        return OR_OK;
    }
    /* ring of past iterates: hist[v % (S+1)] = x after v sweeps */
    int ring = S + 1;
    double **hist = (double **)malloc(sizeof(double *) * (size_t)ring);
    for (int t = 0; t < ring; t++) hist[t] = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(hist[0], x, sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *xn = (double *)malloc(sizeof(double) * (size_t)n);
    long vmax = max_block_volume(&P);
    int status = OR_OK;
    int s = 0;
    for (;;) {
        const double *xc = hist[s % ring];
        double res = or_residual(nx, ny, nz, beff, xc, r) / nbeff;
        if (history) history[s] = res;
        if (!isfinite(res)) { status = OR_NONFINITE; break; }
        if (tol > 0.0 && res <= tol) break;
        if (s == max_sweeps) { status = tol > 0.0 ? OR_NOT_CONVERGED : OR_OK; break; }
#pragma omp parallel
        {
            double *lr = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *ld = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *lp = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *lq = (double *)malloc(sizeof(double) * (size_t)vmax);
#pragma omp for schedule(dynamic, 1)
            for (int b = 0; b < nb; b++) {
                int i0, j0, k0, bx, by, bz;
                block_range(&P, b, &i0, &j0, &k0, &bx, &by, &bz);
                const double *src[6];
                for (int f = 0; f < 6; f++) {
                    int dl = delays ? delays[((long)s * nb + b) * 6 + f] : 0;
                    if (dl < 0) dl = 0;
                    if (dl > S) dl = S;
                    if (dl > s) dl = s;
#if ORACLE_MUTANT == 15
                    dl = 0;   /* planted mistake: the delay table is ignored */
#endif
                    src[f] = hist[(s - dl) % ring];
                }
                for (int i = 0; i < bx; i++)
                    for (int j = 0; j < by; j++)
                        for (int k = 0; k < bz; k++) {
                            long I = i0 + i, J = j0 + j, K = k0 + k;
                            double v = 6.0 * xc[IDX(I, J, K)];
                            /* in-block neighbours from the current iterate,
                             * off-block neighbours from the delayed one */
                            if (I > 0) v -= (i > 0 ? xc : src[0])[IDX(I - 1, J, K)];
                            if (I < nx - 1) v -= (i < bx - 1 ? xc : src[1])[IDX(I + 1, J, K)];
                            if (J > 0) v -= (j > 0 ? xc : src[2])[IDX(I, J - 1, K)];
                            if (J < ny - 1) v -= (j < by - 1 ? xc : src[3])[IDX(I, J + 1, K)];
                            if (K > 0) v -= (k > 0 ? xc : src[4])[IDX(I, J, K - 1)];
                            if (K < nz - 1) v -= (k < bz - 1 ? xc : src[5])[IDX(I, J, K + 1)];
                            lr[((long)i * by + j) * bz + k] = beff[IDX(I, J, K)] - v;
                        }
                block_cg(bx, by, bz, lr, ld, lp, lq, m, 0.0);
                for (int i = 0; i < bx; i++)
                    for (int j = 0; j < by; j++)
                        for (int k = 0; k < bz; k++) {
                            long c = ((long)i * by + j) * bz + k;
                            long G = IDX(i0 + i, j0 + j, k0 + k);
                            xn[G] = xc[G] + ld[c];
                        }
            }
            free(lr); free(ld); free(lp); free(lq);
        }
        s++;
        memcpy(hist[s % ring], xn, sizeof(double) * (size_t)n);
    }
    memcpy(x, hist[s % ring], sizeof(double) * (size_t)n);
    for (int t = 0; t < ring; t++) free(hist[t]);
    free(hist); free(r); free(xn);
    if (sweeps_out) *sweeps_out = s;
    return status;
}

/*
 * Asynchronous outer iterations replayed from a schedule of block sweeps
 * (Section 2.3: a block's next inner solve uses the latest neighbour
 * values it has received, whatever their age; Section 2.1: a process goes
 * on with whatever halo values it holds).  Event e sweeps block
 * ev_block[e] once, starting from that block's own latest values; the
 * values of the neighbour block across face f (-x,+x,-y,+y,-z,+z) are that
 * block's iterate after ev_seen[6e + f] of its own sweeps (entries for
 * faces without a neighbour are ignored).  The sweep is the synchronous
 * one restricted to the block: residual with the global operator, at most
 * m inner CG iterations (FP64, or FP32 storage and accumulation when
 * precision = 1), x_i += d.  Every version of every block is kept.
 * Returns OR_ARG when an event names a version that an earlier event has
 * not produced.  x: initial iterate in (version 0 of every block), every
 * block's latest version out.  sweeps_out (nullable, nb entries): sweeps
 * applied to each block.
 *
 * An event's result depends only on the versions it names, so events are
 * computed level by level (an event's level is one more than the levels of
 * the events that produced its inputs) with the events of one level in
 * parallel; the arithmetic of each event is the same as in schedule order.
 */
int or_async_replay(long nx, long ny, long nz, int gx, int gy, int gz,
                    const int *cx, const int *cy, const int *cz,
                    const double *beff, double *x, int m, int precision,
                    int nev, const int *ev_block, const int *ev_seen, int *sweeps_out)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (nx < 1 || ny < 1 || nz < 1 || m < 1 || nev < 0) return OR_ARG;
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return OR_ARG;
    int nb = gx * gy * gz;
    long vmax = max_block_volume(&P);
    /* pass 1, in schedule order: validate, number the versions, levels */
    int *ver = (int *)calloc((size_t)nb, sizeof(int));
    int *ev_ver = (int *)malloc(sizeof(int) * (size_t)(nev > 0 ? nev : 1));
    int *level = (int *)malloc(sizeof(int) * (size_t)(nev > 0 ? nev : 1));
    int *nbrs = (int *)malloc(sizeof(int) * 6 * (size_t)(nev > 0 ? nev : 1));
    long total_versions = nb;
    int status = OR_OK;
    for (int e = 0; e < nev; e++) {
        int b = ev_block[e];
        if (b < 0 || b >= nb) { status = OR_ARG; break; }
        int bk = b % gz, bj = (b / gz) % gy, bi = b / (gz * gy);
        int nbr[6] = {bi > 0 ? b - gy * gz : -1, bi < gx - 1 ? b + gy * gz : -1,
                      bj > 0 ? b - gz : -1, bj < gy - 1 ? b + gz : -1,
                      bk > 0 ? b - 1 : -1, bk < gz - 1 ? b + 1 : -1};
        for (int f = 0; f < 6; f++) {
            nbrs[6L * e + f] = nbr[f];
            if (nbr[f] >= 0) {
                int w = ev_seen[6L * e + f];
                if (w < 0 || w > ver[nbr[f]]) status = OR_ARG;
            }
        }
        if (status != OR_OK) break;
        ev_ver[e] = ver[b]++;
        total_versions++;
    }
    int *vcount = (int *)malloc(sizeof(int) * (size_t)nb);
    for (int b = 0; b < nb; b++) vcount[b] = ver[b] + 1;
    /* hist[b][v]: block b after v of its sweeps; prod[b][v]: the event that
     * produced it (-1 for the initial values) */
    double ***hist = (double ***)calloc((size_t)nb, sizeof(double **));
    int **prod = (int **)calloc((size_t)nb, sizeof(int *));
    for (int b = 0; b < nb && status == OR_OK; b++) {
        hist[b] = (double **)calloc((size_t)vcount[b], sizeof(double *));
        prod[b] = (int *)malloc(sizeof(int) * (size_t)vcount[b]);
        prod[b][0] = -1;
        int i0, j0, k0, bx, by, bz;
        block_range(&P, b, &i0, &j0, &k0, &bx, &by, &bz);
        for (int v = 0; v < vcount[b]; v++)
            hist[b][v] = (double *)malloc(sizeof(double) * (size_t)bx * by * bz);
        gather(&P, b, x, hist[b][0]);
    }
    int maxlvl = 0;
    for (int e = 0; e < nev && status == OR_OK; e++) {
        int b = ev_block[e];
        prod[b][ev_ver[e] + 1] = e;
        int lv = 0, q = prod[b][ev_ver[e]];
        if (q >= 0 && level[q] + 1 > lv) lv = level[q] + 1;
        for (int f = 0; f < 6; f++) {
            int j = nbrs[6L * e + f];
            if (j < 0) continue;
            q = prod[j][ev_seen[6L * e + f]];
            if (q >= 0 && level[q] + 1 > lv) lv = level[q] + 1;
        }
        level[e] = lv;
        if (lv > maxlvl) maxlvl = lv;
    }
    /* pass 2: the sweeps, level by level */
    for (int lv = 0; lv <= maxlvl && status == OR_OK && nev > 0; lv++) {
#pragma omp parallel
        {
            double *lr = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *ld = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *lp = (double *)malloc(sizeof(double) * (size_t)vmax);
            double *lq = (double *)malloc(sizeof(double) * (size_t)vmax);
            float *fr = (float *)malloc(sizeof(float) * (size_t)vmax);
            float *fd = (float *)malloc(sizeof(float) * (size_t)vmax);
            float *fp = (float *)malloc(sizeof(float) * (size_t)vmax);
            float *fq = (float *)malloc(sizeof(float) * (size_t)vmax);
#pragma omp for schedule(dynamic, 1)
            for (int e = 0; e < nev; e++) {
                if (level[e] != lv) continue;
                int b = ev_block[e];
                const double *src[6] = {NULL, NULL, NULL, NULL, NULL, NULL};
                int src_b[6];
                for (int f = 0; f < 6; f++) {
                    src_b[f] = nbrs[6L * e + f];
                    if (src_b[f] < 0) continue;
                    int w = ev_seen[6L * e + f];
#if ORACLE_MUTANT == 17
                    w = vcount[src_b[f]] - 1;   /* planted mistake: the newest version */
#endif
                    src[f] = hist[src_b[f]][w];
                }
                int i0, j0, k0, bx, by, bz;
                block_range(&P, b, &i0, &j0, &k0, &bx, &by, &bz);
                const double *own = hist[b][ev_ver[e]];
                for (int i = 0; i < bx; i++)
                    for (int j = 0; j < by; j++)
                        for (int k = 0; k < bz; k++) {
                            long I = i0 + i, J = j0 + j, K = k0 + k;
                            long c = ((long)i * by + j) * bz + k;
                            double v = 6.0 * own[c];
                            /* in-block neighbours from the block's own values */
                            if (i > 0) v -= own[c - (long)by * bz];
                            if (j > 0) v -= own[c - bz];
                            if (k > 0) v -= own[c - 1];
                            if (i < bx - 1) v -= own[c + (long)by * bz];
                            if (j < by - 1) v -= own[c + bz];
                            if (k < bz - 1) v -= own[c + 1];
                            /* off-block neighbours from the scheduled versions;
                             * (I2,J2,K2) is the neighbour cell, local to block f */
                            for (int f = 0; f < 6; f++) {
                                int out = (f == 0 && i == 0 && I > 0) ||
                                          (f == 1 && i == bx - 1 && I < nx - 1) ||
                                          (f == 2 && j == 0 && J > 0) ||
                                          (f == 3 && j == by - 1 && J < ny - 1) ||
                                          (f == 4 && k == 0 && K > 0) ||
                                          (f == 5 && k == bz - 1 && K < nz - 1);
                                if (!out) continue;
                                long I2 = I - (f == 0) + (f == 1);
                                long J2 = J - (f == 2) + (f == 3);
                                long K2 = K - (f == 4) + (f == 5);
                                int n0, n1, n2, ex, ey, ez;
                                block_range(&P, src_b[f], &n0, &n1, &n2, &ex, &ey, &ez);
                                v -= src[f][((I2 - n0) * ey + (J2 - n1)) * ez + (K2 - n2)];
                            }
                            lr[c] = beff[IDX(I, J, K)] - v;
                        }
                long vol = (long)bx * by * bz;
                if (precision == 1) {
                    for (long t = 0; t < vol; t++) fr[t] = (float)lr[t];
                    block_cg_f(bx, by, bz, fr, fd, fp, fq, m, 0.0);
                    for (long t = 0; t < vol; t++) ld[t] = (double)fd[t];
                } else {
                    block_cg(bx, by, bz, lr, ld, lp, lq, m, 0.0);
                }
                double *dst = hist[b][ev_ver[e] + 1];
                for (long t = 0; t < vol; t++) dst[t] = own[t] + ld[t];
            }
            free(lr); free(ld); free(lp); free(lq); free(fr); free(fd); free(fp); free(fq);
        }
    }
    if (status == OR_OK)
        for (int b = 0; b < nb; b++) scatter(&P, b, hist[b][ver[b]], x);
    if (sweeps_out)
        for (int b = 0; b < nb; b++) sweeps_out[b] = ver[b];
    for (int b = 0; b < nb; b++) {
        if (hist[b])
            for (int v = 0; v < vcount[b]; v++) free(hist[b][v]);
        free(hist[b]);
        free(prod[b]);
    }
    free(hist); free(prod); free(vcount); free(ver); free(ev_ver); free(level); free(nbrs);
    (void)total_versions;
    return status;
}

/* ------------------------------------------------------------------ */
/* Conventional solver: CG on the whole system (the global Krylov      */
/* baseline the block method is compared against, Section 4)           */
/* ------------------------------------------------------------------ */

int or_cg(long nx, long ny, long nz, const double *beff, double *x, double tol,
          int max_iters, double *history, int *iters_out)
{
    long n = nx * ny * nz;
    if (iters_out) *iters_out = 0;
    double nbeff = or_norm2(n, beff);
    if (nbeff == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (history) history[0] = 0.0;
        return OR_OK;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    or_residual(nx, ny, nz, beff, x, r);
    memcpy(p, r, sizeof(double) * (size_t)n);
    double rho = dot(n, r, r);
    int it = 0, status = OR_OK;
    for (;;) {
        double res = sqrt(rho) / nbeff;   /* recurrence residual */
        if (history) history[it] = res;
        if (!isfinite(res)) { status = OR_NONFINITE; break; }
        if (tol > 0.0 && res <= tol) break;
        if (it == max_iters) { status = tol > 0.0 ? OR_NOT_CONVERGED : OR_OK; break; }
        or_apply(nx, ny, nz, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0)) break;
        double alpha = rho / sigma;
        for (long t = 0; t < n; t++) { x[t] += alpha * p[t]; r[t] -= alpha * q[t]; }
        double rho_new = dot(n, r, r);
        double beta = rho_new / rho;
        for (long t = 0; t < n; t++) p[t] = r[t] + beta * p[t];
        rho = rho_new;
        it++;
    }
    free(r); free(p); free(q);
    if (iters_out) *iters_out = it;
    return status;
}

/* ------------------------------------------------------------------ */
/* Overlapping blocks (Section 3.2, choice of parameters: the block     */
/* overlap, and the multisplitting weights D_i of Section 2.3)          */
/* ------------------------------------------------------------------ */

/*
 * Reading of the paper: the region of block b for overlap o holds the
 * block's own cells and, across each face that has a neighbouring block,
 * the slab of depth o beyond that face (clipped to the interior): the cells
 * a face halo of depth o carries.  Cells off the block's box along two or
 * more axes (edge and corner regions) are not in it.  That is what gives
 * o(2xy + 2yz + 2zx) extra unknowns for an x*y*z block with neighbours on
 * every side, the count the paper states.
 *
 * Each block solves A_RR d = r_R on its region R (the principal submatrix
 * of A: neighbours outside R are zero, i.e. a zero correction there), and
 * the new value of every cell is the one computed by the block that owns
 * it: the weights D_i of the multisplitting B = sum_i D_i M_i^{-1} N_i are
 * the indicator of block i's own cells (restricted weighting).  With o = 0
 * this is the block Jacobi iteration above.
 */

/* how far coordinate c lies outside [a, a + len) (0 when inside) */
static long outside_by(long c, long a, long len)
{
    if (c < a) return a - c;
    if (c >= a + len) return c - (a + len) + 1;
    return 0;
}

/* 1 when interior cell (I,J,K) belongs to block b's region for overlap o */
static int in_region(const part_t *P, int b, int o, long I, long J, long K)
{
    if (I < 0 || J < 0 || K < 0 || I >= P->nx || J >= P->ny || K >= P->nz) return 0;
    int i0, j0, k0, bx, by, bz;
    block_range(P, b, &i0, &j0, &k0, &bx, &by, &bz);
    long dx = outside_by(I, i0, bx), dy = outside_by(J, j0, by), dz = outside_by(K, k0, bz);
#if ORACLE_MUTANT == 11
    /* planted mistake: the region is the whole box grown by o (edges and
     * corners included) */
    return dx <= o && dy <= o && dz <= o;
#else
    int nout = (dx > 0) + (dy > 0) + (dz > 0);
    if (nout == 0) return 1;
    if (nout > 1) return 0;
    return dx + dy + dz <= o;
#endif
}

typedef struct {
    long n;          /* cells in the region */
    long *cell;      /* region cell -> global index, in C order of the grid */
    int *nbr;        /* region cell -> 6 region neighbours (-x,+x,-y,+y,-z,+z; -1 none) */
    unsigned char *own;  /* region cell -> 1 when block b owns it */
} region_t;

static void region_free(region_t *R)
{
    free(R->cell); free(R->nbr); free(R->own);
    R->cell = NULL; R->nbr = NULL; R->own = NULL; R->n = 0;
}

/* Enumerate block b's region (cells in C order) and its neighbour table. */
static void region_build(const part_t *P, int b, int o, region_t *R)
{
    long nx = P->nx, ny = P->ny, nz = P->nz;
    int i0, j0, k0, bx, by, bz;
    block_range(P, b, &i0, &j0, &k0, &bx, &by, &bz);
    /* a box that contains the region: the block grown by o, clipped */
    long a0 = i0 - o < 0 ? 0 : i0 - o, a1 = i0 + bx + o > nx ? nx : i0 + bx + o;
    long b0 = j0 - o < 0 ? 0 : j0 - o, b1 = j0 + by + o > ny ? ny : j0 + by + o;
    long c0 = k0 - o < 0 ? 0 : k0 - o, c1 = k0 + bz + o > nz ? nz : k0 + bz + o;
    long ex = a1 - a0, ey = b1 - b0, ez = c1 - c0;
    long *map = (long *)malloc(sizeof(long) * (size_t)(ex * ey * ez));
    long n = 0;
    for (long I = a0; I < a1; I++)
        for (long J = b0; J < b1; J++)
            for (long K = c0; K < c1; K++) {
                long q = ((I - a0) * ey + (J - b0)) * ez + (K - c0);
                map[q] = in_region(P, b, o, I, J, K) ? n++ : -1;
            }
    R->n = n;
    R->cell = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    R->nbr = (int *)malloc(sizeof(int) * 6 * (size_t)(n > 0 ? n : 1));
    R->own = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
    for (long I = a0; I < a1; I++)
        for (long J = b0; J < b1; J++)
            for (long K = c0; K < c1; K++) {
                long q = ((I - a0) * ey + (J - b0)) * ez + (K - c0);
                long c = map[q];
                if (c < 0) continue;
                R->cell[c] = IDX(I, J, K);
                R->own[c] = outside_by(I, i0, bx) == 0 && outside_by(J, j0, by) == 0 &&
                            outside_by(K, k0, bz) == 0;
                long nb[6] = {-1, -1, -1, -1, -1, -1};
                if (I > a0) nb[0] = map[q - ey * ez];
                if (I < a1 - 1) nb[1] = map[q + ey * ez];
                if (J > b0) nb[2] = map[q - ez];
                if (J < b1 - 1) nb[3] = map[q + ez];
                if (K > c0) nb[4] = map[q - 1];
                if (K < c1 - 1) nb[5] = map[q + 1];
                for (int f = 0; f < 6; f++) R->nbr[6 * c + f] = (int)nb[f];
            }
    free(map);
}

/* q = A_RR p: 6 p minus the region neighbours, in the order -x,+x,-y,+y,-z,+z */
static void region_apply(const region_t *R, const double *p, double *q)
{
    for (long c = 0; c < R->n; c++) {
        double s = 6.0 * p[c];
        for (int f = 0; f < 6; f++) {
            int t = R->nbr[6 * c + f];
            if (t >= 0) s -= p[t];
        }
        q[c] = s;
    }
}

/* CG on A_RR d = r from d = 0 (the same recurrences, stops and guard as
 * block_cg), on the region's cells. */
static int region_cg(const region_t *R, double *r, double *d, double *p, double *q, int m,
                     double inner_tol)
{
    long n = R->n;
    for (long t = 0; t < n; t++) { d[t] = 0.0; p[t] = r[t]; }
    double rho = dot(n, r, r);
    double rho0 = rho;
    if (rho == 0.0) return 0;
    int it = 0;
    while (it < m) {
        region_apply(R, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0)) break;
        double alpha = rho / sigma;
        for (long t = 0; t < n; t++) {
            d[t] += alpha * p[t];
            r[t] -= alpha * q[t];
        }
        it++;
        double rho_new = dot(n, r, r);
        if (inner_tol > 0.0 && sqrt(rho_new) <= inner_tol * sqrt(rho0)) break;
        double beta = rho_new / rho;
        for (long t = 0; t < n; t++) p[t] = r[t] + beta * p[t];
        rho = rho_new;
    }
    return it;
}

/* Cells in block b's region for overlap o (-1 on bad arguments). */
long or_overlap_cells(long nx, long ny, long nz, int gx, int gy, int gz, const int *cx,
                      const int *cy, const int *cz, int o, int b)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (o < 0 || b < 0 || b >= gx * gy * gz) return -1;
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return -1;
    region_t R;
    region_build(&P, b, o, &R);
    long n = R.n;
    region_free(&R);
    return n;
}

/* Region residual r_R = b_eff - A x at the region's cells (global operator:
 * values outside the region are the halo). */
static void region_residual(const part_t *P, const region_t *R, const double *beff,
                            const double *x, double *r)
{
    long nx = P->nx, ny = P->ny, nz = P->nz;
    for (long c = 0; c < R->n; c++) {
        long G = R->cell[c];
        long K = G % nz, J = (G / nz) % ny, I = G / (ny * nz);
        double s = 6.0 * x[G];
        if (I > 0) s -= x[IDX(I - 1, J, K)];
        if (I < nx - 1) s -= x[IDX(I + 1, J, K)];
        if (J > 0) s -= x[IDX(I, J - 1, K)];
        if (J < ny - 1) s -= x[IDX(I, J + 1, K)];
        if (K > 0) s -= x[IDX(I, J, K - 1)];
        if (K < nz - 1) s -= x[IDX(I, J, K + 1)];
        r[c] = beff[G] - s;
    }
}

/* Combine block corrections with the weights D_i: the owner's value. */
static void region_combine(const region_t *R, const double *d, double *dg)
{
    for (long c = 0; c < R->n; c++) {
#if ORACLE_MUTANT == 12
        /* planted mistake: every block's correction added at every region
         * cell (no weights) */
        dg[R->cell[c]] += d[c];
#else
        if (R->own[c]) dg[R->cell[c]] = d[c];
#endif
    }
}

/* Forward declarations: the generic drivers below (any overlap, CG or
 * GMRES inner solves). */
int or_multisplit(long nx, long ny, long nz, int gx, int gy, int gz,
                  const int *cx, const int *cy, const int *cz, int o, int inner,
                  const double *beff, double *x, double tol, int m,
                  double inner_tol, int max_sweeps, double *history,
                  int *sweeps_out, long *inner_out);
int or_multisplit_sweep_some(long nx, long ny, long nz, int gx, int gy, int gz,
                             const int *cx, const int *cy, const int *cz, int o, int inner,
                             const double *beff, const double *x, int nlist,
                             const int *blocks, int m, double inner_tol, double *xout);

/*
 * Synchronous block Jacobi with overlap o and CG inner solves (o = 0:
 * or_block_jacobi).  Same arguments, test, history and statuses as
 * or_block_jacobi (FP64 only).
 */
int or_block_jacobi_ovl(long nx, long ny, long nz, int gx, int gy, int gz,
                        const int *cx, const int *cy, const int *cz, int o,
                        const double *beff, double *x, double tol, int m,
                        double inner_tol, int max_sweeps, double *history,
                        int *sweeps_out, long *inner_out)
{
    return or_multisplit(nx, ny, nz, gx, gy, gz, cx, cy, cz, o, 0, beff, x, tol, m,
                         inner_tol, max_sweeps, history, sweeps_out, inner_out);
}

/*
 * One synchronous sweep with overlap o and CG inner solves restricted to a
 * list of blocks: the owned cells of each listed block get x + d (d from m
 * CG iterations on the block's region); other entries of xout are left
 * untouched.
 */
int or_ovl_sweep_some(long nx, long ny, long nz, int gx, int gy, int gz,
                      const int *cx, const int *cy, const int *cz, int o,
                      const double *beff, const double *x, int nlist,
                      const int *blocks, int m, double inner_tol, double *xout)
{
    return or_multisplit_sweep_some(nx, ny, nz, gx, gy, gz, cx, cy, cz, o, 0, beff, x, nlist,
                                    blocks, m, inner_tol, xout);
}

/* ------------------------------------------------------------------ */
/* Inner stage with GMRES (Sections 3.1 and 4: the experiments used     */
/* GMRES as the inner Krylov solver; Section 3.2: a maximum number of   */
/* inner iterations)                                                    */
/* ------------------------------------------------------------------ */

/*
 * One GMRES(m) cycle on A_RR d = r from d = 0 (the region of a block; with
 * overlap 0 the block itself).  Arnoldi builds an orthonormal basis
 * v_0 = r/||r||, v_1, ... of the Krylov space span{r, A r, A^2 r, ...}: each
 * new vector w = A v_j is orthogonalised against every earlier basis
 * vector with coefficients taken from the same w (classical Gram-Schmidt)
 * and normalised; the (k+1) x k Hessenberg matrix of coefficients is
 * reduced to triangular form by Givens rotations as it grows, which also
 * gives the least-squares residual |g_{k}|.  d = V y minimises
 * ||r - A_RR d||_2 over the Krylov space, with y from the triangular solve.
 * Stops after m steps, when |g_k| <= inner_tol * ||r|| (inner_tol > 0), or
 * when the new vector vanishes (the Krylov space is invariant: exact).
 * Returns the steps taken.
 */
static int region_gmres(const region_t *R, const double *r, double *d, int m,
                        double inner_tol)
{
    long n = R->n;
    for (long t = 0; t < n; t++) d[t] = 0.0;
    double beta = sqrt(dot(n, r, r));
    if (beta == 0.0) return 0;
    double *V = (double *)malloc(sizeof(double) * (size_t)(n * (m + 1)));
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *H = (double *)calloc((size_t)((m + 1) * m), sizeof(double)); /* H[i*m + j] */
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)calloc((size_t)(m + 1), sizeof(double));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    for (long t = 0; t < n; t++) V[t] = r[t] / beta;
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; j++) {
        double *vj = V + (long)j * n;
        region_apply(R, vj, w);
        /* classical Gram-Schmidt: all coefficients from the same w */
        for (int i = 0; i <= j; i++) {
#if ORACLE_MUTANT == 14
            /* planted mistake: the newest basis vector is left out */
            if (i == j) { H[i * m + j] = 0.0; continue; }
#endif
            H[i * m + j] = dot(n, w, V + (long)i * n);
        }
        for (int i = 0; i <= j; i++) {
            const double hij = H[i * m + j];
            const double *vi = V + (long)i * n;
            for (long t = 0; t < n; t++) w[t] -= hij * vi[t];
        }
        double hn = sqrt(dot(n, w, w));
        H[(j + 1) * m + j] = hn;
        /* earlier rotations applied to the new column */
#if ORACLE_MUTANT != 13
        for (int i = 0; i < j; i++) {
            double a = H[i * m + j], b = H[(i + 1) * m + j];
            H[i * m + j] = cs[i] * a + sn[i] * b;
            H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
        }
#endif
        double a = H[j * m + j];
        double den = sqrt(a * a + hn * hn);
        if (!(den > 0.0)) break;                  /* nothing left to reduce */
        cs[j] = a / den;
        sn[j] = hn / den;
        H[j * m + j] = den;
        H[(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        k = j + 1;
        if (!(hn > 0.0)) break;                   /* invariant Krylov space: exact */
        double *vn = V + (long)(j + 1) * n;
        for (long t = 0; t < n; t++) vn[t] = w[t] / hn;
        if (inner_tol > 0.0 && fabs(g[j + 1]) <= inner_tol * beta) break;
    }
    /* back substitution R y = g, then d = V y */
    for (int i = k - 1; i >= 0; i--) {
        double s = g[i];
        for (int l = i + 1; l < k; l++) s -= H[i * m + l] * y[l];
        y[i] = s / H[i * m + i];
    }
    for (int i = 0; i < k; i++) {
        const double *vi = V + (long)i * n;
        for (long t = 0; t < n; t++) d[t] += y[i] * vi[t];
    }
    free(V); free(w); free(H); free(cs); free(sn); free(g); free(y);
    return k;
}

/* Inner solve on a region: 0 = CG, 1 = GMRES.  r is overwritten by CG. */
static int region_inner(const region_t *R, int inner, double *r, double *d, double *p,
                        double *q, int m, double inner_tol)
{
    if (inner == 1) return region_gmres(R, r, d, m, inner_tol);
    return region_cg(R, r, d, p, q, m, inner_tol);
}

/*
 * Synchronous two-stage multisplitting with overlap o (0 = plain blocks)
 * and inner solver `inner` (0 = CG, 1 = GMRES).  Same test, history and
 * statuses as or_block_jacobi (FP64).
 */
int or_multisplit(long nx, long ny, long nz, int gx, int gy, int gz,
                  const int *cx, const int *cy, const int *cz, int o, int inner,
                  const double *beff, double *x, double tol, int m,
                  double inner_tol, int max_sweeps, double *history,
                  int *sweeps_out, long *inner_out)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (sweeps_out) *sweeps_out = 0;
    if (inner_out) *inner_out = 0;
    if (nx < 1 || ny < 1 || nz < 1 || m < 1 || max_sweeps < 0 || o < 0) return OR_ARG;
    if (inner != 0 && inner != 1) return OR_ARG;
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return OR_ARG;
    long n = nx * ny * nz;
    int nb = gx * gy * gz;
    double nbeff = or_norm2(n, beff);
    if (!isfinite(nbeff)) return OR_NONFINITE;
    if (nbeff == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (history) history[0] = 0.0;
        return OR_OK;
    }
    region_t *R = (region_t *)malloc(sizeof(region_t) * (size_t)nb);
    double **dloc = (double **)malloc(sizeof(double *) * (size_t)nb);
    long rmax = 1;
    for (int b = 0; b < nb; b++) {
        region_build(&P, b, o, &R[b]);
        dloc[b] = (double *)malloc(sizeof(double) * (size_t)(R[b].n > 0 ? R[b].n : 1));
        if (R[b].n > rmax) rmax = R[b].n;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *dg = (double *)malloc(sizeof(double) * (size_t)n);
    long inner_total = 0;
    int status = OR_OK;
    double res0 = -1.0;
    int s = 0;
    for (;;) {
        /* global residual: every cell counted once, by its owner */
        double res = blocked_residual_norm(&P, beff, x, r) / nbeff;
        if (history) history[s] = res;
        if (!isfinite(res)) { status = OR_NONFINITE; break; }
        if (res0 < 0.0) res0 = res;
        if (tol > 0.0 && res <= tol) break;
        if (res > 1e6 * res0 && res0 > 0.0) { status = OR_DIVERGED; break; }
        if (s == max_sweeps) { status = tol > 0.0 ? OR_NOT_CONVERGED : OR_OK; break; }
        /* inner solves on the regions, all from this sweep's residual */
#pragma omp parallel
        {
            double *lr = (double *)malloc(sizeof(double) * (size_t)rmax);
            double *lp = (double *)malloc(sizeof(double) * (size_t)rmax);
            double *lq = (double *)malloc(sizeof(double) * (size_t)rmax);
#pragma omp for schedule(dynamic, 1) reduction(+ : inner_total)
            for (int b = 0; b < nb; b++) {
                for (long c = 0; c < R[b].n; c++) lr[c] = r[R[b].cell[c]];
                inner_total += region_inner(&R[b], inner, lr, dloc[b], lp, lq, m, inner_tol);
            }
            free(lr); free(lp); free(lq);
        }
        /* x^(k) = x^(k-1) + sum_i D_i (extended correction of block i) */
        memset(dg, 0, sizeof(double) * (size_t)n);
        for (int b = 0; b < nb; b++) region_combine(&R[b], dloc[b], dg);
#pragma omp parallel for schedule(static)
        for (long t = 0; t < n; t++) x[t] += dg[t];
        s++;
    }
    for (int b = 0; b < nb; b++) { region_free(&R[b]); free(dloc[b]); }
    free(R); free(dloc); free(r); free(dg);
    if (sweeps_out) *sweeps_out = s;
    if (inner_out) *inner_out = inner_total;
    return status;
}

/* One synchronous sweep (overlap o, inner solver `inner`) restricted to a
 * list of blocks: the owned cells of each listed block get x + d; other
 * entries of xout are left untouched. */
int or_multisplit_sweep_some(long nx, long ny, long nz, int gx, int gy, int gz,
                             const int *cx, const int *cy, const int *cz, int o, int inner,
                             const double *beff, const double *x, int nlist,
                             const int *blocks, int m, double inner_tol, double *xout)
{
    part_t P = {nx, ny, nz, gx, gy, gz, cx, cy, cz};
    if (o < 0 || (inner != 0 && inner != 1)) return OR_ARG;
    if (!check_cuts(cx, gx, nx) || !check_cuts(cy, gy, ny) || !check_cuts(cz, gz, nz))
        return OR_ARG;
    int nb = gx * gy * gz;
    for (int t = 0; t < nlist; t++)
        if (blocks[t] < 0 || blocks[t] >= nb) return OR_ARG;
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nlist; t++) {
        region_t R;
        region_build(&P, blocks[t], o, &R);
        size_t sz = sizeof(double) * (size_t)(R.n > 0 ? R.n : 1);
        double *lr = (double *)malloc(sz), *ld = (double *)malloc(sz);
        double *lp = (double *)malloc(sz), *lq = (double *)malloc(sz);
        region_residual(&P, &R, beff, x, lr);
        region_inner(&R, inner, lr, ld, lp, lq, m, inner_tol);
        for (long c = 0; c < R.n; c++)
            if (R.own[c]) xout[R.cell[c]] = x[R.cell[c]] + ld[c];
        free(lr); free(ld); free(lp); free(lq);
        region_free(&R);
    }
    return OR_OK;
}
