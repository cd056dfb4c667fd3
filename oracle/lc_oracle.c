/*
 * Link-cell oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial CPU implementation of what the link-cell force sweep
 * and its task-scheduling analysis compute.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load this file's library; the
 * product path never does.  It shares no code with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (see build.py beside it).
 * -ffp-contract=off matters: every floating-point expression below is meant
 * to round after each operation, with no fused multiply-add.
 *
 * Contents
 *   1. canonical coordinates            (reading of Sec. IV: positions in a
 *                                        periodic box, stored as box fractions)
 *   2. Lennard-Jones pair terms, FP64 and canonical FP32 + int64 fixed point
 *   3. forces by brute force O(N^2) and by the serial link-cell method
 *      (Sec. IV: cells of side >= rc, Newton's third law, half stencil of
 *      Fig. 3; every cell-cell interaction updates both cells); the same
 *      sweep in the paper's loop-exchange order with two-strided colouring
 *      (Sec. VI, strategy 1), run with OpenMP: the benchmark's parallel CPU
 *      reference, checked against the serial sweep bit for bit
 *   4. task creation orders of the link-cell traversal: the basic order
 *      (Sec. V: per cell, intra first then inter; cells x, then y, then z)
 *      and the loop-exchanged two-strided coloured order (Sec. VI, strategy 1)
 *   5. the task dependency DAG by the StarSs definition (Sec. III: a task
 *      depends on every earlier task that touches one of its parameters,
 *      unless both only read it) and its critical path (Sec. V, Eq. 1)
 *   6. velocity Verlet in FP64 with fixed-point forces
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TWO32 4294967296.0
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-5)

/* Cell side must exceed rc by this factor so that FP32 rounding of the pair
 * distance can never admit a pair from non-adjacent cells. */
#define CELL_MARGIN (1.0 + 1.0 / 4096.0)

/* ------------------------------------------------------------------------- */
/* 1. canonical coordinates                                                  */
/* ------------------------------------------------------------------------- */

/* u = floor((x * (1/L)) * 2^32) mod 2^32, per axis.  The product with 2^32 is
 * exact, so u depends only on the FP64 rounding of x * (1/L). */
void orc_canonical(int64_t n, const double *pos, const double *L, uint32_t *u)
{
    for (int d = 0; d < 3; ++d) {
        double inv = 1.0 / L[d];
        for (int64_t i = 0; i < n; ++i) {
            double s = pos[d * n + i] * inv;
            double f = floor(s * TWO32);
            u[d * n + i] = (uint32_t)(int64_t)f;
        }
    }
}

/* Cell index of every particle: c_d = floor(u_d * nc_d / 2^32), linear index
 * cx + nx * (cy + ny * cz). */
void orc_cell_ids(int64_t n, const uint32_t *u, const int32_t *nc, int32_t *cid)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d)
            c[d] = (int64_t)(((uint64_t)u[d * n + i] * (uint64_t)nc[d]) >> 32);
        cid[i] = (int32_t)(c[0] + (int64_t)nc[0] * (c[1] + (int64_t)nc[1] * c[2]));
    }
}

/* ------------------------------------------------------------------------- */
/* 2. pair terms                                                             */
/* ------------------------------------------------------------------------- */

/* Parameters of the canonical FP32 pair evaluation. */
typedef struct {
    float s[3];   /* (float)(L_d * 2^-32): box-fraction unit to length */
    float rc2;    /* (float)(rc * rc) */
    float uc;     /* pair energy at the cutoff, same FP32 sequence */
} fx_par;

static void fx_par_init(fx_par *p, const double *L, double rc)
{
    for (int d = 0; d < 3; ++d) p->s[d] = (float)(L[d] / TWO32);
    p->rc2 = (float)(rc * rc);
    float inv = 1.0f / p->rc2;
    float s6 = inv * inv;
    s6 = s6 * inv;
    float e = 4.0f * s6;
    p->uc = e * (s6 - 1.0f);
}

/* Round-to-nearest-even of v * 2^32 to int64.  The product is exact in FP64,
 * nearbyint rounds in the default (nearest-even) mode.  Sets *ovf when the
 * result cannot be held with headroom (|q| >= 2^62). */
static int64_t q32(float v, int *ovf)
{
    double d = (double)v * TWO32;
    if (!(fabs(d) < 4611686018427387904.0)) { *ovf = 1; return 0; }
    return (int64_t)nearbyint(d);
}

/* Canonical FP32 Lennard-Jones pair between particles i and j.
 * d = r_j - r_i from the signed 32-bit difference of box fractions (this is
 * the minimum image), then, rounding after every operation:
 *   r2 = (dx*dx + dy*dy) + dz*dz            in cutoff iff r2 < rc2
 *   inv = 1/r2,  s6 = (inv*inv)*inv
 *   fs = ((24*inv)*s6)*((2*s6) - 1)         f = fs * d is the force on j
 *   e  = ((4*s6)*(s6 - 1)) - uc             shifted pair energy
 *   w  = fs * r2                            pair virial r . f
 * Each of f_x, f_y, f_z, e, w is then quantised to int64 at scale 2^32.
 * Returns 1 when the pair is inside the cutoff. */
static int pair_fx(const uint32_t *u, int64_t n, int64_t i, int64_t j,
                   const fx_par *p, int64_t q[3], int64_t *qe, int64_t *qw,
                   int *ovf)
{
    float dv[3];
    for (int d = 0; d < 3; ++d) {
        int32_t k = (int32_t)(u[d * n + j] - u[d * n + i]);
        dv[d] = (float)k * p->s[d];
    }
    float r2 = dv[0] * dv[0] + dv[1] * dv[1];
    r2 = r2 + dv[2] * dv[2];
    if (!(r2 < p->rc2)) return 0;
    float inv = 1.0f / r2;
    float s6 = inv * inv;
    s6 = s6 * inv;
    float t = 24.0f * inv;
    t = t * s6;
    float g = 2.0f * s6;
    g = g - 1.0f;
    float fs = t * g;
    for (int d = 0; d < 3; ++d) q[d] = q32(fs * dv[d], ovf);
    float e = 4.0f * s6;
    e = e * (s6 - 1.0f);
    e = e - p->uc;
    *qe = q32(e, ovf);
    *qw = q32(fs * r2, ovf);
    return 1;
}

/* FP64 Lennard-Jones pair with the minimum image taken in FP64.
 * When u is non-NULL the cutoff decision is the canonical FP32 one (so the
 * FP64 sum runs over exactly the pair set of the fixed-point path). */
static int pair_f64(const double *pos, const uint32_t *u, int64_t n,
                    int64_t i, int64_t j, const double *L, double rc,
                    const fx_par *p, double f[3], double *e, double *w,
                    double *mag)
{
    double dv[3];
    for (int d = 0; d < 3; ++d) {
        double x = pos[d * n + j] - pos[d * n + i];
        x -= L[d] * nearbyint(x / L[d]);
        dv[d] = x;
    }
    double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    int in;
    if (u) {
        float dq[3];
        for (int d = 0; d < 3; ++d)
            dq[d] = (float)(int32_t)(u[d * n + j] - u[d * n + i]) * p->s[d];
        float r2f = dq[0] * dq[0] + dq[1] * dq[1];
        r2f = r2f + dq[2] * dq[2];
        in = r2f < p->rc2;
    } else {
        in = r2 < rc * rc;
    }
    if (!in) return 0;
    double inv = 1.0 / r2;
    double s6 = inv * inv * inv;
    double fs = 24.0 * inv * s6 * (2.0 * s6 - 1.0);
    double ic = 1.0 / (rc * rc);
    double s6c = ic * ic * ic;
    for (int d = 0; d < 3; ++d) f[d] = fs * dv[d];
    *e = 4.0 * s6 * (s6 - 1.0) - 4.0 * s6c * (s6c - 1.0);
    *w = fs * r2;
    *mag = fabs(fs) * sqrt(r2);
    return 1;
}

/* ------------------------------------------------------------------------- */
/* 3. forces                                                                 */
/* ------------------------------------------------------------------------- */

/* FP64 brute force over all unordered pairs.  F (3 x N) gets the force on
 * every particle, mag (N, may be NULL) gets sum_j |f_ij|, ew[0] = U, ew[1] = W.
 * u may be NULL (FP64 cutoff) or canonical coordinates (FP32 cutoff set). */
int orc_forces_brute_f64(int64_t n, const double *pos, const uint32_t *u,
                         const double *L, double rc, double *F, double *mag,
                         double *ew, int64_t *npairs)
{
    fx_par p;
    fx_par_init(&p, L, rc);
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    if (mag) memset(mag, 0, sizeof(double) * (size_t)n);
    double U = 0.0, W = 0.0;
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double f[3], e, w, m;
            if (!pair_f64(pos, u, n, i, j, L, rc, &p, f, &e, &w, &m)) continue;
            for (int d = 0; d < 3; ++d) {
                F[d * n + i] -= f[d];
                F[d * n + j] += f[d];
            }
            if (mag) { mag[i] += m; mag[j] += m; }
            U += e;
            W += w;
            ++np;
        }
    ew[0] = U;
    ew[1] = W;
    if (npairs) *npairs = np;
    return ORC_OK;
}

/* Fixed-point brute force: canonical FP32 pairs, int64 sums.
 * F (3 x N int64) is the force in units of 2^-32; ew[0], ew[1] are the
 * energy and virial in the same units. */
int orc_forces_brute_fx(int64_t n, const uint32_t *u, const double *L,
                        double rc, int64_t *F, int64_t *ew, int64_t *npairs)
{
    fx_par p;
    fx_par_init(&p, L, rc);
    memset(F, 0, sizeof(int64_t) * 3 * (size_t)n);
    int64_t E = 0, Wv = 0, np = 0;
    int ovf = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            int64_t q[3], qe, qw;
            if (!pair_fx(u, n, i, j, &p, q, &qe, &qw, &ovf)) continue;
            for (int d = 0; d < 3; ++d) {
                F[d * n + i] -= q[d];
                F[d * n + j] += q[d];
            }
            E += qe;
            Wv += qw;
            ++np;
        }
    ew[0] = E;
    ew[1] = Wv;
    if (npairs) *npairs = np;
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* Fixed-point force on m selected particles by brute force over all other
 * particles: F_i = sum over j != i of the force the canonical pair (i, j)
 * puts on i, i.e. -q(i, j).  Swapping i and j negates the box-fraction
 * difference exactly (the int32 difference of a pair inside the cutoff is
 * never -2^31) and round-to-nearest-even is odd, so q(j, i) = -q(i, j) and
 * this equals what any pair orientation of the sweep accumulates.  F is
 * 3 x m; npair (may be NULL) receives the neighbours of each particle. */
int orc_forces_subset_fx(int64_t n, const uint32_t *u, const double *L, double rc,
                         const int64_t *idx, int64_t m, int64_t *F, int64_t *npair)
{
    fx_par p;
    fx_par_init(&p, L, rc);
    int ovf = 0;
    for (int64_t s = 0; s < m; ++s) {
        const int64_t i = idx[s];
        if (i < 0 || i >= n) return ORC_EINVAL;
        int64_t f[3] = {0, 0, 0}, cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            int64_t q[3], qe, qw;
            if (!pair_fx(u, n, i, j, &p, q, &qe, &qw, &ovf)) continue;
            for (int d = 0; d < 3; ++d) f[d] -= q[d];
            ++cnt;
        }
        for (int d = 0; d < 3; ++d) F[d * m + s] = f[d];
        if (npair) npair[s] = cnt;
    }
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* Link-cell grid with linked lists (head of chain per cell, next per
 * particle), the classic formulation of the method. */
typedef struct {
    int32_t nc[3];
    int64_t ncell;
    int64_t *head;
    int64_t *next;
} lc_cells;

static int cells_build(lc_cells *c, int64_t n, const int32_t *cid_of,
                       const int32_t *nc)
{
    for (int d = 0; d < 3; ++d) c->nc[d] = nc[d];
    c->ncell = (int64_t)nc[0] * nc[1] * nc[2];
    c->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)c->ncell);
    c->next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!c->head || !c->next) return ORC_ENOMEM;
    for (int64_t k = 0; k < c->ncell; ++k) c->head[k] = -1;
    /* insert in reverse so each chain lists particles in increasing index */
    for (int64_t i = n - 1; i >= 0; --i) {
        c->next[i] = c->head[cid_of[i]];
        c->head[cid_of[i]] = i;
    }
    return ORC_OK;
}

static void cells_free(lc_cells *c)
{
    free(c->head);
    free(c->next);
}

static int64_t wrapi(int64_t a, int64_t m) { a %= m; return a < 0 ? a + m : a; }

static int check_grid(const double *L, double rc, const int32_t *nc)
{
    for (int d = 0; d < 3; ++d) {
        if (nc[d] < 3) return ORC_EINVAL;  /* fewer cells would repeat pairs */
        if (L[d] / nc[d] < rc * CELL_MARGIN) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* Serial link-cell sweep with Newton's third law.  Cells are visited with x
 * fastest, then y, then z; each cell computes its intra-cell pairs (each
 * unordered pair once) and then one inter-cell interaction per offset of the
 * half stencil `offs` (noff x 3, int8), writing into both cells.  The half
 * stencil must contain exactly one of d and -d for every nonzero d in
 * {-1,0,1}^3.  mode 0: fixed point (u, F as int64); mode 1: FP64 (pos, F as
 * double, cells from u so both modes see the same grid). */
static int lc_sweep(int mode, int64_t n, const double *pos, const uint32_t *u,
                    const double *L, double rc, const int32_t *nc,
                    const int8_t *offs, int noff, void *Fout, void *ewout,
                    int64_t *npairs)
{
    int rcode = check_grid(L, rc, nc);
    if (rcode) return rcode;
    int32_t *cid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!cid) return ORC_ENOMEM;
    orc_cell_ids(n, u, nc, cid);
    lc_cells c;
    rcode = cells_build(&c, n, cid, nc);
    if (rcode) { free(cid); return rcode; }

    fx_par p;
    fx_par_init(&p, L, rc);
    int ovf = 0;
    int64_t *Fq = (int64_t *)Fout;
    double *Fd = (double *)Fout;
    if (mode == 0) memset(Fq, 0, sizeof(int64_t) * 3 * (size_t)n);
    else memset(Fd, 0, sizeof(double) * 3 * (size_t)n);
    int64_t Eq = 0, Wq = 0, np = 0;
    double Ed = 0.0, Wd = 0.0;

#define VISIT(I, J)                                                          \
    do {                                                                     \
        if (mode == 0) {                                                     \
            int64_t q[3], qe, qw;                                            \
            if (pair_fx(u, n, (I), (J), &p, q, &qe, &qw, &ovf)) {            \
                for (int d = 0; d < 3; ++d) {                                \
                    Fq[d * n + (I)] -= q[d];                                 \
                    Fq[d * n + (J)] += q[d];                                 \
                }                                                            \
                Eq += qe; Wq += qw; ++np;                                    \
            }                                                                \
        } else {                                                             \
            double f[3], e, w, m;                                            \
            if (pair_f64(pos, NULL, n, (I), (J), L, rc, &p, f, &e, &w, &m)) { \
                for (int d = 0; d < 3; ++d) {                                \
                    Fd[d * n + (I)] -= f[d];                                 \
                    Fd[d * n + (J)] += f[d];                                 \
                }                                                            \
                Ed += e; Wd += w; ++np;                                      \
            }                                                                \
        }                                                                    \
    } while (0)

    for (int64_t z = 0; z < nc[2]; ++z)
        for (int64_t y = 0; y < nc[1]; ++y)
            for (int64_t x = 0; x < nc[0]; ++x) {
                int64_t a = x + nc[0] * (y + nc[1] * z);
                /* intra-cell interaction */
                for (int64_t i = c.head[a]; i >= 0; i = c.next[i])
                    for (int64_t j = c.next[i]; j >= 0; j = c.next[j])
                        VISIT(i, j);
                /* inter-cell interactions of the half stencil */
                for (int k = 0; k < noff; ++k) {
                    int64_t bx = wrapi(x + offs[3 * k + 0], nc[0]);
                    int64_t by = wrapi(y + offs[3 * k + 1], nc[1]);
                    int64_t bz = wrapi(z + offs[3 * k + 2], nc[2]);
                    int64_t b = bx + nc[0] * (by + nc[1] * bz);
                    for (int64_t i = c.head[a]; i >= 0; i = c.next[i])
                        for (int64_t j = c.head[b]; j >= 0; j = c.next[j])
                            VISIT(i, j);
                }
            }
#undef VISIT
    if (mode == 0) {
        ((int64_t *)ewout)[0] = Eq;
        ((int64_t *)ewout)[1] = Wq;
    } else {
        ((double *)ewout)[0] = Ed;
        ((double *)ewout)[1] = Wd;
    }
    if (npairs) *npairs = np;
    cells_free(&c);
    free(cid);
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

int orc_forces_lc_fx(int64_t n, const uint32_t *u, const double *L, double rc,
                     const int32_t *nc, const int8_t *offs, int noff,
                     int64_t *F, int64_t *ew, int64_t *npairs)
{
    return lc_sweep(0, n, NULL, u, L, rc, nc, offs, noff, F, ew, npairs);
}

int orc_forces_lc_f64(int64_t n, const double *pos, const uint32_t *u,
                      const double *L, double rc, const int32_t *nc,
                      const int8_t *offs, int noff, double *F, double *ew,
                      int64_t *npairs)
{
    return lc_sweep(1, n, pos, u, L, rc, nc, offs, noff, F, ew, npairs);
}

/* The sweep in the loop-exchange order of Sec. VI (strategy 1): for the
 * intra-cell interaction and then every offset of the half stencil, for each
 * of the 8 parity classes of cells (x, y, z each even or odd), the tasks
 * (cell, cell + offset) of that class run in parallel.  With even cell
 * counts two cells of one class differ by an even number of cells along
 * every axis, while a nonzero offset moves one cell along some axis, so no
 * two tasks of one class touch a common cell and the int64 force adds need
 * no atomics.  The pair arithmetic is the serial sweep's, and integer sums do
 * not depend on their order: the result equals orc_forces_lc_fx bit for bit.
 * nthreads <= 0 takes OpenMP's default; *threads_used reports the count. */
int orc_forces_loopex_omp(int64_t n, const uint32_t *u, const double *L, double rc,
                          const int32_t *nc, const int8_t *offs, int noff, int nthreads,
                          int64_t *F, int64_t *ew, int64_t *npairs, int *threads_used)
{
    int rcode = check_grid(L, rc, nc);
    if (rcode) return rcode;
    for (int d = 0; d < 3; ++d)
        if (nc[d] % 2) return ORC_EINVAL;  /* the colouring needs even counts */
    int32_t *cid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!cid) return ORC_ENOMEM;
    orc_cell_ids(n, u, nc, cid);
    lc_cells c;
    rcode = cells_build(&c, n, cid, nc);
    if (rcode) { free(cid); return rcode; }
    fx_par p;
    fx_par_init(&p, L, rc);
    memset(F, 0, sizeof(int64_t) * 3 * (size_t)n);
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    int64_t Eq = 0, Wq = 0, np = 0;
    int ovf = 0, used = 1;
    const int64_t hx = nc[0] / 2, hy = nc[1] / 2, hz = nc[2] / 2;
    for (int k = -1; k < noff; ++k) {  /* k = -1: the intra-cell interaction */
        for (int col = 0; col < 8; ++col) {
            const int64_t cx = col & 1, cy = (col >> 1) & 1, cz = col >> 2;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : Eq, Wq, np) \
    reduction(| : ovf)
            for (int64_t t = 0; t < hx * hy * hz; ++t) {
                if (t == 0) used = omp_get_num_threads();
                const int64_t x = cx + 2 * (t % hx), y = cy + 2 * ((t / hx) % hy),
                              z = cz + 2 * (t / (hx * hy));
                const int64_t a = x + nc[0] * (y + nc[1] * z);
                int64_t b = a;
                if (k >= 0) {
                    const int64_t bx = wrapi(x + offs[3 * k + 0], nc[0]);
                    const int64_t by = wrapi(y + offs[3 * k + 1], nc[1]);
                    const int64_t bz = wrapi(z + offs[3 * k + 2], nc[2]);
                    b = bx + nc[0] * (by + nc[1] * bz);
                }
                for (int64_t i = c.head[a]; i >= 0; i = c.next[i])
                    for (int64_t j = k < 0 ? c.next[i] : c.head[b]; j >= 0; j = c.next[j]) {
                        int64_t q[3], qe, qw;
                        int o = 0;
                        if (pair_fx(u, n, i, j, &p, q, &qe, &qw, &o)) {
                            for (int d = 0; d < 3; ++d) {
                                F[d * n + i] -= q[d];
                                F[d * n + j] += q[d];
                            }
                            Eq += qe; Wq += qw; ++np;
                        }
                        ovf |= o;
                    }
            }
        }
    }
    ew[0] = Eq;
    ew[1] = Wq;
    if (npairs) *npairs = np;
    if (threads_used) *threads_used = used;
    cells_free(&c);
    free(cid);
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* 4. task creation orders                                                   */
/* ------------------------------------------------------------------------- */

/* Cells of a periodic grid dims[0] x dims[1] x dims[2] (2D: dims[2] = 1).
 * `order` lists the stencil in evaluation order, n entries of (dx, dy, dz);
 * (0,0,0) is the intra-cell interaction.
 *
 * loopex == 0: the basic traversal -- for every cell (x fastest, then y,
 *   then z), one task per stencil entry in `order`.
 * loopex == 1: loop exchange with two-strided colouring -- for every stencil
 *   entry in `order`, for every colour (cx, cy, cz) in {0,1}^D with cx
 *   fastest (D = 2 or 3), for every cell of that colour (x fastest).  Needs
 *   even dims along every used axis.
 *
 * A task is the pair (cellA, cellB) = (cell, cell + offset, wrapped).
 * Returns the number of tasks written, or a negative error. */
int orc_lc_tasks(const int32_t *dims, const int8_t *order, int n, int loopex,
                 int32_t *cellA, int32_t *cellB)
{
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    int64_t t = 0;
    if (!loopex) {
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x)
                    for (int k = 0; k < n; ++k) {
                        int64_t bx = wrapi(x + order[3 * k], nx);
                        int64_t by = wrapi(y + order[3 * k + 1], ny);
                        int64_t bz = wrapi(z + order[3 * k + 2], nz);
                        cellA[t] = (int32_t)(x + nx * (y + ny * z));
                        cellB[t] = (int32_t)(bx + nx * (by + ny * bz));
                        ++t;
                    }
        return (int)t;
    }
    int ncz = nz > 1 ? 2 : 1;
    if ((nx % 2) || (ny % 2) || (nz > 1 && (nz % 2))) return ORC_EINVAL;
    for (int k = 0; k < n; ++k)
        for (int cz = 0; cz < ncz; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    for (int64_t z = cz; z < nz; z += (nz > 1 ? 2 : 1))
                        for (int64_t y = cy; y < ny; y += 2)
                            for (int64_t x = cx; x < nx; x += 2) {
                                int64_t bx = wrapi(x + order[3 * k], nx);
                                int64_t by = wrapi(y + order[3 * k + 1], ny);
                                int64_t bz = wrapi(z + order[3 * k + 2], nz);
                                cellA[t] = (int32_t)(x + nx * (y + ny * z));
                                cellB[t] = (int32_t)(bx + nx * (by + ny * bz));
                                ++t;
                            }
    return (int)t;
}

/* ------------------------------------------------------------------------- */
/* 5. dependency DAG and critical path                                       */
/* ------------------------------------------------------------------------- */

/* Parameter access modes, as declared on a StarSs task. */
#define ORC_IN 0
#define ORC_OUT 1
#define ORC_INOUT 2

/* Task t has parameters addr[pstart[t] .. pstart[t+1]) with modes `mode`.
 * By the StarSs rule, t depends on every earlier task s with which it shares
 * an address that at least one of the two writes (read-after-write,
 * write-after-read, write-after-write).  With unit task durations the
 * earliest finishing step of t is depth[t] = 1 + max(depth[s]) over those s;
 * the critical path is max depth.  Written as the definition reads: every
 * earlier task is examined, O(T^2 P^2).  pred (may be NULL) receives, per
 * task, one predecessor attaining the max depth (-1 if none) -- the
 * "simplified DAG" edges. */
int orc_dag_generic(int T, const int32_t *pstart, const int64_t *addr,
                    const int32_t *mode, int32_t *depth, int32_t *pred,
                    int32_t *cp)
{
    int32_t best = 0;
    for (int t = 0; t < T; ++t) {
        int32_t dmax = 0, arg = -1;
        for (int s = 0; s < t; ++s) {
            int dep = 0;
            for (int a = pstart[t]; a < pstart[t + 1] && !dep; ++a)
                for (int b = pstart[s]; b < pstart[s + 1]; ++b)
                    if (addr[a] == addr[b] &&
                        (mode[a] != ORC_IN || mode[b] != ORC_IN)) {
                        dep = 1;
                        break;
                    }
            if (dep && depth[s] >= dmax) {
                /* ties go to the latest such task */
                dmax = depth[s];
                arg = s;
            }
        }
        depth[t] = dmax + 1;
        if (pred) pred[t] = arg;
        if (depth[t] > best) best = depth[t];
    }
    *cp = best;
    return ORC_OK;
}

/* The same definition specialised to link-cell tasks: both cells of a task
 * are inout (Sec. IV), an intra-cell task has its single cell.  Still
 * examines every earlier task. */
int orc_dag_lc(int T, const int32_t *cellA, const int32_t *cellB,
               int32_t *depth, int32_t *cp)
{
    int32_t best = 0;
    for (int t = 0; t < T; ++t) {
        int32_t dmax = 0;
        for (int s = 0; s < t; ++s) {
            int share = cellA[s] == cellA[t] || cellA[s] == cellB[t] ||
                        cellB[s] == cellA[t] || cellB[s] == cellB[t];
            if (share && depth[s] > dmax) dmax = depth[s];
        }
        depth[t] = dmax + 1;
        if (depth[t] > best) best = depth[t];
    }
    *cp = best;
    return ORC_OK;
}

/* Weighted critical path by the same definition: task t can finish no
 * earlier than w[t] after every earlier task sharing a cell has finished;
 * returns the largest finish time in *cp. */
int orc_dag_lc_weighted(int T, const int32_t *cellA, const int32_t *cellB,
                        const double *w, double *finish, double *cp)
{
    double best = 0.0;
    for (int t = 0; t < T; ++t) {
        double start = 0.0;
        for (int s = 0; s < t; ++s) {
            int share = cellA[s] == cellA[t] || cellA[s] == cellB[t] ||
                        cellB[s] == cellA[t] || cellB[s] == cellB[t];
            if (share && finish[s] > start) start = finish[s];
        }
        finish[t] = start + w[t];
        if (finish[t] > best) best = finish[t];
    }
    *cp = best;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* 6. velocity Verlet                                                        */
/* ------------------------------------------------------------------------- */

/* Kinetic energy in units of 2^-32: sum over particles of the int64 rounding
 * of ((vx*vx + vy*vy) + vz*vz) * 0.5 * 2^32. */
static int64_t ke_fx(int64_t n, const double *v)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        double s = v[i] * v[i] + v[n + i] * v[n + i];
        s = s + v[2 * n + i] * v[2 * n + i];
        k += (int64_t)nearbyint((s * 0.5) * TWO32);
    }
    return k;
}

/* Kick-drift-kick velocity Verlet, unit mass, FP64 state, fixed-point
 * forces from the serial link-cell sweep (cells rebuilt every step; the
 * pair set does not depend on the grid).  For each step:
 *   a = F * 2^-32;  v = v + (0.5*dt)*a;  x = x + dt*v;
 *   recompute F at x;  a = F * 2^-32;  v = v + (0.5*dt)*a.
 * trace (nsteps+1) x 2 holds [KE, PE] in units of 2^-32 after every step
 * (row 0: initial state).  pos and vel (3 x N) are updated in place; F
 * (3 x N int64) holds the final forces. */
int orc_verlet_fx(int64_t n, double *pos, double *vel, const double *L,
                  double rc, const int32_t *nc, const int8_t *offs, int noff,
                  double dt, int nsteps, int64_t *F, int64_t *trace)
{
    uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)(n > 0 ? n : 1));
    if (!u) return ORC_ENOMEM;
    int64_t ew[2];
    orc_canonical(n, pos, L, u);
    int rcode = orc_forces_lc_fx(n, u, L, rc, nc, offs, noff, F, ew, NULL);
    if (rcode) { free(u); return rcode; }
    trace[0] = ke_fx(n, vel);
    trace[1] = ew[0];
    double hdt = 0.5 * dt;
    for (int s = 1; s <= nsteps; ++s) {
        for (int64_t k = 0; k < 3 * n; ++k) {
            double a = (double)F[k] * (1.0 / TWO32);
            vel[k] = vel[k] + hdt * a;
            pos[k] = pos[k] + dt * vel[k];
        }
        orc_canonical(n, pos, L, u);
        rcode = orc_forces_lc_fx(n, u, L, rc, nc, offs, noff, F, ew, NULL);
        if (rcode) { free(u); return rcode; }
        for (int64_t k = 0; k < 3 * n; ++k) {
            double a = (double)F[k] * (1.0 / TWO32);
            vel[k] = vel[k] + hdt * a;
        }
        trace[2 * s] = ke_fx(n, vel);
        trace[2 * s + 1] = ew[0];
    }
    free(u);
    return ORC_OK;
}
