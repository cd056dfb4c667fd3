/*
 * lc.h -- C-ABI of the MI355X link-cell force sweep with conflict-free cell
 * schedules.
 *
 * The method (Niethammer, Glass, Gracia, "Avoiding Serialization Effects in
 * Data / Dependency aware Task Parallel Algorithms for Spatial
 * Decomposition"):
 *   - Sec. IV: link-cell (LC) method -- the periodic box is cut into cells of
 *     side >= rc; with Newton's third law every pair is evaluated once and
 *     both particles are updated, so a cell only visits the half stencil of
 *     Fig. 3 (13 neighbour cells in 3D) plus itself.  One task = one
 *     cell-cell interaction, and it writes into BOTH cells.
 *   - Sec. V: because tasks that write a common cell are serialised, the
 *     ORDER in which tasks are created fixes the critical path of the task
 *     DAG and hence the attainable speedup S = t_s / t_cp (Eq. 1), modelled by
 *     S(Delta, k, n) = n k / (n + Delta (k - 1)) (Eq. 2, 3, 4).
 *   - Sec. VI: remedies -- loop exchange with two-strided colouring
 *     (strategy 1), nested tasks (2), buffer + reduce (3).
 *
 * Conventions
 *   - Every function returns an int status: LC_OK (0) or a negative LC_E*
 *     code; lc_last_error() gives a thread-local message for the last error.
 *     No C++ exception crosses this boundary.
 *   - Device pointers (marked [device]) are caller-owned HIP device memory;
 *     the library never frees them.  Host pointers are marked [host].
 *     Opaque handles (lc_schedule, lc_workspace) are created and destroyed by
 *     the library and belong to the device that was current at creation.
 *   - Particle arrays are SoA "3 x N": all x, then all y, then all z, each
 *     row N elements long and contiguous.
 *   - Device work is enqueued asynchronously on `stream` (a hipStream_t,
 *     NULL = the null stream); no call below synchronises unless it says so.
 *   - Fixed point: forces, energies and virials are int64 in units of 2^-32
 *     (multiply by 2^-32 to get reduced LJ units).  Integer sums commute, so
 *     every schedule yields the same bits.
 *
 * Canonical pair arithmetic (the definition the GPU and any checker share):
 *   box fraction   u_d = floor((x_d * (1/L_d)) * 2^32) mod 2^32   (FP64)
 *   separation     d_d = (float)(int32)(u_d[j] - u_d[i]) * s_d,
 *                  s_d = (float)(L_d * 2^-32)   -- minimum image for free
 *   then in FP32, rounding after every operation (no FMA):
 *     r2 = (dx*dx + dy*dy) + dz*dz;   pair used iff r2 < (float)(rc*rc)
 *     inv = 1/r2 (correctly rounded); s6 = (inv*inv)*inv
 *     fs = ((24*inv)*s6)*((2*s6) - 1);    force on j = +fs*d, on i = -fs*d
 *     e  = ((4*s6)*(s6 - 1)) - e_c        (e_c: same sequence at r2 = rc2)
 *     w  = fs*r2
 *   each of fs*d_x, fs*d_y, fs*d_z, e, w rounded to nearest-even int64 at
 *   scale 2^32.
 */
#ifndef LC_H
#define LC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LC_OK 0
#define LC_EINVAL (-1)    /* bad argument (sizes, null pointers, grid)      */
#define LC_ENOMEM (-2)    /* host or device allocation failed               */
#define LC_EHIP (-3)      /* a HIP runtime call failed                      */
#define LC_ESCHED (-4)    /* schedule validator: a phase has shared writes  */
#define LC_EOVERFLOW (-5) /* fixed-point range exceeded (device flag)       */
#define LC_EDISP (-6)     /* a particle moved more than skin/2 (device flag)*/
#define LC_ECAPACITY (-7) /* a size exceeds a documented maximum            */
#define LC_EABORT (-8)    /* a dataflow evaluation was abandoned (flag)     */

/* Device status flags (lc_workspace_status). */
#define LC_FLAG_OVERFLOW 1u  /* |quantised term| >= 2^62 or r2 == 0          */
#define LC_FLAG_DISP 2u      /* displacement since rebuild > skin / 2        */
#define LC_FLAG_FALLBACK 4u  /* a cell group exceeded the LDS tile and ran
                                through the global-memory path (info only)   */
#define LC_FLAG_ABORT 8u     /* a dataflow wait exceeded its time limit: the
                                evaluation was abandoned, forces incomplete  */

/* Last error message of the calling thread (never NULL). */
const char *lc_last_error(void);

/* ---- grid --------------------------------------------------------------- */

#define LC_GRID_EVEN 1 /* round the cell count per axis down to even       */
#define LC_GRID_HALF 2 /* cells of side >= (rc + skin) / 2: the stencil
                          reaches 2 cells (Sec. IV takes side >= rc; the
                          half-size cells visit fewer candidate pairs)       */
#define LC_GRID_2D 4   /* a flat system: one cell along z (every particle
                          at the same z); schedules use the 2D stencil of
                          Fig. 3a and the 2D orders of Fig. 5               */

/* Periodic cell grid (Sec. IV: cells of side >= rc).  Filled by
 * lc_make_grid; plain data, may be copied. */
typedef struct lc_grid {
    double box[3];     /* edge lengths L_d                                  */
    double inv_box[3]; /* 1 / L_d                                           */
    double rc;         /* cutoff radius                                     */
    double skin;       /* extra cell width for delayed rebuilds             */
    int32_t nc[3];     /* cells per axis, each >= 3                         */
    int32_t ncell;     /* nc[0] * nc[1] * nc[2]                             */
    float scale[3];    /* (float)(L_d * 2^-32)                              */
    float rc2;         /* (float)(rc * rc)                                  */
    float ecut;        /* canonical pair energy at r2 = rc2                 */
    int32_t reach;     /* stencil reach in cells: 1, or 2 with LC_GRID_HALF  */
} lc_grid;

/* [host] nc_d = floor(L_d / (rc * (1 + 2^-12) + skin)), the largest count
 * whose cell side covers rc plus the skin with a margin that FP32 rounding of
 * r2 cannot cross; with LC_GRID_HALF, floor(2 L_d / (...)) (two cells cover
 * it, reach 2).  flags: LC_GRID_EVEN | LC_GRID_HALF.  Returns LC_EINVAL when
 * an axis gets fewer than 2 reach + 1 cells (pairs would be visited twice) or
 * ncell >= 2^31.  With LC_GRID_2D the z axis keeps one cell (box[2] only has
 * to be positive; the particles must share one z) and the x, y rules apply;
 * it cannot be combined with LC_GRID_HALF.  Schedules and sweeps follow the grid's reach; at reach 2
 * there is no LC_SCHED_BLOCK8 (LC_SCHED_LOOPEX colours with stride 3 and
 * needs cell counts divisible by 3), the presets OPT/BEST/BAD are not defined
 * (pass the order as LC_SCHED_CUSTOM offsets in [-2, 2]), and batches take
 * reach-1 3D grids only (no LC_GRID_HALF, no LC_GRID_2D). */
int lc_make_grid(const double box[3], double rc, double skin, int flags,
                 lc_grid *out);

/* ---- workspace ---------------------------------------------------------- */

typedef struct lc_workspace lc_workspace;

/* [host] Device scratch for up to max_n particles and max_cells cells
 * (cell ids, per-cell counters, scan partials, status flags, Verlet
 * reference positions and staging).  Allocates with hipMalloc on the
 * current device and clears it (synchronises the device).  A workspace
 * serves one stream at a time: the cell build keeps its per-cell counters
 * cleared between calls instead of clearing them at the start of each. */
int lc_workspace_create(int64_t max_n, int64_t max_cells, lc_workspace **out);
void lc_workspace_destroy(lc_workspace *ws);

/* LDS tile sizing hint: the largest number of particles in one cell (0 =
 * estimate from the mean density).  A work-group stages its footprint cells
 * in LDS when they fit the tile and otherwise runs the (exact but slower)
 * global-memory path, flagged with LC_FLAG_FALLBACK.  The hint also picks the
 * kernel: the 16-bit candidate filter stages cells of up to 60 particles, so
 * a larger hint (or, without one, a mean above 30) selects the unfiltered
 * sweep. */
int lc_workspace_set_tile_hint(lc_workspace *ws, int32_t max_per_cell);

/* Clear the device status flags (async on stream).  It also re-zeroes the
 * workspace's energy partial slots, cell counters and scan status words,
 * which every call otherwise leaves zero for the next (a call that failed
 * part-way may not have). */
int lc_workspace_clear_status(lc_workspace *ws, void *stream);
/* Synchronise `stream` and return the device status flags (LC_FLAG_*). */
int lc_workspace_status(lc_workspace *ws, void *stream, uint32_t *flags);
/* Synchronise `stream` and turn the status flags into a status: LC_EOVERFLOW
 * when a pair term left the fixed-point range (forces wrong), else LC_EABORT
 * when a dataflow evaluation was abandoned (forces incomplete), else LC_EDISP
 * when a Verlet run moved a particle more than skin / 2 between rebuilds
 * (pairs may have been missed since), else LC_OK (LC_FLAG_FALLBACK is
 * information only).  The flags stay set until lc_workspace_clear_status.
 * Device calls return before their kernels run, so this is where the three
 * device-side failures surface as status codes. */
int lc_workspace_check(lc_workspace *ws, void *stream);

/* ---- a1: cell build (Sec. IV) ------------------------------------------- */

/* Counting sort of N particles into the cells of g.
 *   pos      [device] double 3 x N, any real coordinates (wrapped here)
 *   cell_start [device] int32 ncell + 1: particles of cell c are sorted
 *            slots cell_start[c] .. cell_start[c+1]-1 (cells x fastest)
 *   perm     [device] int32 N: sorted slot k holds input particle perm[k]
 *   coord    [device] uint32 3 x N: box fractions u of the sorted particles
 * Order inside a cell is unspecified (atomic ranks); forces do not depend on
 * it.  Needs a workspace created with max_n >= N, max_cells >= ncell. */
int lc_build_cells(const lc_grid *g, const double *pos, int64_t n,
                   int32_t *cell_start, int32_t *perm, uint32_t *coord,
                   lc_workspace *ws, void *stream);

/* Gather rows of a double 3 x N array (and an optional int32 N array) by
 * perm: out[:, k] = in[:, perm[k]].  [device] buffers, in != out. */
int lc_gather(const int32_t *perm, int64_t n, const double *in3, double *out3,
              const int32_t *in_ids, int32_t *out_ids, void *stream);

/* ---- a2: schedules (Sec. V, Sec. VI strategy 1) ------------------------- */

/* Creation orders / execution strategies. */
#define LC_SCHED_LEX 0          /* basic order: per cell (x, y, z fastest to
                                   slowest) intra then the 13 offsets in
                                   ascending (dz, dy, dx); run as the levels
                                   of its task DAG                          */
#define LC_SCHED_OPT 1          /* x neighbour first, intra last (Delta = 1)*/
#define LC_SCHED_BEST 2         /* intra, x neighbour, rest (Delta = 2)     */
#define LC_SCHED_BAD 3          /* intra first, x neighbour last (Delta=14) */
#define LC_SCHED_LOOPEX 4       /* loop exchange + 2-strided colouring
                                   (offset-major, 2x2x2 colours; needs even
                                   cell counts); run as DAG levels (27)     */
#define LC_SCHED_BLOCK8 5       /* 2x2x2-coloured blocks of cells: 8
                                   conflict-free phases, one work-group per
                                   block, LDS accumulation, plain read-
                                   modify-write.  A task joins the block of
                                   its lower corner cell (per axis the
                                   smaller coordinate of its two cells), so
                                   a block's footprint is the block grown by
                                   the stencil's reach towards +x, +y, +z */
#define LC_SCHED_ATOMIC_TILE 6  /* BLOCK8's groups in ONE phase with global
                                   int64 atomic write-back                  */
#define LC_SCHED_ATOMIC_PAIR 7  /* one phase, one group per home cell, every
                                   pair adds into both particles with global
                                   int64 atomics (the plain atomics baseline)*/
#define LC_SCHED_CUSTOM 8       /* basic order with a caller-given stencil
                                   order (offsets argument)                 */
#define LC_SCHED_BUFFER 9       /* Sec. VI strategy 3, buffer + reduce:
                                   BLOCK8's groups in ONE phase; each group
                                   stores its footprint sums (plain stores)
                                   into its own replica slot of a partial
                                   buffer, then a gather kernel sums the
                                   replicas of every particle.  No colours,
                                   no atomics; R_max x 24 B per particle of
                                   workspace memory (grown on first use)    */
#define LC_SCHED_FULLSHELL 10   /* comparison baseline without Newton's third
                                   law: each home cell with all 27 cells of
                                   its full shell, forces kept on the home
                                   side only (every pair evaluated twice);
                                   blocks of home cells in ONE phase, plain
                                   stores, no colours, no atomics, no
                                   replicas.  Forces are bit-identical to the
                                   Newton-3 kinds (the reversed pair negates
                                   the separation exactly)                  */
#define LC_SCHED_COUNT 11

typedef struct lc_schedule lc_schedule;

typedef struct lc_schedule_info {
    int32_t kind;
    int32_t nphase;   /* kernel launches per force evaluation               */
    int64_t ntask;    /* cell-cell interactions (14 per cell)               */
    int64_t ngroup;   /* work-groups over all phases                        */
    int32_t max_group_tasks;
    int32_t max_group_cells;
    int32_t write_mode; /* 0 plain RMW, 1 atomic tile, 2 atomic per pair,
                           3 replica buffer + gather                        */
    int32_t max_replicas; /* LC_SCHED_BUFFER: replica slots per particle   */
} lc_schedule_info;

/* [host] Build the task list of `kind` for grid g, split it into phases
 * whose work-groups write disjoint cells (validated: LC_ESCHED otherwise),
 * and upload it to the current device.  offsets/n: for LC_SCHED_CUSTOM the
 * stencil order (n x 3 int8, (0,0,0) = intra, the other n-1 entries one of
 * d / -d for every neighbour d); ignored (may be NULL) for other kinds. */
int lc_make_schedule(const lc_grid *g, int kind, const int8_t *offsets, int n,
                     lc_schedule **out);
/* As lc_make_schedule, with the block shape of the block kinds: block_min
 * [host] 3 x int32, the largest block per axis (>= 1, <= 64).  The
 * uncoloured kinds (LC_SCHED_ATOMIC_TILE / BUFFER / FULLSHELL) cut each axis
 * into ceil(n / size) near-equal blocks.  LC_SCHED_BLOCK8 rounds that count
 * up to even (the 2-colouring), then down by twos while a block would be
 * narrower than the stencil's reach (1; 2 on grids of cells of side rc/2):
 * a footprint reaches that far past its block towards +x, +y and +z, so
 * same-coloured blocks stay a whole block apart.  NULL = the BLOCK8
 * partition with at most {1, 3, 3} for all three ({2, 2, 2} for BLOCK8 and
 * {1, 2, 2} for the uncoloured kinds on rc/2 grids).  Larger blocks mean
 * fewer, bigger work-groups and less halo write-back per particle; smaller
 * ones fit denser boxes into the LDS tile.  A work-group holds at most 512
 * tasks and 128 footprint cells (LC_ECAPACITY otherwise).  The autotuner
 * picks the shape. */
int lc_make_schedule_ex(const lc_grid *g, int kind, const int8_t *offsets,
                        int n, const int32_t *block_min, lc_schedule **out);
int lc_schedule_info_get(const lc_schedule *s, lc_schedule_info *out);
/* [host] The tasks of a creation-order schedule (LEX, OPT, BEST, BAD,
 * CUSTOM, LOOPEX) in creation order, the order the dataflow executors take
 * them: cells A[t], B[t] (host int32 arrays of cap >= T entries); *ntask =
 * T.  LC_EINVAL for the other kinds, LC_ECAPACITY (with *ntask set) when
 * cap < T. */
int lc_schedule_tasks(const lc_schedule *s, int32_t *A, int32_t *B, int64_t cap,
                      int64_t *ntask);
/* [host] For every cell, the number of work-group footprints (over all
 * phases) that hold it: the replica slots its particles get under
 * LC_SCHED_BUFFER, the write-backs they get under the tiled kinds.  count
 * [host] int32 of cap >= ncell entries (x fastest). */
int lc_schedule_cell_footprints(const lc_schedule *s, int32_t *count, int64_t cap);
void lc_schedule_free(lc_schedule *s);

/* Load-aware variant of lc_make_schedule_ex (the weighted tasks of the
 * paper's equal-duration assumption, Sec. V, relaxed): the work-groups of
 * every phase are launched in decreasing order of estimated work -- the sum
 * over a group's tasks of n_A n_B (n_A (n_A - 1) / 2 for an intra task) --
 * so heavy groups start first and a launch ends on light ones.  cell_counts
 * [host] int32 per cell (e.g. the differences of cell_start); LC_EINVAL if
 * NULL or negative.  The schedule stays valid for any later particle
 * distribution; only its launch order, and the LDS tile (sized to hold its
 * largest footprint under these counts; a work-group whose footprint
 * outgrows it later takes the exact global-memory path and sets
 * LC_FLAG_FALLBACK), were chosen for this one. */
int lc_make_schedule_weighted(const lc_grid *g, int kind, const int8_t *offsets,
                              int n, const int32_t *block_min,
                              const int32_t *cell_counts, lc_schedule **out);

/* [host] The estimated work of every work-group of s in launch order, as
 * lc_make_schedule_weighted orders it: work [host] double, one per group
 * (lc_schedule_info.ngroup). */
int lc_schedule_group_work(const lc_schedule *s, const int32_t *cell_counts,
                           double *work);

/* [host only] Build and validate the schedule of `kind` like
 * lc_make_schedule, without touching a device; fills *out. */
int lc_schedule_plan(const lc_grid *g, int kind, const int8_t *offsets, int n,
                     lc_schedule_info *out);
/* [host only] As lc_schedule_plan, with the block shape of
 * lc_make_schedule_ex (NULL = default). */
int lc_schedule_plan_ex(const lc_grid *g, int kind, const int8_t *offsets, int n,
                        const int32_t *block_min, lc_schedule_info *out);

/* [host only] The tasks of the schedule lc_schedule_plan_ex builds, in
 * launch order: task t couples cells A[t] and B[t] (A == B for an intra
 * task), runs in work-group grp[t] (groups numbered in launch order over
 * all phases) and phase phase[t].  A, B, grp, phase: host int32 arrays of
 * cap >= T entries, each may be NULL to skip it; *ntask = T (set also when
 * cap < T, which returns LC_ECAPACITY).  Lets a caller check a schedule
 * without a device: that every stencil pair is kept once, what each work-
 * group's footprint is, and that a phase's groups touch disjoint cells. */
int lc_schedule_plan_tasks(const lc_grid *g, int kind, const int8_t *offsets, int n,
                           const int32_t *block_min, int32_t *A, int32_t *B, int32_t *grp,
                           int32_t *phase, int64_t cap, int64_t *ntask);

/* [host only] The schedule validator on an explicit phase list: phase p runs
 * work-groups phase_grp[p] .. phase_grp[p+1]-1, group k writes the cells
 * foot_cells[grp_foot[k] .. grp_foot[k+1]-1].  Returns LC_OK when every
 * phase's groups write pairwise disjoint cells (so plain read-modify-write
 * is race-free), LC_ESCHED otherwise, LC_EINVAL on malformed input. */
int lc_validate_phases(int64_t ncell, int32_t nphase, const int32_t *phase_grp,
                       const int32_t *grp_foot, const int32_t *foot_cells);

/* ---- a3: serialisation degree (Sec. V, Eq. 1-4) ------------------------- */

typedef struct lc_sd_result {
    int64_t tasks;    /* T                                                  */
    int64_t cp;       /* critical path, in tasks (unit durations)           */
    double speedup;   /* S = T / cp  (Eq. 1)                                */
    double degree;    /* cp / T, 1 = fully serial                           */
    int32_t n;        /* tasks per stencil                                  */
    int32_t delta;    /* stencil displacement Delta (0 for LC_SCHED_LOOPEX:
                         no stencil displacement chains the cells)          */
    double s_eq2;     /* Eq. 2 with k = number of cells (k itself when
                         Delta = 0)                                         */
    double s_max;     /* Eq. 3: n / Delta (+infinity when Delta = 0)        */
} lc_sd_result;

/* [host only] Critical path of the task DAG of a creation order under the
 * StarSs inout rule (consecutive tasks touching a cell are dependent).
 *   dims  cells per axis; dims[2] == 1 selects the 2D stencil of Fig. 3(a)
 *   kind  LC_SCHED_LEX/OPT/BEST/BAD/LOOPEX/CUSTOM (2D presets: Fig. 5 naive,
 *         optimal, best basic, bad)
 *   level_hist [host, optional] int64 array of length hist_len: tasks per
 *         DAG level (level l at index l-1); entries beyond cp are zeroed.
 * O(T) time (last-writer recurrence). */
int lc_serialization_degree(const int32_t dims[3], int kind,
                            const int8_t *offsets, int n, int64_t *level_hist,
                            int64_t hist_len, lc_sd_result *out);

/* [host only] Weighted critical path (relaxes the equal-duration assumption
 * of Sec. V): task (A, B) lasts n_A * n_B, an intra task n_A (n_A - 1) / 2,
 * with cell_counts [host] int32 per cell (x fastest, as lc_build_cells
 * orders cells).  Same creation orders as lc_serialization_degree.
 * work = sum of durations, cp = weighted longest path, S = work / cp. */
typedef struct lc_wsd_result {
    int64_t tasks;
    double work;
    double cp;
    double speedup;
} lc_wsd_result;
int lc_serialization_degree_weighted(const int32_t dims[3], int kind,
                                     const int8_t *offsets, int n,
                                     const int32_t *cell_counts,
                                     lc_wsd_result *out);

/* ---- a4-a6: force sweep ------------------------------------------------- */

#define LC_PREC_FP32 0 /* canonical FP32 pair arithmetic (bit-exact)        */
#define LC_PREC_FP64 1 /* FP64 pair arithmetic from the same box fractions,
                          same pair set (the FP32 cutoff test), same int64
                          quantisation -- a precision reference             */

/* One Lennard-Jones force evaluation over all cell-cell tasks of s, phase by
 * phase: the link-cell sweep of Sec. IV, where each task is one cell-cell
 * interaction of the half stencil (Fig. 3) that, with Newton's third law,
 * adds every pair's force into both of its cells.  Inputs come from
 * lc_build_cells on the same grid:
 *   cell_start [device] int32 ncell+1;  coord [device] uint32 3 x N
 *   F   [device] int64 3 x N, cell-sorted order, OVERWRITTEN with the force
 *   ew  [device] int64 [3]: OVERWRITTEN with {energy, virial, pairs in
 *       cutoff} (energy/virial in units of 2^-32)
 * Status flags (overflow, fallback) accumulate in ws.  LC_SCHED_BUFFER
 * keeps its partial buffer in ws; the first call (or a larger N) allocates
 * it with hipMalloc, later calls do not allocate. */
int lc_compute_forces(const lc_grid *g, const lc_schedule *s,
                      const int32_t *cell_start, const uint32_t *coord,
                      int64_t n, int64_t *F, int64_t *ew, int precision,
                      lc_workspace *ws, void *stream);

/* Profiling variant of lc_compute_forces: the same launches, each sweep
 * phase and the closing launch (the gather of LC_SCHED_BUFFER, else the
 * energy sums) bracketed by HIP events on `stream`; synchronises and returns
 * the summed device time of the sweep kernels in *sweep_ms (the zero-fill of
 * F and ew is not included) and, if phase_ms is not NULL, the time of each
 * phase followed by that of the closing launch (host array of nphase + 1
 * doubles). */
int lc_compute_forces_profiled(const lc_grid *g, const lc_schedule *s,
                               const int32_t *cell_start, const uint32_t *coord,
                               int64_t n, int64_t *F, int64_t *ew, int precision,
                               lc_workspace *ws, void *stream, double *sweep_ms,
                               double *phase_ms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * force evaluation as lc_compute_forces, with no workspace.  Its scratch --
 * the energy slots, a status word and the replica buffer of LC_SCHED_BUFFER
 * -- is a file-scope device array of LC_NOALLOC_SCRATCH_BYTES that every
 * device the library runs on holds until the process ends.  The call makes
 * no hipMalloc, hipFree or other allocating call.
 *   arguments as lc_compute_forces;
 *   flags [device, optional] uint32: status bits (LC_FLAG_*) are OR-ed into
 *         it (the caller clears it); NULL: the bits go to the scratch and are
 *         not reported;
 *   the LDS tile is sized from the mean density (no tile hint).
 * LC_ECAPACITY, before anything is enqueued, when LC_SCHED_BUFFER's replica
 * buffer (max_replicas x 24 B + 4 B per particle) exceeds the scratch (about
 * 2.6 M particles at 8 replicas).  All calls on one device share the one
 * array and each clears what it needs on `stream` first: calls that overlap
 * on one device (other streams, other threads) race and give wrong results;
 * serialise them. */
#define LC_NOALLOC_SCRATCH_BYTES (64ll << 20)
int lc_compute_forces_noalloc(const lc_grid *g, const lc_schedule *s,
                              const int32_t *cell_start, const uint32_t *coord, int64_t n,
                              int64_t *F, int64_t *ew, int precision, uint32_t *flags,
                              void *stream);

/* Self-check of the sweep's fast reciprocal (the FP32 pair arithmetic takes
 * 1/r^2 as the IEEE quotient; pairs with 0.3 <= r^2 < 128 get it from the
 * hardware estimate plus one Newton-Raphson step).  Compares that device
 * routine with IEEE division on every float whose bit pattern lies in
 * [lo_bits, hi_bits) and writes the number of differing results to
 * *mismatches (host).  Synchronous; allocates 8 bytes of device memory for
 * the count.  The range the sweep relies on is [0x3e800000, 0x43000000),
 * i.e. [0.25, 128). */
int lc_selftest_recip(uint32_t lo_bits, uint32_t hi_bits, uint64_t *mismatches);

/* ---- Sec. VI strategy 2 and the mutual exclusion of Sec. VII: dataflow
 * execution of a creation order on the device -------------------------- */
#define LC_DF_ORDERED 0 /* the StarSs inout dependences of the creation order:
                           a task starts once every earlier task on either of
                           its cells has finished (per-cell sequence
                           counters); the run follows the order's critical
                           path without one launch per DAG level          */
#define LC_DF_MUTEX 1   /* the tasks in creation order under mutual exclusion
                           on the two cells they write (the clause Sec. VII
                           asks for): no order between them, no two at once
                           on one cell                                     */
#define LC_DF_NESTED 2  /* Sec. VI strategy 2: per cell one chain, intra
                           then the stencil neighbours in order, each chain
                           started as soon as a runner is free; the writes
                           of concurrent chains are kept apart by the same
                           per-cell mutual exclusion (not for LOOPEX)      */
/* One force evaluation by the dataflow executor `mode` (LC_DF_*) over the
 * tasks of schedule s, which must be a creation-order kind (LEX, OPT, BEST,
 * BAD, CUSTOM, LOOPEX).  One persistent launch of single-wave task runners
 * takes work units (a task, or a chain for NESTED) in creation order; each
 * waits for its cells (counters or locks, lower cell first), evaluates the
 * cell pair with the canonical pair arithmetic and adds into F directly.
 * Results are bit-identical to lc_compute_forces.  Every wait is bounded by
 * limit_ms of wall time: on expiry the evaluation is abandoned (all runners
 * stop, LC_FLAG_ABORT is set, F is incomplete) instead of hanging.  Cells may
 * hold at most 256 particles (LC_ECAPACITY when the workspace's tile hint
 * says more).  Arguments otherwise as lc_compute_forces (FP32 pair math). */
int lc_compute_forces_dataflow(const lc_grid *g, const lc_schedule *s, int mode,
                               const int32_t *cell_start, const uint32_t *coord, int64_t n,
                               int64_t *F, int64_t *ew, double limit_ms, lc_workspace *ws,
                               void *stream);
/* lc_compute_forces_dataflow with an execution log, so that a checker can
 * verify the strategy's constraint (Sec. VI strategy 2; the mutual exclusion
 * of Sec. VII) from what the device did.  log [device] int32 2 x T (T = the
 * schedule's task count): log[t] receives task t's start ticket, taken once
 * its cells were granted and before any of its work, log[T + t] its end
 * ticket, taken after all of its force adds have completed and before its
 * cells are released; both come from one device counter (0, 1, 2, ... in the
 * order the runners reach those points).  Hence ordered: start[t] >
 * end[t'] for every earlier task t' sharing a cell with t; mutex and nested:
 * the [start, end] intervals of tasks sharing a cell are disjoint; nested:
 * a chain's tasks run one after another.  Entries of tasks an abandoned
 * evaluation never ran are left as they were. */
int lc_compute_forces_dataflow_log(const lc_grid *g, const lc_schedule *s, int mode,
                                   const int32_t *cell_start, const uint32_t *coord, int64_t n,
                                   int64_t *F, int64_t *ew, double limit_ms, int32_t *log,
                                   lc_workspace *ws, void *stream);

/* ---- a7: velocity Verlet ------------------------------------------------ */

/* nsteps kick-drift-kick steps (unit mass) on a cell-sorted state:
 *   pos, vel [device] double 3 x N; ids [device] int32 N (particle identity,
 *   permuted along at every rebuild, may be NULL); F [device] int64 3 x N;
 *   cell_start [device] int32 ncell+1, perm [device] int32 N, coord
 *   [device] uint32 3 x N as in lc_build_cells.
 * Step: a = F*2^-32; v = v + (0.5 dt)*a; x = x + dt*v; every rebuild_every
 * steps rebuild cells and reorder pos/vel/ids; F = forces(x);
 * v = v + (0.5 dt)*a.  trace receives {KE, PE} in
 * units of 2^-32, KE = sum_i rint(0.5*((vx^2+vy^2)+vz^2)
 * * 2^32).  A displacement beyond skin/2 since the last rebuild raises
 * LC_FLAG_DISP (check with lc_workspace_status).  The call starts by sorting
 * into cells and evaluating forces at the given positions, so pos/vel/ids may
 * come in any order and F/cell_start/perm/coord are outputs; trace [device]
 * int64 (nsteps+1) x 2, row 0 being the initial state. */
int lc_verlet_step(const lc_grid *g, const lc_schedule *s, double *pos,
                   double *vel, int32_t *ids, int64_t n, int64_t *F,
                   int32_t *cell_start, int32_t *perm, uint32_t *coord,
                   double dt, int nsteps, int rebuild_every, int64_t *trace,
                   lc_workspace *ws, void *stream);

/* Kinetic energy {sum of rint(0.5 v^2 2^32)} into ke[0] (device int64);
 * ws provides the partial-sum slots. */
int lc_kinetic_energy(const double *vel, int64_t n, int64_t *ke,
                      lc_workspace *ws, void *stream);

/* ---- a8: batched independent boxes -------------------------------------- */

/* One periodic box of a batch: its grid (lc_make_grid) and particle count.
 * In the batch's packed arrays box b owns the particles [pstart_b, pstart_b
 * + n_b) and the cells [cstart_b, cstart_b + ncell_b), in box order. */
typedef struct lc_box_desc {
    lc_grid grid;
    int64_t n;
} lc_box_desc;

/* How a box is split into work-groups. */
#define LC_BATCH_AUTO 0   /* whole box in one work-group when it has <= 36
                             cells and <= 768 particles, else blocks sized
                             to the box density                           */
#define LC_BATCH_WHOLE 1  /* one work-group owns the whole box            */
#define LC_BATCH_BLOCKS 2 /* buffer + reduce blocks (as LC_SCHED_BUFFER)  */

typedef struct lc_batch lc_batch;

typedef struct lc_batch_info {
    int32_t nbox;
    int32_t nwhole;       /* boxes run as one work-group                   */
    int64_t ntot;         /* particles over all boxes                      */
    int64_t ncell;        /* cells over all boxes                          */
    int64_t ngroup;       /* work-groups of one force evaluation           */
    int64_t ntask;        /* cell-cell tasks over all boxes                */
    int32_t max_replicas; /* replica slots per particle (buffer + reduce)  */
    int32_t lds_tile;     /* particles per work-group tile                 */
} lc_batch_info;

/* [host] Build the combined schedule of nbox boxes (Sec. VI strategy 3 for
 * split boxes; whole-box groups need no reduction partner) and upload it to
 * the current device.  modes: per-box LC_BATCH_* (NULL = all AUTO). */
int lc_batch_create(const lc_box_desc *boxes, int nbox, const int32_t *modes,
                    lc_batch **out);

#define LC_BATCH_WRITE_BUFFER 0 /* each group stores into its replica slots,
                                   a gather sums them (Sec. VI strategy 3)  */
#define LC_BATCH_WRITE_ATOMIC 1 /* the same groups add their LDS sums into F
                                   with global int64 atomics, no gather (the
                                   tile-atomics baseline)                    */
typedef struct lc_batch_opts {
    int32_t tile;       /* LDS tile (particles) a split box's block shape is
                           sized for: the first of {3,3,3}, {2,3,3},
                           {2,2,3}, {1,3,3}, {1,2,2}, {1,1,2}, {1,1,1}
                           whose footprint is expected (box density + 35%)
                           to fit; 512 (four work-groups per CU), 768 (0 =
                           default, three), 1024 or 2048                    */
    int32_t write_mode; /* LC_BATCH_WRITE_*                                 */
} lc_batch_opts;
/* lc_batch_create with options (NULL = defaults); LC_EINVAL on other tile
 * sizes or write modes.  The autotuner tries the tile sizes. */
int lc_batch_create_ex(const lc_box_desc *boxes, int nbox, const int32_t *modes,
                       const lc_batch_opts *opts, lc_batch **out);
int lc_batch_info_get(const lc_batch *b, lc_batch_info *out);
/* [host] pstart, cstart: host int64 arrays of nbox + 1 entries. */
int lc_batch_offsets(const lc_batch *b, int64_t *pstart, int64_t *cstart);
void lc_batch_free(lc_batch *b);

/* Counting sort of all boxes at once.  pos [device] double 3 x ntot (box b's
 * particles at pstart_b..), cell_start [device] int32 ncell+1 (global slots),
 * perm [device] int32 ntot (sorted slot -> input index, stays inside the
 * box), coord [device] uint32 3 x ntot.  ws: max_n >= ntot, max_cells >=
 * ncell. */
int lc_batch_build_cells(const lc_batch *b, const double *pos,
                         int32_t *cell_start, int32_t *perm, uint32_t *coord,
                         lc_workspace *ws, void *stream);

/* One force evaluation of every box: all work-groups of all boxes in ONE
 * sweep launch (persistent != 0: a grid sized to the device draws groups from
 * a ticket counter) plus one gather launch.  Groups are launched heaviest
 * first: task count times the square of the box's particles per cell.
 * F [device] int64
 * 3 x ntot; ew [device] int64 nbox x 3 {energy, virial, pairs} per box. */
int lc_batch_forces(const lc_batch *b, const int32_t *cell_start,
                    const uint32_t *coord, int64_t *F, int64_t *ew,
                    int persistent, lc_workspace *ws, void *stream);

/* HIP graph of lc_batch_forces with fixed buffers, captured on `stream`
 * (which must not be the legacy null stream); replays are bit-identical
 * evaluations.  lc_graph_launch enqueues one replay on `stream`.  The graph
 * holds the addresses of the batch's tables, of ws's scratch and of the
 * caller's buffers: all of them must outlive it (free the graph first).
 * While it lives, ws's replica buffer cannot grow: a call that would need a
 * larger one on ws (lc_compute_forces / lc_batch_forces / another capture)
 * returns LC_ECAPACITY instead of moving it. */
typedef struct lc_graph lc_graph;
int lc_batch_graph_create(const lc_batch *b, const int32_t *cell_start,
                          const uint32_t *coord, int64_t *F, int64_t *ew,
                          int persistent, lc_workspace *ws, void *stream,
                          lc_graph **out);
/* HIP graph of one lc_compute_forces evaluation (Sec. IV's cell-pair tasks
 * under schedule s: its phase launches and the closing gather or energy
 * launch, in order) with fixed buffers, captured on `stream` (not the legacy
 * null stream).  Replays recompute F and ew from the current contents of
 * cell_start and coord, bit-identical to lc_compute_forces; replaying
 * removes the per-launch host overhead between a schedule's launches.  The
 * grid, s, ws and the buffers must outlive the graph; ws's replica buffer
 * is pinned as for lc_batch_graph_create.  LC_EINVAL as lc_compute_forces,
 * LC_EHIP when capture or instantiation fails. */
int lc_forces_graph_create(const lc_grid *g, const lc_schedule *s, const int32_t *cell_start,
                           const uint32_t *coord, int64_t n, int64_t *F, int64_t *ew,
                           int precision, lc_workspace *ws, void *stream, lc_graph **out);
int lc_graph_launch(lc_graph *gr, void *stream);
void lc_graph_free(lc_graph *gr);

#ifdef __cplusplus
}
#endif

#endif /* LC_H */
