// lc.hip -- MI355X (gfx950) kernels and C-ABI of the link-cell force sweep.
//
// Kernels
//   k_fill64 / k_fill32     zero-fill (used instead of hipMemsetAsync so the
//                           whole path can sit inside a captured graph)
//   k_bin                   count pass: particles per cell (one counter
//                           atomic per cell and wave)
//   k_scan_lb               exclusive scan of per-cell counts -> cell_start
//                           (one pass, decoupled look-back between tiles)
//   k_scatter               counting-sort scatter: the cell again, a rank
//                           claimed from the counter, perm + sorted box
//                           fractions
//   k_sweep<CAP,WMODE,F64,FF>  one phase of cell-cell tasks (Sec. IV): per
//                           work-group a group of tasks whose footprint cells
//                           are staged in LDS; lanes own j particles, loop over
//                           i; in-cutoff pairs are compacted into a per-wave
//                           queue and evaluated in full waves; int64 forces
//                           accumulate in LDS and are written back with plain
//                           read-modify-write (conflict-free phase), into
//                           replica slots (buffer + reduce), home particles
//                           only (full shell) or with global atomics
//   k_gather_partials       buffer + reduce: sum each particle's replicas
//   k_dataflow<MODE>        creation-order executors (ordered / mutex /
//                           nested), one wave per task runner
//   k_selftest_recip        the fast reciprocal against IEEE division
//   k_kick_ke_drift / k_gather_kick_ke_drift / k_kick_ke
//                           velocity Verlet halves (FP64): a step's closing
//                           half kick with the kinetic energy, fused with the
//                           next step's opening half kick and drift (and, for
//                           buffer + reduce, with the replica gather)
//   k_gather                reorder SoA rows by a permutation
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lc.h"
#include "lc_sched.h"

#pragma clang fp contract(off)

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                           \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(LC_EHIP, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

#define LAUNCHCHK(what)                                                        \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess)                                                  \
            return fail(LC_EHIP, "launch %s: %s", what, hipGetErrorString(e_));\
    } while (0)

extern "C" const char *lc_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------

struct lc_workspace {
    int device = 0;
    int64_t max_n = 0, max_cells = 0;
    int32_t *counts = nullptr;   // max_cells: per-cell counters
    uint32_t *flags = nullptr;   // device status flags
    int64_t *ew = nullptr;       // 3: energy, virial, pairs
    int64_t *part = nullptr;     // kPartSlots x 3 spread partial sums
    int64_t *kpart = nullptr;    // kPartSlots spread kinetic-energy sums
    int64_t *ke = nullptr;       // 1
    double *xref = nullptr;      // 3N positions at the last rebuild
    double *tmp3 = nullptr;      // 3N staging for reorders
    int32_t *tmpi = nullptr;     // N staging for ids
    long long *pbuf = nullptr;   // replica partial sums (buffer + reduce)
    int64_t pbuf_elems = 0;
    int32_t max_per_cell = 0;    // tile sizing hint (0: mean density)
    int32_t *df_sync = nullptr;  // dataflow: per-cell counter or lock
    int32_t *df_ctl = nullptr;   // dataflow: ticket, abort
    int live_graphs = 0;         // graphs captured with this workspace, not yet freed
    unsigned long long *lb_status = nullptr;  // single-pass scan: tile status words
    int32_t *lb_done = nullptr;               // single-pass scan: tiles finished
    int64_t lb_tiles = 0;
};

struct lc_schedule {
    int device = 0;
    int ncu = 256;
    int32_t nc[3] = {0, 0, 0};
    lcs::HostSchedule h;
    int32_t *grp_task = nullptr, *grp_foot = nullptr, *foot_cells = nullptr;
    uint32_t *task_ab = nullptr;
    int32_t *foot_rep = nullptr;  // replica slot | count << 16 (buffer + reduce), home flag
    // the same groups at a fixed stride (see SweepArgs), or none
    uint32_t *fx_task = nullptr;
    int32_t *fx_foot = nullptr, *fx_rep = nullptr, *fx_cnt = nullptr;
    int fx_tmax = 0, fx_fmax = 0;
    // creation-order kinds: tasks in creation order and, per task, how many
    // earlier tasks touch its cells A and B (dataflow executors)
    int32_t *df_a = nullptr, *df_b = nullptr, *df_seqa = nullptr, *df_seqb = nullptr;
    // load-aware schedules: the largest footprint in particles under the
    // counts they were built from (0: unknown); sizes the LDS tile
    int64_t foot_max = 0;
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

constexpr int kPartSlots = 1024;    // spread slots for global int64 sums
constexpr int kWG = 512;            // threads per sweep work-group
constexpr int kNW = kWG / 64;       // waves per sweep work-group
constexpr int kQ = 192;             // per-wave pair queue (>= 128 + 63)
constexpr int kWB0 = lcs::kMaxGroupCells;  // first thread of the write-back waves
constexpr int kFPad = 64;           // filter rows past the footprint (see SweepLDS)
constexpr int kFFCell = kFPad - 4;  // largest cell the filter path stages
constexpr int kMaxT = lcs::kMaxGroupTasks;
constexpr int kMaxChunks = 64;      // chunk tables cover groups of up to 4096 slots
constexpr int kMaxF = lcs::kMaxGroupCells;

static_assert(kMaxT <= kWG && kMaxF <= kWG, "tables scanned one item per thread");
static_assert(kMaxF <= 256, "footprint cell of a particle is stored in one byte");
static_assert(kWB0 % 64 == 0 && kWB0 >= kMaxF && kWB0 + 64 <= kWG, "write-back waves");

typedef short short2v __attribute__((ext_vector_type(2)));

struct PairParams {
    float s[3];    // (float)(L * 2^-32)
    float rc2;     // (float)(rc * rc)
    int thr16;     // candidate filter bound in (unit16)^2, see filter16_bound
    float ecut;    // canonical pair energy at rc2
    double sd[3];  // L * 2^-32 (exact) for the FP64 variant
    double rc2d;   // rc * rc
    double ecutd;  // FP64 pair energy at rc
};

// Box fraction of one coordinate: floor((x * (1/L)) * 2^32) mod 2^32.
__device__ __forceinline__ uint32_t canon(double x, double inv) {
    double s = x * inv;
    double f = floor(s * 4294967296.0);
    return (uint32_t)(long long)f;
}

__device__ __forceinline__ int cell_of(uint32_t u, int nc) {
    return (int)(((unsigned long long)u * (unsigned long long)nc) >> 32);
}

// Round-to-nearest-even of v * 2^32 as int64; flags |q| >= 2^62 and NaN.
__device__ __forceinline__ long long q32f(float v, uint32_t &ovf) {
    float s = v * 4294967296.0f;  // exact scaling by a power of two
    if (!(fabsf(s) < 4611686018427387904.0f)) {
        ovf = 1u;
        return 0;
    }
    return (long long)rintf(s);
}

__device__ __forceinline__ long long q32d(double v, uint32_t &ovf) {
    double s = v * 4294967296.0;
    if (!(fabs(s) < 4611686018427387904.0)) {
        ovf = 1u;
        return 0;
    }
    return (long long)rint(s);
}

__device__ __forceinline__ float canon_d(uint32_t uj, uint32_t ui, float s) {
    return (float)(int)(uj - ui) * s;
}

// Canonical FP32 cutoff test (identical in both precisions).
__device__ __forceinline__ float canon_r2(uint32_t ix, uint32_t iy, uint32_t iz,
                                          uint32_t jx, uint32_t jy, uint32_t jz,
                                          const PairParams &p) {
    float dx = canon_d(jx, ix, p.s[0]);
    float dy = canon_d(jy, iy, p.s[1]);
    float dz = canon_d(jz, iz, p.s[2]);
    float r2 = dx * dx + dy * dy;
    return r2 + dz * dz;
}

// One pair: returns false when outside the cutoff.  q* receive the
// quantised force on j (i gets the negation), energy and virial.
template <bool F64>
__device__ __forceinline__ bool pair_terms(uint32_t ix, uint32_t iy, uint32_t iz,
                                           uint32_t jx, uint32_t jy, uint32_t jz,
                                           const PairParams &p, long long &qx,
                                           long long &qy, long long &qz,
                                           long long &qe, long long &qw,
                                           uint32_t &ovf) {
    float dx = canon_d(jx, ix, p.s[0]);
    float dy = canon_d(jy, iy, p.s[1]);
    float dz = canon_d(jz, iz, p.s[2]);
    float r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    if (!(r2 < p.rc2)) return false;
    if constexpr (!F64) {
        float inv = 1.0f / r2;
        float s6 = inv * inv;
        s6 = s6 * inv;
        float t = 24.0f * inv;
        t = t * s6;
        float g = 2.0f * s6;
        g = g - 1.0f;
        float fs = t * g;
        qx = q32f(fs * dx, ovf);
        qy = q32f(fs * dy, ovf);
        qz = q32f(fs * dz, ovf);
        float e = 4.0f * s6;
        e = e * (s6 - 1.0f);
        e = e - p.ecut;
        qe = q32f(e, ovf);
        qw = q32f(fs * r2, ovf);
    } else {
        double ddx = (double)(int)(jx - ix) * p.sd[0];
        double ddy = (double)(int)(jy - iy) * p.sd[1];
        double ddz = (double)(int)(jz - iz) * p.sd[2];
        double r2d = ddx * ddx + ddy * ddy + ddz * ddz;
        double inv = 1.0 / r2d;
        double s6 = inv * inv * inv;
        double fs = 24.0 * inv * s6 * (2.0 * s6 - 1.0);
        qx = q32d(fs * ddx, ovf);
        qy = q32d(fs * ddy, ovf);
        qz = q32d(fs * ddz, ovf);
        qe = q32d(4.0 * s6 * (s6 - 1.0) - p.ecutd, ovf);
        qw = q32d(fs * r2d, ovf);
    }
    return true;
}

// LDS int64 accumulation (wraps modulo 2^64 like the sums it forms)
__device__ __forceinline__ void lds_sub64(long long *p, long long v) {
    __hip_atomic_fetch_sub((unsigned long long *)p, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Cross-lane steps of a wave-wide inclusive scan, all in DPP (no LDS round
// trips): row_shr 1, 2, 4, 8 scan each row of 16 lanes, then row_bcast 15
// (into rows 1 and 3) and row_bcast 31 (into rows 2 and 3) carry the row
// totals across.  A lane with no source reads `id`.  Every lane of the wave
// must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_from(int id, int x) {
    return __builtin_amdgcn_update_dpp(id, x, CTRL, ROWS, 0xf, false);
}

__device__ __forceinline__ int wave_scan_incl(int x) {
    x += dpp_from<0x111, 0xf>(0, x);
    x += dpp_from<0x112, 0xf>(0, x);
    x += dpp_from<0x114, 0xf>(0, x);
    x += dpp_from<0x118, 0xf>(0, x);
    x += dpp_from<0x142, 0xa>(0, x);
    x += dpp_from<0x143, 0xc>(0, x);
    return x;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_from64(long long x) {
    const uint32_t lo = (uint32_t)dpp_from<CTRL, ROWS>(0, (int)(uint32_t)x);
    const uint32_t hi = (uint32_t)dpp_from<CTRL, ROWS>(0, (int)(uint32_t)((uint64_t)x >> 32));
    return (long long)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ long long wave_scan_incl(long long x) {
    x += dpp_from64<0x111, 0xf>(x);
    x += dpp_from64<0x112, 0xf>(x);
    x += dpp_from64<0x114, 0xf>(x);
    x += dpp_from64<0x118, 0xf>(x);
    x += dpp_from64<0x142, 0xa>(x);
    x += dpp_from64<0x143, 0xc>(x);
    return x;
}

// Wave-wide sum (wraps modulo 2^64), the same value in every lane.
__device__ __forceinline__ long long wave_sum64(long long v) {
    const long long x = wave_scan_incl(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), 63);
    return (long long)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int wave_max32(int v) {
    const int lo = INT_MIN;
    v = max(v, dpp_from<0x111, 0xf>(lo, v));
    v = max(v, dpp_from<0x112, 0xf>(lo, v));
    v = max(v, dpp_from<0x114, 0xf>(lo, v));
    v = max(v, dpp_from<0x118, 0xf>(lo, v));
    v = max(v, dpp_from<0x142, 0xa>(lo, v));
    v = max(v, dpp_from<0x143, 0xc>(lo, v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Exclusive scan of one value per thread over a work-group of NT threads.
template <int NT, typename T>
__device__ T block_scan_excl(T v, T *s_w, T &total) {
    static_assert(NT % 64 == 0 && NT <= 64 * 64, "whole waves, at most 64 of them");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T x = wave_scan_incl(v);
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (w == 0) {  // the wave totals, scanned by wave 0 (all of its lanes active)
        const T t = lane < NT / 64 ? s_w[lane] : (T)0;
        const T inc = wave_scan_incl(t);
        if (lane < NT / 64) s_w[lane] = inc - t;
        if (lane == NT / 64 - 1) s_w[NT / 64] = inc;
    }
    __syncthreads();
    total = s_w[NT / 64];
    T r = x - v + s_w[w];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

__global__ void k_fill64(long long *p, int64_t n, long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

__global__ void k_fill32(int *p, int64_t n, int v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

static int grid_for(int64_t n, int bs) {
    int64_t b = (n + bs - 1) / bs;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

static int fill64(long long *p, int64_t n, hipStream_t st) {
    if (n <= 0) return LC_OK;
    hipLaunchKernelGGL(k_fill64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, 0LL);
    LAUNCHCHK("fill64");
    return LC_OK;
}

static int fill32(int *p, int64_t n, hipStream_t st) {
    if (n <= 0) return LC_OK;
    hipLaunchKernelGGL(k_fill32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, 0);
    LAUNCHCHK("fill32");
    return LC_OK;
}

template <typename T>
static int dalloc(T **p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) return fail(LC_ENOMEM, "hipMalloc(%lld bytes): %s",
                                     (long long)(sizeof(T) * count), hipGetErrorString(e));
    return LC_OK;
}

// ---------------------------------------------------------------------------
// a1: cell build
// ---------------------------------------------------------------------------

struct GridArgs {
    double inv[3];
    int nc[3];
};

// The lanes of a wave that fall into one cell share a single atomic on the
// cell's counter.  Returns this lane's mask of the active lanes in its cell
// (0 for an inactive lane).  Particles stored near each other (a lattice, or
// an array already sorted by cell) then cost one counter update per cell and
// wave instead of one per particle, all of them on the same address.
__device__ __forceinline__ unsigned long long wave_cell_group(bool act, int cc) {
    if (!act) cc = -1;
    // one pass per distinct cell among the active lanes (at most 64)
    unsigned long long todo = __ballot(act), mine = 0ull;
    while (todo) {
        const int lead = (int)__builtin_ctzll(todo);
        const int lcell = __builtin_amdgcn_readlane(cc, lead);
        const unsigned long long same = __ballot(cc == lcell);
        if (cc == lcell) mine = same;
        todo &= ~same;
    }
    return act ? mine : 0ull;
}

// Cell of a particle from its coordinates; its box fractions in u.
__device__ __forceinline__ int cell_and_fractions(const double *__restrict__ pos, int64_t n,
                                                  int64_t i, const double *inv, const int *nc,
                                                  uint32_t u[3]) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
        u[d] = canon(pos[d * n + i], inv[d]);
        c[d] = cell_of(u[d], nc[d]);
    }
    return c[0] + nc[0] * (c[1] + nc[1] * c[2]);
}

// Count pass: every particle adds one to its cell's counter.  Nothing is
// stored per particle; the scatter pass computes the cell again.
__global__ __launch_bounds__(256) void k_bin(const double *__restrict__ pos, int64_t n,
                                             GridArgs ga, int *__restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n;
    int cc = 0;
    uint32_t u[3];
    if (act) cc = cell_and_fractions(pos, n, i, ga.inv, ga.nc, u);
    const unsigned long long mine = wave_cell_group(act, cc);
    const int lane = threadIdx.x & 63;
    if (mine && !(mine & ((1ull << lane) - 1ull))) atomicAdd(&counts[cc], __popcll(mine));
}

// Rank of a particle in its cell, claimed in the scatter pass: the cell's
// counter still holds the cell's size after the scan, and every wave group
// takes its ranks by subtracting its size, so the counters end cleared for
// the next build.  Ranks inside a cell follow the order of the claims (the
// order of particles within a cell is not fixed; every reader treats a cell
// as a set).
__device__ __forceinline__ int wave_cell_claim(bool act, int cc, int *__restrict__ counts) {
    const int lane = threadIdx.x & 63;
    const unsigned long long mine = wave_cell_group(act, cc);
    const unsigned long long below = mine & ((1ull << lane) - 1ull);
    const int k = __popcll(mine);
    int top = 0;
    if (mine && !below) top = atomicSub(&counts[cc], k);
    top = __shfl(top, mine ? (int)__builtin_ctzll(mine) : lane);
    return top - k + __popcll(below);
}

// ---- single-pass scan (decoupled look-back) ------------------------------
//
// Work-group b scans tile b of kLbTile counters and publishes the tile's
// total in status[b]; it then looks back over the lower tiles (64 at a time,
// one per lane of its first wave), adding their totals until it meets one
// that has published its inclusive prefix (tile 0 does so at once), and
// publishes its own.  Status words are 64-bit: flag (1 = tile total, 2 =
// inclusive prefix) << 62 | value, read and written with device-scope atomics
// (coherent across the XCDs' caches).  A tile only waits for lower tiles,
// which the hardware dispatches first, and every wait is bounded (abort
// flag).  The last work-group to finish clears the status words for the next
// scan.  The counters are left as they are: the scatter pass claims its
// ranks from them and leaves them cleared.
constexpr int kLbBS = 1024, kLbIPT = 4, kLbTile = kLbBS * kLbIPT;
constexpr unsigned long long kLbAgg = 1ull << 62, kLbPre = 2ull << 62;

__global__ __launch_bounds__(kLbBS) void k_scan_lb(const int *__restrict__ counts, int64_t m,
                                                   int *__restrict__ out,
                                                   unsigned long long *__restrict__ status,
                                                   int *__restrict__ done,
                                                   uint32_t *__restrict__ flags,
                                                   unsigned long long limit) {
    __shared__ int s_w[kLbBS / 64 + 1];
    __shared__ int s_excl, s_last;
    const int b = (int)blockIdx.x, tid = (int)threadIdx.x, lane = tid & 63;
    const int64_t base = (int64_t)b * kLbTile + (int64_t)tid * kLbIPT;
    int v[kLbIPT];
    if (base + kLbIPT <= m) {  // 16-byte aligned: counts come from hipMalloc
        const int4 q = *reinterpret_cast<const int4 *>(counts + base);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < kLbIPT; ++k) v[k] = base + k < m ? counts[base + k] : 0;
    }
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kLbIPT; ++k) sum += v[k];
    int total;
    int run = block_scan_excl<kLbBS>(sum, s_w, total);
    if (tid == 0)
        __hip_atomic_store(&status[b], (b == 0 ? kLbPre : kLbAgg) | (uint32_t)total,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid < 64) {  // look-back by the first wave
        int excl = 0;
        bool ok = true;
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        for (int w = b - 1; w >= 0 && ok; w -= 64) {
            const int q = w - lane;  // lane 0: the nearest lower tile
            unsigned long long sv = 0ull;
            if (q >= 0) {
                for (;;) {
                    sv = __hip_atomic_load(&status[q], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (sv >> 62) break;
                    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                        atomicOr(flags, (uint32_t)LC_FLAG_ABORT);
                        sv = kLbPre;  // give up: the output is wrong, the wait ends
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            // the nearest tile with an inclusive prefix ends the walk
            const unsigned long long pre = __ballot(q >= 0 && (sv >> 62) == 2ull);
            const int stop = pre ? (int)__builtin_ctzll(pre) : 64;
            int val = (q >= 0 && lane <= stop) ? (int)(uint32_t)sv : 0;
            excl += wave_sum64((long long)val);  // wave-uniform
            if (pre) ok = false;
        }
        if (tid == 0) {
            s_excl = excl;
            if (b > 0)
                __hip_atomic_store(&status[b], kLbPre | (uint32_t)(excl + total),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    run += s_excl;
#pragma unroll
    for (int k = 0; k < kLbIPT; ++k) {
        if (base + k < m) {
            out[base + k] = run;
            run += v[k];
        }
    }
    if (b == (int)gridDim.x - 1 && tid == 0) out[m] = s_excl + total;
    // the last work-group out clears the status words
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        for (int q = tid; q < (int)gridDim.x; q += kLbBS) status[q] = 0ull;
        if (tid == 0) *done = 0;
    }
}

// cell_start from the cell counters (left as they are).
static int scan_counts(lc_workspace *ws, int64_t m, int32_t *cell_start, hipStream_t st) {
    const int64_t nt = (m + kLbTile - 1) / kLbTile;
    if (nt < 1 || nt > ws->lb_tiles) return fail(LC_ECAPACITY, "scan: %lld cells", (long long)m);
    hipLaunchKernelGGL(k_scan_lb, dim3((unsigned)nt), dim3(kLbBS), 0, st, ws->counts, m, cell_start,
                       ws->lb_status, ws->lb_done, ws->flags,
                       100000000ull /* 1 s of s_memrealtime */);
    LAUNCHCHK("k_scan_lb");
    return LC_OK;
}

__global__ __launch_bounds__(256) void k_scatter(const double *__restrict__ pos, int64_t n,
                                                 GridArgs ga, const int *__restrict__ cell_start,
                                                 int *__restrict__ counts, int *__restrict__ perm,
                                                 uint32_t *__restrict__ coord) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n;
    int cc = 0;
    uint32_t u[3] = {0u, 0u, 0u};
    if (act) cc = cell_and_fractions(pos, n, i, ga.inv, ga.nc, u);
    const int r = wave_cell_claim(act, cc, counts);
    if (!act) return;
    const int64_t dst = (int64_t)cell_start[cc] + r;
    perm[dst] = (int)i;
    for (int d = 0; d < 3; ++d) coord[d * n + dst] = u[d];
}

static int build_cells_impl(const lc_grid *g, const double *pos, int64_t n, int32_t *cell_start,
                            int32_t *perm, uint32_t *coord, lc_workspace *ws, hipStream_t st) {
    const int64_t m = g->ncell;
    GridArgs ga;
    for (int d = 0; d < 3; ++d) {
        ga.inv[d] = g->inv_box[d];
        ga.nc[d] = g->nc[d];
    }
    // the cell counters are clear: the workspace starts so and every scatter
    // pass leaves them so
    if (n > 0) {
        hipLaunchKernelGGL(k_bin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n, ga,
                           ws->counts);
        LAUNCHCHK("k_bin");
    }
    int rc = scan_counts(ws, m, cell_start, st);
    if (rc) return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n,
                           ga, cell_start, ws->counts, perm, coord);
        LAUNCHCHK("k_scatter");
    }
    return LC_OK;
}

// ---------------------------------------------------------------------------
// a4/a5: the tile sweep
// ---------------------------------------------------------------------------

struct SweepArgs {
    const int *grp_task;
    const int *grp_foot;
    const int *foot_cells;
    const uint32_t *task_ab;
    int grp_base;
    const int *cell_start;
    const uint32_t *coord;
    int64_t n;
    long long *F;
    // WMODE 3: replica slot of each footprint entry | (the cell's replica
    // count << 16); WMODE 4: home flag
    const int *foot_rep;
    long long *pbuf;      // replica partial sums (WMODE 3), 3 x n per slot
    int *rcnt;            // replica count per particle, written by replica 0 (WMODE 3)
    long long *part;  // kPartSlots x 3 partial {energy, virial, pairs}
    uint32_t *flags;
    PairParams pp;
    // batched boxes (all NULL for a single box)
    const int *grp_box;        // box of each group
    const PairParams *ppar;    // pair parameters per box
    long long *ew_box;         // per-box {energy, virial, pairs}, summed atomically
    // persistent launch: work-groups draw groups from this ticket counter
    int *ticket;
    int ngroups;
    // Optional copy of the group tables at a fixed stride: group g's task
    // entries at fx_task[g * fx_tmax ..], footprint cells (-1 past the end)
    // and replica entries at fx_foot / fx_rep[g * fx_fmax ..], {nt, nf} at
    // fx_cnt[2 g].  A group's setup then reads them all in one round trip.
    const uint32_t *fx_task;
    const int *fx_foot, *fx_rep, *fx_cnt;
    int fx_tmax, fx_fmax;
};

// Exact round-to-nearest-even of v * 2^32 to int64 for |v| < 2^19: the FP64
// sum (double)v + 1.5 * 2^20 lies in [2^20, 2^21), where the FP64 spacing is
// 2^-32, so its one rounding takes v to the nearest multiple of 2^-32 (ties
// to even), and that multiple's count sits in the low mantissa bits:
// bits = bits(1.5 * 2^20) + round(v * 2^32).
constexpr long long kQ32Bias = 0x4138000000000000LL;  // bits of 1.5 * 2^20
// The quantised value plus kQ32Bias (modulo 2^64): a sum of n such terms
// is the sum of the quantised values plus n kQ32Bias, so sums can skip the
// per-term subtraction and remove n kQ32Bias once.
__device__ __forceinline__ long long q32_biased(float v) {
    const double d = (double)v + 1572864.0;  // 1.5 * 2^20
    return (long long)__double_as_longlong(d);
}
__device__ __forceinline__ long long q32_magic(float v) {
    return q32_biased(v) - kQ32Bias;
}

// IEEE (correctly rounded) 1/x for x in [kRcpLo, kRcpHi): the hardware
// estimate, within one ulp, refined by one Newton-Raphson step in fused
// multiply-adds (Markstein's reciprocal iteration).  Equality with IEEE
// division is checked for every float of the range (lc_selftest_recip).
constexpr float kRcpLo = 0.25f, kRcpHi = 128.0f;
__device__ __forceinline__ float rcp_nr(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(e, r, r);
}

// Pairs at least this far apart (r^2 >= 0.3, reduced units) have all five
// quantised terms below 2^17 in magnitude -- at r^2 = 0.3: |f_x| <= fs r
// = 1.19e5, w = fs r^2 = 6.5e4, |e| <= 5.4e3, and the LJ terms only shrink
// with r -- so q32_magic applies to all of them with no per-term range test.
// Closer pairs (not met in a liquid or a crystal) and pairs beyond the
// reciprocal's checked range take IEEE division and q32f, which also flags
// overflow.
constexpr float kFastR2 = 0.3f;
static_assert(kFastR2 >= kRcpLo, "fast pairs lie in the checked reciprocal range");

// Lennard-Jones terms of one pair from inv = 1/r^2, in the canonical order.
__device__ __forceinline__ void lj_terms(float inv, float dx, float dy, float dz, float r2,
                                         float ecut, float &fx, float &fy, float &fz, float &e,
                                         float &w) {
    float s6 = inv * inv;
    s6 = s6 * inv;
    float t = 24.0f * inv;
    t = t * s6;
    float g = 2.0f * s6;
    g = g - 1.0f;
    const float fs = t * g;
    e = 4.0f * s6;
    e = e * (s6 - 1.0f);
    e = e - ecut;
    fx = fs * dx;
    fy = fs * dy;
    fz = fs * dz;
    w = fs * r2;
}

// FP32 pair terms with the fast reciprocal and quantisation; same values as
// pair_terms<false>.  BIASED: qe and qw come with kQ32Bias added (modulo
// 2^64), for sums that remove the bias once per pair counted.  With a
// non-null `flags`, the slow path raises LC_FLAG_OVERFLOW there itself and
// `ovf` is scratch: a caller then carries no overflow state through its
// loop (the fast path cannot overflow).
template <bool BIASED = false>
__device__ __forceinline__ bool pair_terms_fast(const uint4 ui, const uint4 uj, const PairParams &p,
                                                long long &qx, long long &qy, long long &qz,
                                                long long &qe, long long &qw, uint32_t &ovf,
                                                uint32_t *flags = nullptr) {
    float dx = canon_d(uj.x, ui.x, p.s[0]);
    float dy = canon_d(uj.y, ui.y, p.s[1]);
    float dz = canon_d(uj.z, ui.z, p.s[2]);
    float r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    if (!(r2 < p.rc2)) return false;
    float fx, fy, fz, e, w;
    if (r2 >= kFastR2 && r2 < kRcpHi) {
        lj_terms(rcp_nr(r2), dx, dy, dz, r2, p.ecut, fx, fy, fz, e, w);
        qx = q32_magic(fx);
        qy = q32_magic(fy);
        qz = q32_magic(fz);
        qe = BIASED ? q32_biased(e) : q32_magic(e);
        qw = BIASED ? q32_biased(w) : q32_magic(w);
    } else {
        lj_terms(1.0f / r2, dx, dy, dz, r2, p.ecut, fx, fy, fz, e, w);
        qx = q32f(fx, ovf);
        qy = q32f(fy, ovf);
        qz = q32f(fz, ovf);
        qe = q32f(e, ovf);
        qw = q32f(w, ovf);
        if constexpr (BIASED) {
            qe = (long long)((unsigned long long)qe + (unsigned long long)kQ32Bias);
            qw = (long long)((unsigned long long)qw + (unsigned long long)kQ32Bias);
        }
        if (flags && ovf) atomicOr(flags, (uint32_t)LC_FLAG_OVERFLOW);
    }
    return true;
}

// Shared memory of one sweep work-group.  FF: the tile also holds the
// 16-bit coordinates of the candidate filter.
template <int CAP, int WMODE, bool FF>
struct SweepLDS {
    // box fractions, one array per axis (a random pair read is then three
    // 4-byte reads, which conflict less in the LDS banks than one 12-byte
    // read at a 16-byte stride)
    uint32_t ux[CAP], uy[CAP], uz[CAP];
    // filter coordinates: the top 16 bits of the box fractions, x | y << 16
    // and z; the filter reads rows aoff .. aoff + kmax - 1 for every lane
    // (kmax: the wave's largest cell A), so it runs past the footprint by
    // less than kFPad when no cell holds more than kFFCell
    uint2 h[FF ? CAP + kFPad : 1];
    long long acc[WMODE == 2 ? 1 : 3][WMODE == 2 ? 1 : CAP];  // int64 forces
    int fg[kMaxF];          // global first slot of each footprint cell
    int fl[kMaxF + 1];      // local first slot (prefix over the footprint)
    int frep[WMODE >= 3 ? kMaxF : 1];  // replica slot (3) / home flag (4) of each footprint cell
    uint8_t pc[CAP];        // footprint cell of each staged particle
    int ta[kMaxT];          // task: local first slot of A | (count of A << 16)
    int tb[kMaxT];          // task: local first slot of B, bit 31 = intra
    int tslot[kMaxT + 1];   // prefix of |B| over the tasks
    // per 64-slot chunk (nslot <= 64 * kMaxChunks): the task of its first
    // slot, a mask of the slots where a later task starts, and the largest
    // cell A among its tasks
    int ct0[kMaxChunks];
    unsigned long long cmask[kMaxChunks];
    int ckmax[kMaxChunks];
    long long w64[kNW + 1];
    uint32_t q[kNW][kQ];    // per-wave queue of in-cutoff pairs (see sweep_pairs)
    long long red[kNW][3];
    int w[kNW + 1];
    int big;  // a footprint cell holds more than kFFCell particles
};

// Global slot of a local footprint index.
template <class L>
__device__ __forceinline__ int64_t foot_gidx(const L &sh, int nf, int l) {
    int lo = 0, hi = nf;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sh.fl[mid] <= l) lo = mid; else hi = mid;
    }
    return (int64_t)sh.fg[lo] + (l - sh.fl[lo]);
}

// Footprint cell (local index) holding a local particle index.
template <class L>
__device__ __forceinline__ int foot_cell(const L &sh, int nf, int l) {
    int lo = 0, hi = nf;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sh.fl[mid] <= l) lo = mid; else hi = mid;
    }
    return lo;
}

// The candidate loop and pair evaluation of one work-group.
//   STAGED: the footprint's box fractions and accumulators live in LDS;
//           otherwise box fractions come from global memory and every pair
//           adds into F with global atomics.
//   FF:     candidates first pass a 16-bit integer filter (the top halves of
//           the box fractions against an enlarged cutoff, see
//           filter16_bound); the exact canonical test is repeated when the
//           pair is evaluated.
// Lanes own j slots (64 consecutive slots of the concatenated B cells of the
// group's tasks) and loop over the i particles of their task's cell A;
// pairs inside the cutoff are compacted into a per-wave queue and evaluated
// 128 at a time (two full-wave batches), so the Lennard-Jones arithmetic
// runs on full waves.  A staged queue entry holds the byte offsets of the
// pair's two rows in a 4-byte per-particle array, 4 i | 4 j << 16 (the LDS
// reads take them as addresses as they are; i, j < CAP <= 2048); unstaged,
// it holds i | j << 16 (up to 65535 footprint particles).
template <int CAP, int WMODE, bool F64, bool STAGED, bool FF>
__device__ __forceinline__ void sweep_pairs(SweepLDS<CAP, WMODE, FF> &sh, const SweepArgs &a,
                                            const PairParams &pp, int f0, int nf, int nt,
                                            int nslot, long long &e_sum, long long &w_sum,
                                            long long &p_cnt, uint32_t &ovf) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n = a.n;
    uint32_t *q = sh.q[wave];
    int qn = 0;  // wave-uniform queue length
    constexpr uint32_t kEs = STAGED ? 2u : 0u;  // entry scale: i << kEs | j << (16 + kEs)
    static_assert(!STAGED || CAP <= 16384, "staged entries hold 4 i in 16 bits");

    // box fractions of the particle of entry field b (staged: the byte
    // offset of its 4-byte rows; unstaged: its local index)
    auto load_u = [&](uint32_t b) -> uint4 {
        if constexpr (STAGED) {
            auto row = [&](const uint32_t *arr) {
                return *(const uint32_t *)((const char *)arr + b);
            };
            return make_uint4(row(sh.ux), row(sh.uy), row(sh.uz), 0u);
        } else {
            const int64_t gi = foot_gidx(sh, nf, (int)b);
            return make_uint4(a.coord[gi], a.coord[n + gi], a.coord[2 * n + gi], 0u);
        }
    };

    // one queued pair: its coordinates are loaded first (load), so that the
    // loads of two batches are in flight together, then evaluated (eval)
    struct PairIn {
        uint4 ui, uj;
        uint32_t bi, bj;  // the entry's two fields (see kEs)
    };
    auto load = [&](uint32_t ent) -> PairIn {
        PairIn r;
        r.bi = ent & 0xffffu;
        r.bj = ent >> 16;
        r.ui = load_u(r.bi);
        r.uj = load_u(r.bj);
        return r;
    };
    // int64 accumulator k of the staged particle whose 4-byte rows start at
    // byte b
    auto acc_at = [&](int k, uint32_t b) -> long long * {
        return (long long *)((char *)&sh.acc[k][0] + 2 * b);
    };
    auto eval = [&](const PairIn &pin) {
        const int il = (int)(pin.bi >> kEs), jl = (int)(pin.bj >> kEs);
        const uint4 ui = pin.ui, uj = pin.uj;
        long long qx, qy, qz, qe, qw;
        bool in;
        if constexpr (F64) {
            in = pair_terms<true>(ui.x, ui.y, ui.z, uj.x, uj.y, uj.z, pp, qx, qy, qz, qe, qw, ovf);
        } else {
            uint32_t o = 0u;  // the slow path raises the flag itself
            in = pair_terms_fast<true>(ui, uj, pp, qx, qy, qz, qe, qw, o, a.flags);
        }
        if (!in) return;
        // (FP32: biased energy and virial terms, corrected below)
        e_sum = (long long)((unsigned long long)e_sum + (unsigned long long)qe);
        w_sum = (long long)((unsigned long long)w_sum + (unsigned long long)qw);
        p_cnt += 1;
        if constexpr (STAGED && WMODE != 2) {
            lds_sub64(acc_at(0, pin.bi), qx);  // ds_sub_u64: no negation
            lds_sub64(acc_at(1, pin.bi), qy);
            lds_sub64(acc_at(2, pin.bi), qz);
            if constexpr (WMODE != 4) {  // full shell: j gets its force from (j, i)
                atomicAdd((unsigned long long *)acc_at(0, pin.bj), (unsigned long long)qx);
                atomicAdd((unsigned long long *)acc_at(1, pin.bj), (unsigned long long)qy);
                atomicAdd((unsigned long long *)acc_at(2, pin.bj), (unsigned long long)qz);
            }
        } else {
            // global path: into F, or (buffer + reduce) into this group's
            // replica slots, which no other group writes
            int64_t gi = foot_gidx(sh, nf, il), gj = foot_gidx(sh, nf, jl);
            unsigned long long *Fi = (unsigned long long *)a.F, *Fj = Fi;
            if constexpr (WMODE == 3) {
                const int ri = sh.frep[foot_cell(sh, nf, il)] & 0xffff;
                const int rj = sh.frep[foot_cell(sh, nf, jl)] & 0xffff;
                Fi = (unsigned long long *)a.pbuf + (int64_t)ri * 3 * n;
                Fj = (unsigned long long *)a.pbuf + (int64_t)rj * 3 * n;
            }
            atomicAdd(&Fi[gi], (unsigned long long)(-qx));
            atomicAdd(&Fi[n + gi], (unsigned long long)(-qy));
            atomicAdd(&Fi[2 * n + gi], (unsigned long long)(-qz));
            if constexpr (WMODE != 4) {
                atomicAdd(&Fj[gj], (unsigned long long)qx);
                atomicAdd(&Fj[n + gj], (unsigned long long)qy);
                atomicAdd(&Fj[2 * n + gj], (unsigned long long)qz);
            }
        }
    };

    // queue an in-cutoff pair (m: the wave's ballot of in); evaluate 64 at
    // a time
    auto push_ent = [&](unsigned long long m, bool in, uint32_t ent) {
        if (in) {
            const int below = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            q[qn + below] = ent;
        }
        qn += (int)__popcll(m);
        if (qn >= 128) {  // two batches, their loads in flight together
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            const PairIn p0 = load(q[lane]), p1 = load(q[lane + 64]);
            const uint32_t rest = lane + 128 < qn ? q[lane + 128] : 0u;
            eval(p0);
            eval(p1);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            if (lane + 128 < qn) q[lane] = rest;
            qn -= 128;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        }
    };
    auto push = [&](bool in, int il, uint32_t jbits) {
        push_ent(__ballot(in), in, ((uint32_t)il << kEs) | jbits);
    };

    const bool tables = nslot <= 64 * kMaxChunks;
    for (int c = wave; c * 64 < nslot; c += kNW) {
        const int base = c * 64;
        const int s = base + lane;
        const bool valid = s < nslot;
        int t, kmax_c = 0;
        if (tables) {
            // the chunk's first task plus the task starts at or below this
            // lane's slot (no task starts past nslot)
            const unsigned long long m = sh.cmask[c] >> 1;
            t = __builtin_amdgcn_readfirstlane(sh.ct0[c]) +
                (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            kmax_c = __builtin_amdgcn_readfirstlane(sh.ckmax[c]);
        } else {
            // task of the chunk's first slot (one wave-uniform search), then
            // each lane steps forward to its own task
            int lo = 0, hi = nt;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sh.tslot[mid] <= base) lo = mid; else hi = mid;
            }
            t = __builtin_amdgcn_readfirstlane(lo);
            const int slast = min(s, nslot - 1);
            while (sh.tslot[t + 1] <= slast) ++t;
        }
        const int jj = s - sh.tslot[t];
        const int bo = sh.tb[t];
        const bool intra = bo < 0;
        const int jl = (bo & 0x7fffffff) + jj;
        const uint32_t jbits = (uint32_t)jl << (16 + kEs);
        const int ta = sh.ta[t];
        const int aoff = ta & 0xffff;
        // i runs over cell A; an intra task keeps each unordered pair once
        // (i before j inside the cell)
        if constexpr (STAGED && FF) {
            // Two stages per block of up to 32 i.  A tight integer filter
            // (a superset of the cutoff sphere, see filter16_bound; the exact
            // canonical test is repeated when the pair is evaluated) shifts
            // one bit per candidate i into a mask, first i highest; all lanes
            // of a task read the same row, which LDS broadcasts.  The set
            // bits are then queued, each lane starting at its own bit so that
            // a batch's i-side adds spread over addresses.
            const int na = valid ? (ta >> 16) : 0;
            const int a0 = valid ? aoff : 0;
            const int kmax = tables ? kmax_c : __builtin_amdgcn_readfirstlane(wave_max32(na));
            const uint2 hj = valid ? sh.h[jl] : make_uint2(0u, 0u);
            // intra: i before j (each unordered pair once), or, in the full
            // shell, every i but j itself
            const int lim = (intra && WMODE != 4) ? min(jj, na) : na;
            const uint32_t rot = (uint32_t)jj & 31u, rot4 = rot << kEs;
            // one candidate row: 16-bit differences wrap modulo the box (the
            // minimum image up to one unit per axis); r2 - bound is negative
            // (sign bit set) inside, and the sign bit is shifted into m
            // The first dot product takes the bound from a register it does
            // not overwrite (the three-operand form; the compiler would copy
            // the bound into the accumulating two-operand form, one more
            // instruction per row).
            const int nthr = -pp.thr16;
            auto row = [&](const uint2 hi, uint32_t m) -> uint32_t {
                const short2v dxy =
                    __builtin_bit_cast(short2v, hj.x) - __builtin_bit_cast(short2v, hi.x);
                const short2v dz0 =
                    __builtin_bit_cast(short2v, hj.y) - __builtin_bit_cast(short2v, hi.y);
                int t;
                asm("v_dot2_i32_i16 %0, %1, %1, %2" : "=v"(t) : "v"(dz0), "v"(nthr));
                t = __builtin_amdgcn_sdot2(dxy, dxy, t, false);
                return __builtin_amdgcn_alignbit(m, (uint32_t)t, 31);
            };
            for (int k0 = 0; k0 < kmax; k0 += 32) {
                const int kr = min(kmax - k0, 32);  // rows read, uniform
                const uint2 *ha = &sh.h[a0 + k0];
                uint32_t m = 0u;
                int k = 0;
                for (; k + 4 <= kr; k += 4) {  // four rows per address step
                    m = row(ha[k], m);
                    m = row(ha[k + 1], m);
                    m = row(ha[k + 2], m);
                    m = row(ha[k + 3], m);
                }
                for (; k < kr; ++k) m = row(ha[k], m);
                // row k sits at bit kr - 1 - k; keep rows k < lim - k0
                const int nv = lim - k0;
                m = nv <= 0 ? 0u : nv >= kr ? m : m & ~((1u << (kr - nv)) - 1u);
                if constexpr (WMODE == 4) {  // drop the self pair
                    const int sj = jj - k0;
                    if (intra && sj >= 0 && sj < kr) m &= ~(1u << (kr - 1 - sj));
                }
                m = __builtin_amdgcn_alignbit(m, m, rot);  // rotate right
                // entry of the bit at (rotated) position p: (4 i | 4 j << 16)
                // with i = a0 + k0 + kr - 1 - ((p + rot) & 31), no borrow
                // into j
                const uint32_t ebase = ((uint32_t)(a0 + k0 + kr - 1) << kEs) | jbits;
                for (;;) {
                    const bool has = m != 0u;
                    const unsigned long long bal = __ballot(has);
                    if (!bal) break;
                    uint32_t e = 0u;
                    if (has) {
                        e = ebase - ((((uint32_t)__builtin_ctz(m) << kEs) + rot4) &
                                     (31u << kEs));
                        m &= m - 1u;
                    }
                    push_ent(bal, has, e);
                }
            }
        } else {
            // diagonal order: lane jj visits i = (k + jj) mod na, so lanes of
            // one task touch different i at each step (spreads the i-side
            // atomics); an intra task keeps a pair when i < j
            const uint4 uj = valid ? load_u((uint32_t)jl << kEs) : make_uint4(0u, 0u, 0u, 0u);
            const int na = valid ? (ta >> 16) : 0;
            const int kdiag = tables ? kmax_c : wave_max32(na);
            int ik = na > 0 ? jj % na : 0;
            for (int k = 0; k < kdiag; ++k) {
                const bool act = k < na && (!intra || (WMODE == 4 ? ik != jj : ik < jj));
                bool in = false;
                if (act) {
                    const uint4 ui = load_u((uint32_t)(aoff + ik) << kEs);
                    in = canon_r2(ui.x, ui.y, ui.z, uj.x, uj.y, uj.z, pp) < pp.rc2;
                }
                push(in, aoff + ik, jbits);
                ik = ik + 1 == na ? 0 : ik + 1;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (lane < qn) eval(load(q[lane]));
    if (lane + 64 < qn) eval(load(q[lane + 64]));
    if constexpr (!F64) {  // remove the bias of the p_cnt energy and virial terms
        const unsigned long long b = (unsigned long long)p_cnt * (unsigned long long)kQ32Bias;
        e_sum = (long long)((unsigned long long)e_sum - b);
        w_sum = (long long)((unsigned long long)w_sum - b);
    }
}

// What a group's setup reads from global memory before its LDS work: the
// group's task and footprint ranges, each thread's task entry and footprint
// cell (with its replica slot and particle range).  The reads form a chain
// of three dependent round trips (ranges; entries; cell starts); a
// persistent work-group runs the chain for its next group while it works on
// the current one.
struct GroupPre {
    int g, box;           // group, its box (batched launches)
    int t0, nt, f0, nf;   // task and footprint ranges
    int hv;               // ranges as loaded, one value per lane (see pre_head)
    uint32_t ab;          // task entry of this thread (tid < nt)
    int c, rep;           // footprint cell of this thread (-1: none), replica slot
    int gs, ge;           // its particle range
};

// The ranges are read with one vector load (lanes 0-4 fetch the five
// values), not scalar loads: a wait for scalar loads is also a wait for LDS,
// so scalar prefetches would stall the current group's first barrier.
__device__ __forceinline__ void pre_head(const SweepArgs &a, int g, GroupPre &p) {
    const int lane = threadIdx.x & 63;
    const int *src = lane == 1   ? a.grp_task + g + 1
                     : lane == 2 ? a.grp_foot + g
                     : lane == 3 ? a.grp_foot + g + 1
                     : lane == 4 && a.grp_box ? a.grp_box + g
                                              : a.grp_task + g;
    p.g = g;
    p.hv = *src;
}

__device__ __forceinline__ void pre_head_done(const SweepArgs &a, GroupPre &p) {
    p.t0 = __builtin_amdgcn_readlane(p.hv, 0);
    p.nt = __builtin_amdgcn_readlane(p.hv, 1) - p.t0;
    p.f0 = __builtin_amdgcn_readlane(p.hv, 2);
    p.nf = __builtin_amdgcn_readlane(p.hv, 3) - p.f0;
    p.box = a.grp_box ? __builtin_amdgcn_readlane(p.hv, 4) : 0;
}

template <int WMODE>
__device__ __forceinline__ void pre_foot(const SweepArgs &a, GroupPre &p) {
    const int tid = threadIdx.x;
    p.ab = tid < p.nt ? a.task_ab[p.t0 + tid] : 0u;
    p.c = tid < p.nf ? a.foot_cells[p.f0 + tid] : -1;
    p.rep = (WMODE >= 3 && tid < p.nf) ? a.foot_rep[p.f0 + tid] : 0;
}

// Both steps of pre_head / pre_foot in one round trip, from the fixed-stride
// tables.
template <int WMODE>
__device__ __forceinline__ void pre_fixed(const SweepArgs &a, int g, GroupPre &p) {
    const int tid = threadIdx.x, lane = tid & 63;
    p.g = g;
    p.box = 0;
    const int hv = a.fx_cnt[2 * g + (lane & 1)];
    const int64_t tb = (int64_t)g * a.fx_tmax, fb = (int64_t)g * a.fx_fmax;
    p.ab = tid < a.fx_tmax ? a.fx_task[tb + tid] : 0u;
    p.c = tid < a.fx_fmax ? a.fx_foot[fb + tid] : -1;
    p.rep = (WMODE >= 3 && tid < a.fx_fmax) ? a.fx_rep[fb + tid] : 0;
    p.t0 = 0;
    p.f0 = 0;
    p.nt = __builtin_amdgcn_readlane(hv, 0);
    p.nf = __builtin_amdgcn_readlane(hv, 1);
}

__device__ __forceinline__ void pre_cells(const SweepArgs &a, GroupPre &p) {
    p.gs = p.c >= 0 ? a.cell_start[p.c] : 0;
    p.ge = p.c >= 0 ? a.cell_start[p.c + 1] : 0;
}

// All work of one task group (see k_sweep).  p: the group's prefetched
// setup data.  With PF the next group's chain (nx, whose ranges are already
// loaded) is advanced at two points of this group's work, so that its loads
// are in flight while this group computes; *stage counts the links done.
template <int CAP, int WMODE, bool F64, bool FF, bool PF>
__device__ __forceinline__ void sweep_group(SweepLDS<CAP, WMODE, FF> &sh, const SweepArgs &a,
                                            const GroupPre &p, GroupPre &nx, int &stage) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = p.g;
    const PairParams pp = a.ppar ? a.ppar[p.box] : a.pp;
    const int nt = p.nt, f0 = p.f0, nf = p.nf;
    const int64_t n = a.n;

    // footprint table and local layout
    const uint32_t my_ab = p.ab;
    int cnt = 0;
    if (tid < nf) {
        if constexpr (WMODE >= 3) sh.frep[tid] = p.rep;
        cnt = p.ge - p.gs;
        sh.fg[tid] = p.gs;
    }
    int total;
    if constexpr (FF) {
        if (tid == 0) sh.big = 0;  // ordered before the scan's barriers
    }
    const int lofs = block_scan_excl<kWG>(cnt, sh.w, total);
    if (tid < nf) sh.fl[tid] = lofs;
    if (tid == 0) sh.fl[nf] = total;
    if (total > 65535) {  // local indices are packed in 16 bits
        if (tid == 0) atomicOr(a.flags, (uint32_t)LC_FLAG_OVERFLOW);
        return;
    }
    if constexpr (FF) {
        if (cnt > kFFCell) sh.big = 1;
    }
    if (total <= CAP)  // footprint cell of every particle (nf <= 256)
        for (int r = 0; r < cnt; ++r) sh.pc[lofs + r] = (uint8_t)tid;
    __syncthreads();
    bool staged = total <= CAP;
    if constexpr (FF) staged = staged && !sh.big;
    if (!staged && tid == 0) atomicOr(a.flags, (uint32_t)LC_FLAG_FALLBACK);

    // Stage the footprint, one particle per thread and round.  The global
    // loads are issued first, all in flight together, and land in registers
    // while the task table is built; the LDS stores follow.  With plain
    // write-back (WMODE 0) the accumulators start from the current forces,
    // which no other work-group of this phase touches, so the write-back
    // below is a plain store.
    constexpr int NK = (CAP + kWG - 1) / kWG;
    uint32_t su[NK][3];
    long long sfo[WMODE == 0 ? NK : 1][3];
    if (staged) {
#pragma unroll
        for (int r = 0; r < NK; ++r) {
            const int k = tid + r * kWG;
            if (k < total) {
                const int f = sh.pc[k];
                const int64_t gi = (int64_t)sh.fg[f] + (k - sh.fl[f]);
                su[r][0] = a.coord[gi];
                su[r][1] = a.coord[n + gi];
                su[r][2] = a.coord[2 * n + gi];
                if constexpr (WMODE == 0) {
                    sfo[r][0] = a.F[gi];
                    sfo[r][1] = a.F[n + gi];
                    sfo[r][2] = a.F[2 * n + gi];
                }
            }
        }
    }
    if constexpr (WMODE == 3) {
        if (!staged) {  // the global path accumulates into the replica slots
            for (int k = tid; k < total; k += kWG) {
                const int f = foot_cell(sh, nf, k);
                const int64_t gi = (int64_t)sh.fg[f] + (k - sh.fl[f]);
                const int fr = sh.frep[f];
                long long *P = a.pbuf + (int64_t)(fr & 0xffff) * 3 * n;
                P[gi] = 0;
                P[n + gi] = 0;
                P[2 * n + gi] = 0;
                if ((fr & 0xffff) == 0) a.rcnt[gi] = fr >> 16;
            }
            __syncthreads();
        }
    }
    if constexpr (WMODE == 4) {
        if (!staged) {  // the global path adds into F: clear the home particles
            for (int k = tid; k < total; k += kWG) {
                const int f = foot_cell(sh, nf, k);
                if (!sh.frep[f]) continue;
                const int64_t gi = (int64_t)sh.fg[f] + (k - sh.fl[f]);
                a.F[gi] = 0;
                a.F[n + gi] = 0;
                a.F[2 * n + gi] = 0;
            }
            __threadfence();
            __syncthreads();
        }
    }
    // task table: a task with an empty cell has no pairs and is dropped; the
    // others are numbered densely in the order given, so that consecutive
    // tasks own consecutive j slots
    int na_t = 0, nb_t = 0, ta_v = 0, tb_v = 0;
    if (tid < nt) {
        const int la = (int)(my_ab & 0xffffu), lb = (int)(my_ab >> 16);
        na_t = sh.fl[la + 1] - sh.fl[la];
        nb_t = sh.fl[lb + 1] - sh.fl[lb];
        ta_v = sh.fl[la] | (na_t << 16);
        tb_v = sh.fl[lb] | (la == lb ? (int)0x80000000 : 0);
    }
    const bool live = na_t > 0 && nb_t > 0;
    if (tid < kMaxChunks) {  // ordered before the atomics by the scan's barriers
        sh.cmask[tid] = 0ull;
        sh.ckmax[tid] = 0;
    }
    long long tot64;
    const long long pre = block_scan_excl<kWG>(live ? (1LL << 32) | nb_t : 0LL, sh.w64, tot64);
    const int ntl = (int)(tot64 >> 32), nslot = (int)(uint32_t)tot64;
    if (live) {
        const int ct = (int)(pre >> 32), so = (int)(uint32_t)pre;
        sh.ta[ct] = ta_v;
        sh.tb[ct] = tb_v;
        sh.tslot[ct] = so;
        if (nslot <= 64 * kMaxChunks) {
            if (so & 63) atomicOr(&sh.cmask[so >> 6], 1ull << (so & 63));
            for (int c = so >> 6; c <= (so + nb_t - 1) >> 6; ++c) {
                if (c << 6 >= so) sh.ct0[c] = ct;  // the task holding the chunk's first slot
                atomicMax(&sh.ckmax[c], na_t);
            }
        }
    }
    if (tid == 0) sh.tslot[ntl] = nslot;
    if (staged) {
#pragma unroll
        for (int r = 0; r < NK; ++r) {
            const int k = tid + r * kWG;
            if (k < total) {
                const uint32_t ux = su[r][0], uy = su[r][1], uz = su[r][2];
                for (int d = 0; d < 3; ++d) {
                    if constexpr (WMODE == 0)
                        sh.acc[d][k] = sfo[r][d];
                    else if constexpr (WMODE == 1 || WMODE >= 3)
                        sh.acc[d][k] = 0;
                }
                sh.ux[k] = ux;
                sh.uy[k] = uy;
                sh.uz[k] = uz;
                if constexpr (FF) sh.h[k] = make_uint2((ux >> 16) | (uy & 0xffff0000u), uz >> 16);
            }
        }
    }
    __syncthreads();
    if constexpr (PF) {  // next group: task entries and footprint cells
        pre_head_done(a, nx);
        pre_foot<WMODE>(a, nx);
        stage = 2;
    }

    long long e_sum = 0, w_sum = 0, p_cnt = 0;
    uint32_t ovf = 0;
    if (staged)
        sweep_pairs<CAP, WMODE, F64, true, FF>(sh, a, pp, f0, nf, ntl, nslot, e_sum, w_sum, p_cnt,
                                               ovf);
    else
        sweep_pairs<CAP, WMODE, F64, false, FF>(sh, a, pp, f0, nf, ntl, nslot, e_sum, w_sum, p_cnt,
                                                ovf);
    if constexpr (PF) {  // next group: particle ranges of its footprint cells
        pre_cells(a, nx);
        stage = 3;
    }

    // energy, virial, pair count: reduce over the work-group, then one
    // atomic per sum into a slot spread by group index (same-address global
    // atomics from every work-group would serialise)
    e_sum = wave_sum64(e_sum);
    w_sum = wave_sum64(w_sum);
    p_cnt = wave_sum64(p_cnt);
    if (lane == 0) {
        sh.red[wave][0] = e_sum;
        sh.red[wave][1] = w_sum;
        sh.red[wave][2] = p_cnt;
    }
    if (__ballot(ovf != 0u) && lane == 0) atomicOr(a.flags, (uint32_t)LC_FLAG_OVERFLOW);
    __syncthreads();
    // With a next group in flight (PF) the global stores and atomics of the
    // tail are issued by the waves from kWB0 on only.  The first waves hold
    // the next group's footprint loads, and one counter tracks a wave's
    // loads and stores alike, so a wait for those loads would otherwise also
    // wait for this group's stores to complete.
    constexpr int wb0 = PF ? kWB0 : 0;
    const int wt = tid - wb0;
    if (wt >= 0 && wt < 3) {
        long long v = 0;
        for (int k = 0; k < kNW; ++k) v += sh.red[k][wt];
        long long *dst = a.ew_box ? &a.ew_box[p.box * 3 + wt]
                                  : &a.part[(g % kPartSlots) * 3 + wt];
        atomicAdd((unsigned long long *)dst, (unsigned long long)v);
    }

    if constexpr (WMODE == 3) {
        if (!staged) return;
        for (int k = wt < 0 ? total : wt; k < total; k += kWG - wb0) {
            const int f = sh.pc[k];
            const int64_t gi = (int64_t)sh.fg[f] + (k - sh.fl[f]);
            const int fr = sh.frep[f];
            long long *P = a.pbuf + (int64_t)(fr & 0xffff) * 3 * n;
            P[gi] = sh.acc[0][k];
            P[n + gi] = sh.acc[1][k];
            P[2 * n + gi] = sh.acc[2][k];
            // the cell's first replica also records how many there are
            if ((fr & 0xffff) == 0) a.rcnt[gi] = fr >> 16;
        }
    } else if constexpr (WMODE == 4) {
        if (!staged) return;
        for (int k = wt < 0 ? total : wt; k < total; k += kWG - wb0) {
            const int f = sh.pc[k];
            if (!sh.frep[f]) continue;  // home particles only
            const int64_t gi = (int64_t)sh.fg[f] + (k - sh.fl[f]);
            a.F[gi] = sh.acc[0][k];
            a.F[n + gi] = sh.acc[1][k];
            a.F[2 * n + gi] = sh.acc[2][k];
        }
    } else if constexpr (WMODE != 2) {
        if (!staged) return;
        unsigned long long *F = (unsigned long long *)a.F;
        for (int k = wt < 0 ? total : wt; k < total; k += kWG - wb0) {
            const int f = sh.pc[k];
            const int64_t gi = (int64_t)sh.fg[f] + (k - sh.fl[f]);
            for (int d = 0; d < 3; ++d) {
                const unsigned long long v = (unsigned long long)sh.acc[d][k];
                if constexpr (WMODE == 0)
                    F[d * n + gi] = v;
                else
                    atomicAdd(&F[d * n + gi], v);
            }
        }
    }
}

// One phase of cell-cell tasks.  Without a ticket counter every work-group
// runs group grp_base + blockIdx.x; with one (persistent launch) each
// work-group keeps drawing the next group until all ngroups are taken.
// WMODE: 0 = accumulate in LDS, plain read-modify-write of the footprint
//        (the phase must be conflict-free); 1 = accumulate in LDS, global
//        atomic write-back; 2 = every pair adds into global memory with
//        atomics; 3 = accumulate in LDS, plain stores into the group's
//        replica slots (buffer + reduce); 4 = full shell: only the i side
//        accumulates, plain stores of the group's home particles.
// Occupancy: a 512-particle tile (40 KB of LDS) leaves room for four
// work-groups per compute unit, which then need at most 64 VGPRs (eight
// waves per SIMD); a 768-particle tile for three at 80 VGPRs (six waves).
// The register allocator spills a few dozen values, mostly outside the pair
// loops, which costs less than the group setup latency the extra
// work-group hides (measured at 256k: 2x2x3 blocks 62.5 -> 60.3 us per
// evaluation, 1x2x3 73.8 -> 68.5 us).  Larger tiles are held to two
// work-groups by LDS anyway.
template <int CAP, int WMODE, bool F64, bool FF>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(CAP <= 512 ? 8 : CAP <= 768 ? 6 : 1)))
void k_sweep(SweepArgs a) {
    __shared__ SweepLDS<CAP, WMODE, FF> sh;
    __shared__ int s_tk[1];
    GroupPre p, nx;
    int stage = 0;
    if (!a.ticket) {
        if (a.fx_task) {
            pre_fixed<WMODE>(a, a.grp_base + blockIdx.x, p);
        } else {
            pre_head(a, a.grp_base + blockIdx.x, p);
            pre_head_done(a, p);
            pre_foot<WMODE>(a, p);
        }
        pre_cells(a, p);
        sweep_group<CAP, WMODE, F64, FF, false>(sh, a, p, nx, stage);
        return;
    }
    // Persistent: tickets are drawn one group ahead, so the next group is
    // known while the current one runs and its setup reads overlap it.  The
    // first two groups of every work-group are fixed (no burst of atomics on
    // the one counter at launch); the counter hands out the rest.
    const int grid = (int)gridDim.x;
    int k = (int)blockIdx.x, kn = k + grid;
    if (k >= a.ngroups) return;
    pre_head(a, a.grp_base + k, p);
    pre_head_done(a, p);
    pre_foot<WMODE>(a, p);
    pre_cells(a, p);
    for (;;) {
        const bool more = kn < a.ngroups;  // uniform
        int tk = 0;
        if (more) {
            pre_head(a, a.grp_base + kn, nx);
            if (threadIdx.x == 0) tk = 2 * grid + atomicAdd(a.ticket, 1);  // after next
        }
        stage = 1;
        if (more)
            sweep_group<CAP, WMODE, F64, FF, true>(sh, a, p, nx, stage);
        else
            sweep_group<CAP, WMODE, F64, FF, false>(sh, a, p, nx, stage);
        if (threadIdx.x == 0) s_tk[0] = tk;
        __syncthreads();
        if (!more) break;
        const int knn = s_tk[0];  // rewritten only after the next group's barriers
        if (stage < 2) {  // the group left early
            pre_head_done(a, nx);
            pre_foot<WMODE>(a, nx);
        }
        if (stage < 3) pre_cells(a, nx);
        p = nx;
        kn = knn;
    }
}

// Sum the spread partial slots into out[0..NC) (one work-group of 256
// threads; NC = 3 for {energy, virial, pairs}, 1 for the kinetic energy),
// then clear the slots it read: every evaluation leaves them zero for the
// next, so no clearing launch is needed (the workspace zeroes them once when
// it is created).  Each thread issues all its loads before the sums, so the
// work-group waits for one round trip.
constexpr int kPartPer = kPartSlots / 256;
static_assert(kPartSlots % 256 == 0, "partial slots per thread");

template <int NC>
__device__ __forceinline__ void reduce_parts_wg(long long *__restrict__ part,
                                                long long *__restrict__ out, int half = 0) {
    __shared__ long long s_w[4][NC];
    long long x[kPartPer][NC];
#pragma unroll
    for (int r = 0; r < kPartPer; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) x[r][c] = part[(threadIdx.x + 256 * r) * NC + c];
    long long v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = 0;
#pragma unroll
    for (int r = 0; r < kPartPer; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            v[c] += x[r][c];
            part[(threadIdx.x + 256 * r) * NC + c] = 0;
        }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        v[c] = wave_sum64(v[c]);
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6][c] = v[c];
    }
    __syncthreads();
    // half: every pair was counted twice (full shell), so the sum is even
    // and halves exactly
    if (threadIdx.x < NC) {
        const int c = threadIdx.x;
        out[c] = (s_w[0][c] + s_w[1][c] + s_w[2][c] + s_w[3][c]) >> half;
    }
}

template <int NC>
__global__ __launch_bounds__(256) void k_reduce_parts(long long *__restrict__ part,
                                                      long long *__restrict__ out, int half) {
    reduce_parts_wg<NC>(part, out, half);
}

// Sum of particle p's replica slots 0 .. R-1 (slot r's three components at
// pbuf[r 3n + c n + p]), two slots at a time, so that each thread has six
// loads in flight.  Callers clamp R to the schedule's replica count, so a
// stale count (from a group that gave up) cannot send the loads past the
// buffer.
__device__ __forceinline__ void sum_replicas(const long long *__restrict__ pbuf, int64_t n,
                                             int64_t p, int R, long long f[3]) {
    f[0] = f[1] = f[2] = 0;
    int r = 0;
    for (; r + 2 <= R; r += 2) {
        const long long *P = pbuf + (int64_t)r * 3 * n, *Q = P + 3 * n;
        const long long a0 = P[p], a1 = P[n + p], a2 = P[2 * n + p];
        const long long b0 = Q[p], b1 = Q[n + p], b2 = Q[2 * n + p];
        f[0] += a0 + b0;
        f[1] += a1 + b1;
        f[2] += a2 + b2;
    }
    if (r < R) {
        const long long *P = pbuf + (int64_t)r * 3 * n;
        f[0] += P[p];
        f[1] += P[n + p];
        f[2] += P[2 * n + p];
    }
}

// Buffer + reduce: F of every particle = sum of its cell's replica slots.
// With part != NULL one extra work-group (the first, dispatched before the
// others, so its serial sums do not trail the launch) sums the energy slots
// instead, which saves a launch.
__global__ __launch_bounds__(256) void k_gather_partials(
    const long long *__restrict__ pbuf, const int *__restrict__ rcnt, int rmax, int64_t n,
    long long *__restrict__ F, long long *__restrict__ part, long long *__restrict__ ew) {
    if (part && blockIdx.x == 0) {
        reduce_parts_wg<3>(part, ew);
        return;
    }
    const int64_t p = (int64_t)(blockIdx.x - (part ? 1 : 0)) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    long long f[3];
    sum_replicas(pbuf, n, p, min(rcnt[p], rmax), f);  // rcnt: p's cell's replicas (sweep)
    F[p] = f[0];
    F[n + p] = f[1];
    F[2 * n + p] = f[2];
}

// ---------------------------------------------------------------------------
// Dataflow executors: one persistent launch of single-wave task runners that
// take work units in creation order (Sec. VI strategy 2, and the mutual
// exclusion Sec. VII asks for).
// ---------------------------------------------------------------------------
// Largest cell a runner stages (LDS): CELL = 64 when the workspace's tile
// hint allows it (15 KB of LDS per runner at 256, under 4 KB at 64, so
// about three times as many runners fit a compute unit), else 256.
constexpr int kDfCell = 256;

struct DfArgs {
    const int32_t *ta, *tb;      // tasks in creation order: cells A, B
    const int32_t *seqa, *seqb;  // earlier tasks touching A, B (ORDERED)
    int64_t nunit;               // work units (tasks, or chains for NESTED)
    int64_t ntask;
    int chain;                   // tasks per unit (NESTED)
    const int32_t *cell_start;
    const uint32_t *coord;
    int64_t n;
    long long *F;
    long long *part;             // spread energy slots
    int *sync;                   // per cell: completed tasks (ORDERED) or lock
    int *ctl;                    // [0] unit ticket, [1] abort, [2] log ticket
    int *log;                    // optional: start ticket of task t at [t],
                                 // end ticket at [ntask + t]
    uint32_t *flags;
    PairParams pp;
    unsigned long long limit;    // longest wait in s_memrealtime ticks (100 MHz)
};

// Bounded wait of lane 0 for `ok(v)` on *p, or (cas) for the lock at *p to
// be free and taken (only lane 0 polls, inside a divergent branch, so the
// accesses are vector memory operations).  Gives up when another runner has
// aborted or after a.limit ticks, then aborts everyone.  Returns the outcome
// to all lanes.
template <class OK>
__device__ __forceinline__ bool df_wait(const DfArgs &a, int *p, OK ok, bool cas) {
    int got = 1;
    if (threadIdx.x == 0) {
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        for (;;) {
            if (cas) {  // test, then test-and-set
                if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                    atomicCAS(p, 0, 1) == 0)
                    break;
            } else if (ok(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                break;
            }
            if (__hip_atomic_load(&a.ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                got = 0;
                break;
            }
            if (__builtin_amdgcn_s_memrealtime() - t0 > a.limit) {
                __hip_atomic_store(&a.ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicOr(a.flags, (uint32_t)LC_FLAG_ABORT);
                got = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);  // 64 clocks between polls
        }
    }
    got = __builtin_amdgcn_readfirstlane(got);
    return got != 0;
}

// Ordered: bounded wait of lane 0 until the counters of cells A and B show
// qa and qb completed earlier tasks; both counters are read in every poll,
// so a task whose two predecessors finished long ago passes in one round
// trip.  Outcome as df_wait.
__device__ __forceinline__ bool df_wait2(const DfArgs &a, int A, int B, int qa, int qb) {
    int got = 1;
    if (threadIdx.x == 0) {
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        bool da = false, db = A == B;
        for (;;) {
            const int va = da ? qa : __hip_atomic_load(&a.sync[A], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            const int vb = db ? qb : __hip_atomic_load(&a.sync[B], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            da = va == qa;
            db = vb == qb;
            if (da && db) break;
            if (__hip_atomic_load(&a.ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                got = 0;
                break;
            }
            if (__builtin_amdgcn_s_memrealtime() - t0 > a.limit) {
                __hip_atomic_store(&a.ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicOr(a.flags, (uint32_t)LC_FLAG_ABORT);
                got = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    got = __builtin_amdgcn_readfirstlane(got);
    return got != 0;
}

// A task's inputs, loaded before the runner waits for its cells (they are
// read-only, so the loads need no order with the waits and leave the
// critical path): the two cells, their particle ranges, cell A's box
// fractions (particle lane + 64 r in register r) and the box fraction of
// cell B's particle `lane`.
template <int CELL>
struct DfPre {
    static constexpr int kPer = CELL / 64;  // particles of cell A per lane
    int A, B, sA, na, sB, nb;
    uint32_t ax[kPer], ay[kPer], az[kPer];
    uint4 ub;
};

template <int CELL>
__device__ __forceinline__ void df_load(const DfArgs &a, int64_t t, DfPre<CELL> &p) {
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    p.A = a.ta[t];
    p.B = a.tb[t];
    p.sA = a.cell_start[p.A];
    p.na = a.cell_start[p.A + 1] - p.sA;
    p.sB = a.cell_start[p.B];
    p.nb = a.cell_start[p.B + 1] - p.sB;
#pragma unroll
    for (int r = 0; r < DfPre<CELL>::kPer; ++r) {
        const int k = lane + 64 * r;
        if (k < p.na) {
            p.ax[r] = a.coord[p.sA + k];
            p.ay[r] = a.coord[n + p.sA + k];
            p.az[r] = a.coord[2 * n + p.sA + k];
        }
    }
    p.ub = make_uint4(0u, 0u, 0u, 0u);
    if (lane < p.nb)
        p.ub = make_uint4(a.coord[p.sB + lane], a.coord[n + p.sB + lane],
                          a.coord[2 * n + p.sB + lane], 0u);
}

// One cell-pair task by one wave.  A's box fractions are staged in LDS.  A
// cell B of at most 64 particles is covered by 64 / nb lane groups: lane
// (j, part) takes B's particle j and every parts-th i of A, in diagonal
// order (i = (k + j) mod na), so each (i, j) is visited once and the lanes
// of one step add into different A particles; larger cells take B 64
// particles at a time.  Intra tasks keep i before j.  Both sides accumulate
// in LDS, then go into F with device atomics: plain read-modify-writes would
// need a device-scope release and acquire around every task, which on a GPU
// of several L2 caches (one per XCD) writes back and invalidates a whole L2
// each time; integer adds commute, so the result is the same.  The caller
// waits for the adds to complete before it releases the cells.
template <int CELL>
__device__ __forceinline__ void df_task(const DfArgs &a, const DfPre<CELL> &p, uint32_t (*su)[CELL],
                                        long long (*acc)[CELL], long long (*accb)[CELL],
                                        long long &e_sum, long long &w_sum, long long &p_cnt,
                                        uint32_t &ovf) {
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int na = p.na, nb = p.nb, sA = p.sA, sB = p.sB;
    if (na > CELL || nb > CELL) {  // the host checks the tile hint first
        if (lane == 0) atomicOr(a.flags, (uint32_t)LC_FLAG_OVERFLOW);
        return;
    }
    const bool intra = p.A == p.B;
#pragma unroll
    for (int r = 0; r < DfPre<CELL>::kPer; ++r) {
        const int k = lane + 64 * r;
        if (k < na) {
            su[0][k] = p.ax[r];
            su[1][k] = p.ay[r];
            su[2][k] = p.az[r];
            acc[0][k] = acc[1][k] = acc[2][k] = 0;
        }
        if (!intra && k < nb) accb[0][k] = accb[1][k] = accb[2][k] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    long long(*accj)[CELL] = intra ? acc : accb;
    const int parts = (nb > 0 && nb <= 64) ? 64 / nb : 1;
    for (int j0 = 0; j0 < nb; j0 += 64) {
        const int jr = parts > 1 ? lane % nb : lane;  // B particle within this chunk
        const int part = parts > 1 ? lane / nb : 0;
        const int jl = j0 + jr;
        const bool vj = part < parts && jl < nb;
        uint4 uj;
        if (j0 == 0) {  // p.ub holds B's particle `lane`: fetch particle jr's
            uj.x = (uint32_t)__shfl((int)p.ub.x, jr);
            uj.y = (uint32_t)__shfl((int)p.ub.y, jr);
            uj.z = (uint32_t)__shfl((int)p.ub.z, jr);
        } else {
            uj = vj ? make_uint4(a.coord[sB + jl], a.coord[n + sB + jl],
                                 a.coord[2 * n + sB + jl], 0u)
                    : make_uint4(0u, 0u, 0u, 0u);
        }
        long long fx = 0, fy = 0, fz = 0;
        if (vj) {
            for (int k = part; k < na; k += parts) {
                int i = k + jr;
                i = i >= na ? i - na : i;
                i = i >= na ? i % na : i;
                if (intra && i >= jl) continue;
                const uint4 ui = make_uint4(su[0][i], su[1][i], su[2][i], 0u);
                long long qx, qy, qz, qe, qw;
                if (!pair_terms_fast(ui, uj, a.pp, qx, qy, qz, qe, qw, ovf)) continue;
                e_sum += qe;
                w_sum += qw;
                p_cnt += 1;
                lds_sub64(&acc[0][i], qx);
                lds_sub64(&acc[1][i], qy);
                lds_sub64(&acc[2][i], qz);
                fx += qx;
                fy += qy;
                fz += qz;
            }
            atomicAdd((unsigned long long *)&accj[0][jl], (unsigned long long)fx);
            atomicAdd((unsigned long long *)&accj[1][jl], (unsigned long long)fy);
            atomicAdd((unsigned long long *)&accj[2][jl], (unsigned long long)fz);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (int k = lane; k < na; k += 64) {
        atomicAdd((unsigned long long *)&a.F[sA + k], (unsigned long long)acc[0][k]);
        atomicAdd((unsigned long long *)&a.F[n + sA + k], (unsigned long long)acc[1][k]);
        atomicAdd((unsigned long long *)&a.F[2 * n + sA + k], (unsigned long long)acc[2][k]);
    }
    if (!intra) {
        for (int k = lane; k < nb; k += 64) {
            atomicAdd((unsigned long long *)&a.F[sB + k], (unsigned long long)accb[0][k]);
            atomicAdd((unsigned long long *)&a.F[n + sB + k], (unsigned long long)accb[1][k]);
            atomicAdd((unsigned long long *)&a.F[2 * n + sB + k], (unsigned long long)accb[2][k]);
        }
    }
}

// A ticket of the log counter for task t's start (end: at[ntask + t]),
// taken by lane 0.  The atomic returns its value before anything after it
// is issued, so the ticket order follows the order in which the runners
// passed these points.
__device__ __forceinline__ void df_ticket(const DfArgs &a, int64_t at) {
    if (a.log && threadIdx.x == 0) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        a.log[at] = atomicAdd(&a.ctl[2], 1);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
}

// MODE 0: ordered (sequence counters), 1: mutual exclusion per task,
// 2: nested (a chain per unit, mutual exclusion per task).  CELL: the
// largest cell staged (64 or 256 particles).
template <int MODE, int CELL>
__global__ __launch_bounds__(64) void k_dataflow(DfArgs a) {
    __shared__ uint32_t su[3][CELL];
    __shared__ long long acc[3][CELL];
    __shared__ long long accb[3][CELL];
    const int lane = threadIdx.x;
    long long e_sum = 0, w_sum = 0, p_cnt = 0;
    uint32_t ovf = 0;
    bool stop = false;
    // Units come from one counter in creation order, a runner taking its
    // next ticket when its unit is done: ordered, one task per ticket (a
    // runner blocked on one task then holds back no other); mutex, 8
    // consecutive tasks per ticket (consecutive tasks often share a cell,
    // and the counter sees fewer atomics); nested, one chain per ticket.
    // Every unit held belongs to a running runner, and the smallest
    // unfinished one is its runner's current unit with all its predecessors
    // done, so the ordered waits always progress; locks are taken lower cell
    // first, so mutual exclusion cannot deadlock either.
    constexpr int kBatch = MODE == 1 ? 8 : 1;
    int64_t unit = 0, uend = 0;
    while (!stop) {
        if (unit == uend) {
            int u = 0;
            if (lane == 0) u = atomicAdd(&a.ctl[0], kBatch);
            unit = __builtin_amdgcn_readfirstlane(u);
            uend = unit + kBatch;
        }
        if (unit >= a.nunit) break;
        const int64_t t0 = MODE == 2 ? unit * a.chain : unit;
        const int64_t t1 = MODE == 2 ? t0 + a.chain : t0 + 1;
        ++unit;
        for (int64_t t = t0; t < t1; ++t) {
            DfPre<CELL> p;
            df_load<CELL>(a, t, p);  // in flight while the cells are awaited
            const int A = p.A, B = p.B;
            const int lo = A < B ? A : B, hi = A < B ? B : A;
            if constexpr (MODE == 0) {
                if (!df_wait2(a, A, B, a.seqa[t], a.seqb[t])) {
                    stop = true;
                    break;
                }
            } else {
                auto any = [](int) { return true; };
                if (!df_wait(a, &a.sync[lo], any, true)) {
                    stop = true;
                    break;
                }
                if (hi != lo && !df_wait(a, &a.sync[hi], any, true)) {
                    if (lane == 0) __hip_atomic_store(&a.sync[lo], 0, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                    stop = true;
                    break;
                }
            }
            df_ticket(a, t);
            df_task<CELL>(a, p, su, acc, accb, e_sum, w_sum, p_cnt, ovf);
            // the task has finished when its force adds have completed:
            // wait for them (the whole wave's memory operations) before the
            // end ticket and the release
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_waitcnt(0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            df_ticket(a, a.ntask + t);
            if (lane == 0) {
                if constexpr (MODE == 0) {
                    atomicAdd(&a.sync[A], 1);
                    if (B != A) atomicAdd(&a.sync[B], 1);
                } else {
                    if (hi != lo)
                        __hip_atomic_store(&a.sync[hi], 0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&a.sync[lo], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    e_sum = wave_sum64(e_sum);
    w_sum = wave_sum64(w_sum);
    p_cnt = wave_sum64(p_cnt);
    if (lane == 0) {
        long long *dst = &a.part[(blockIdx.x % kPartSlots) * 3];
        atomicAdd((unsigned long long *)&dst[0], (unsigned long long)e_sum);
        atomicAdd((unsigned long long *)&dst[1], (unsigned long long)w_sum);
        atomicAdd((unsigned long long *)&dst[2], (unsigned long long)p_cnt);
    }
    if (__ballot(ovf != 0u) && lane == 0) atomicOr(a.flags, (uint32_t)LC_FLAG_OVERFLOW);
}

// A phase with more groups than the device holds at once runs persistent:
// as many work-groups as fit (occupancy x compute units), each drawing
// groups from the phase's ticket counter, which the caller has zeroed.
// Otherwise one work-group per group.
template <int CAP, int WMODE, bool F64, bool FF>
static int launch_sweep_t(SweepArgs a, int ngroups, int ncu, int *ticket, hipStream_t st) {
    static int per_cu = 0;  // resident work-groups per compute unit (0: not known yet)
    int res = per_cu;
    if (res == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(&k_sweep<CAP, WMODE, F64, FF>), kWG, 0) ==
                hipSuccess &&
            nb >= 1)
            per_cu = res = nb;
        else
            res = 1;  // query refused (e.g. during capture): one per CU, not cached
    }
    int grid = ngroups;
    a.ticket = nullptr;
    a.ngroups = ngroups;
    if (ticket && ngroups > res * ncu) {
        grid = res * ncu;
        a.ticket = ticket;
    }
    hipLaunchKernelGGL((k_sweep<CAP, WMODE, F64, FF>), dim3(grid), dim3(kWG), 0, st, a);
    LAUNCHCHK("k_sweep");
    return LC_OK;
}

// LDS tile capacities (particles): with the integer filter {512, 768, 1024,
// 2048}, without {1024, 2048, 3072}.
template <int WMODE, bool F64, bool FF>
static int launch_sweep_c(int cap, const SweepArgs &a, int ng, int ncu, int *tk, hipStream_t st) {
    if constexpr (FF) {
        if (cap <= 512) return launch_sweep_t<512, WMODE, F64, true>(a, ng, ncu, tk, st);
        if (cap <= 768) return launch_sweep_t<768, WMODE, F64, true>(a, ng, ncu, tk, st);
        if (cap <= 1024) return launch_sweep_t<1024, WMODE, F64, true>(a, ng, ncu, tk, st);
        return launch_sweep_t<2048, WMODE, F64, true>(a, ng, ncu, tk, st);
    } else {
        if (cap <= 1024) return launch_sweep_t<1024, WMODE, F64, false>(a, ng, ncu, tk, st);
        if (cap <= 2048) return launch_sweep_t<2048, WMODE, F64, false>(a, ng, ncu, tk, st);
        return launch_sweep_t<3072, WMODE, F64, false>(a, ng, ncu, tk, st);
    }
}

static int launch_sweep(int cap, int wmode, bool f64, bool ff, const SweepArgs &a, int ng,
                        int ncu, int *tk, hipStream_t st) {
    if (f64) {
        if (wmode == 0) return launch_sweep_c<0, true, false>(cap, a, ng, ncu, tk, st);
        if (wmode == 1) return launch_sweep_c<1, true, false>(cap, a, ng, ncu, tk, st);
        if (wmode == 3) return launch_sweep_c<3, true, false>(cap, a, ng, ncu, tk, st);
        if (wmode == 4) return launch_sweep_c<4, true, false>(cap, a, ng, ncu, tk, st);
        return launch_sweep_c<2, true, false>(cap, a, ng, ncu, tk, st);
    }
    if (ff) {
        if (wmode == 0) return launch_sweep_c<0, false, true>(cap, a, ng, ncu, tk, st);
        if (wmode == 1) return launch_sweep_c<1, false, true>(cap, a, ng, ncu, tk, st);
        if (wmode == 3) return launch_sweep_c<3, false, true>(cap, a, ng, ncu, tk, st);
        if (wmode == 4) return launch_sweep_c<4, false, true>(cap, a, ng, ncu, tk, st);
    }
    if (wmode == 0) return launch_sweep_c<0, false, false>(cap, a, ng, ncu, tk, st);
    if (wmode == 1) return launch_sweep_c<1, false, false>(cap, a, ng, ncu, tk, st);
    if (wmode == 3) return launch_sweep_c<3, false, false>(cap, a, ng, ncu, tk, st);
    if (wmode == 4) return launch_sweep_c<4, false, false>(cap, a, ng, ncu, tk, st);
    return launch_sweep_c<2, false, false>(cap, a, ng, ncu, tk, st);
}

// Bound of the integer candidate filter.  A coordinate's top 16 bits differ
// between two particles by the exact minimum-image difference in units of
// L/2^16 to within one unit, so a pair inside the cutoff has a 16-bit
// squared distance below (rc/u + sqrt 3)^2, u the smallest axis unit; the
// bound uses rc slightly enlarged (the canonical FP32 r2 may round below the
// exact one) and +2 units.  0: the filter is not used (axes whose units
// differ by more than 25% would make the superset needlessly wide).
static int filter16_bound(const double box[3], float rc2, bool flat = false) {
    // a flat system's z differences are all zero: only x and y set the units
    const double bz = flat ? box[0] : box[2];
    const double umin = std::min(box[0], std::min(box[1], bz)) / 65536.0;
    const double umax = std::max(box[0], std::max(box[1], bz)) / 65536.0;
    if (!(umin > 0.0) || umax > 1.25 * umin) return 0;
    const double ru = std::sqrt((double)rc2) * (1.0 + 1e-5) / umin + 2.0;
    const double t = std::ceil(ru * ru) + 1.0;
    return t < 2.0e9 ? (int)t : 0;
}

static PairParams pair_params(const lc_grid *g) {
    PairParams p;
    for (int d = 0; d < 3; ++d) {
        p.s[d] = g->scale[d];
        p.sd[d] = g->box[d] / 4294967296.0;
    }
    p.rc2 = g->rc2;
    p.thr16 = filter16_bound(g->box, g->rc2, g->nc[2] == 1);
    p.ecut = g->ecut;
    p.rc2d = g->rc * g->rc;
    const double ic = 1.0 / p.rc2d;
    const double s6 = ic * ic * ic;
    p.ecutd = 4.0 * s6 * (s6 - 1.0);
    return p;
}

// Footprint entries as the sweep reads them: with buffer + reduce, the
// replica slot | (the cell's replica count << 16); otherwise as built.
static std::vector<int32_t> device_foot_rep(const lcs::HostSchedule &h) {
    std::vector<int32_t> out(h.foot_rep);
    if (h.write_mode == 3)
        for (size_t f = 0; f < out.size(); ++f)
            out[f] |= h.cell_rep[(size_t)h.foot_cells[f]] << 16;
    return out;
}

// Buffer + reduce scratch: rmax replica slots of 3 x n int64, then n int32
// replica counts.
static int64_t pbuf_elems(int rmax, int64_t n) { return (int64_t)rmax * 3 * n + (n + 1) / 2; }
static int *rcnt_of(lc_workspace *ws, int rmax, int64_t n) {
    return (int *)(ws->pbuf + (int64_t)rmax * 3 * n);
}

static int ensure_pbuf(lc_workspace *ws, int64_t need) {
    if (need <= ws->pbuf_elems) return LC_OK;
    // a captured graph holds the current buffer's address
    if (ws->live_graphs > 0)
        return fail(LC_ECAPACITY,
                    "the workspace's replica buffer would have to grow (%lld -> %lld elements) "
                    "while %d graph(s) captured with it are alive",
                    (long long)ws->pbuf_elems, (long long)need, ws->live_graphs);
    (void)hipFree(ws->pbuf);
    ws->pbuf = nullptr;
    ws->pbuf_elems = 0;
    int rc = dalloc(&ws->pbuf, need);
    if (rc) return rc;
    ws->pbuf_elems = need;
    return LC_OK;
}

// Device memory a force evaluation uses beyond its inputs and outputs: the
// spread energy slots (zero on entry, left zero), the status word, the
// replica buffer of buffer + reduce (pbuf_elems(rmax, n) elements, only read
// for that kind) and the tile sizing hint.
struct SweepScratch {
    long long *part;
    uint32_t *flags;
    long long *pbuf;
    int32_t max_per_cell;
};

// gather = false (buffer + reduce only): leave the replica slots and the
// energy slots for the caller to sum (the Verlet loop folds both into its
// kick pass); F and ew are not written.
static int forces_run(const lc_grid *g, const lc_schedule *s, const int32_t *cell_start,
                      const uint32_t *coord, int64_t n, int64_t *F, int64_t *ew, int precision,
                      const SweepScratch &sc, hipStream_t st, hipEvent_t *ev,
                      bool gather = true) {
    const bool buffered = s->h.write_mode == 3;
    const bool fullshell = s->h.write_mode == 4;  // writes every particle itself
    int rc = (buffered || fullshell) ? LC_OK : fill64((long long *)F, 3 * n, st);
    if (rc) return rc;
    const int nphase = (int)s->h.phase_grp.size() - 1;
    SweepArgs a;
    a.grp_task = s->grp_task;
    a.grp_foot = s->grp_foot;
    a.foot_cells = s->foot_cells;
    a.task_ab = s->task_ab;
    a.cell_start = cell_start;
    a.coord = coord;
    a.n = n;
    a.F = (long long *)F;
    a.foot_rep = s->foot_rep;
    a.pbuf = sc.pbuf;
    a.rcnt = buffered ? (int *)(sc.pbuf + (int64_t)s->h.rmax * 3 * n) : nullptr;
    a.fx_task = s->fx_task;
    a.fx_foot = s->fx_foot;
    a.fx_rep = s->fx_rep;
    a.fx_cnt = s->fx_cnt;
    a.fx_tmax = s->fx_tmax;
    a.fx_fmax = s->fx_fmax;
    a.part = sc.part;
    a.grp_box = nullptr;
    a.ppar = nullptr;
    a.ew_box = nullptr;
    a.ticket = nullptr;
    a.ngroups = 0;
    a.flags = sc.flags;
    a.pp = pair_params(g);
    // LDS tile: expected particles of the largest footprint with headroom
    const double mean = g->ncell > 0 ? (double)n / (double)g->ncell : 0.0;
    // the filter stages cells of up to kFFCell particles; denser cells take
    // the unfiltered kernel rather than the global fallback
    const int32_t hint = sc.max_per_cell;
    const bool dense = hint > 0 ? hint > kFFCell : mean > 0.5 * kFFCell;
    const bool ff = a.pp.thr16 > 0 && precision == LC_PREC_FP32 && s->h.write_mode != 2 && !dense;
    // (a load-aware schedule knows its largest footprint exactly for the
    // counts it was built from: a tile that holds it, no larger; otherwise
    // 80% of the footprint's cells all at the largest cell, but at least
    // the mean footprint with 15% to spare)
    const double need =
        s->foot_max > 0 ? (double)s->foot_max
        : hint > 0 ? std::max((double)hint * s->h.max_cells * 0.8, mean * s->h.max_cells * 1.15)
                   : mean * s->h.max_cells * 1.35;
    int cap;
    if (ff)
        cap = need <= 512 ? 512 : need <= 768 ? 768 : (need <= 1024 ? 1024 : 2048);
    else
        cap = need <= 1024 ? 1024 : (need <= 2048 ? 2048 : 3072);
    for (int p = 0; p < nphase; ++p) {
        const int ng = s->h.phase_grp[p + 1] - s->h.phase_grp[p];
        if (ng <= 0) continue;
        a.grp_base = s->h.phase_grp[p];
        if (ev) HIPCHK(hipEventRecord(ev[2 * p], st));
        // one work-group per group: the hardware refills a compute unit as
        // soon as a group ends, which balances better than a persistent loop
        rc = launch_sweep(cap, s->h.write_mode, precision == LC_PREC_FP64, ff && need <= 2048, a,
                          ng, s->ncu, nullptr, st);
        if (rc) return rc;
        if (ev) HIPCHK(hipEventRecord(ev[2 * p + 1], st));
    }
    if (ev) HIPCHK(hipEventRecord(ev[2 * nphase], st));
    if (buffered && n > 0) {  // gather + the energy sums in one launch
        if (gather) {
            hipLaunchKernelGGL(k_gather_partials, dim3((unsigned)((n + 255) / 256 + 1)),
                               dim3(256), 0, st, (const long long *)sc.pbuf,
                               (const int *)a.rcnt, s->h.rmax, n, (long long *)F, sc.part,
                               (long long *)ew);
            LAUNCHCHK("k_gather_partials");
        }
    } else {
        hipLaunchKernelGGL(k_reduce_parts<3>, dim3(1), dim3(256), 0, st, sc.part,
                           (long long *)ew, fullshell ? 1 : 0);
        LAUNCHCHK("k_reduce_parts");
    }
    if (ev) HIPCHK(hipEventRecord(ev[2 * nphase + 1], st));
    return LC_OK;
}

// A force evaluation with the workspace's scratch; buffer + reduce grows
// the workspace's replica buffer on first use.
static int forces_impl(const lc_grid *g, const lc_schedule *s, const int32_t *cell_start,
                       const uint32_t *coord, int64_t n, int64_t *F, int64_t *ew, int precision,
                       lc_workspace *ws, hipStream_t st, hipEvent_t *ev = nullptr,
                       bool gather = true) {
    if (s->h.write_mode == 3) {
        int rc = ensure_pbuf(ws, pbuf_elems(s->h.rmax, n));
        if (rc) return rc;
    }
    SweepScratch sc;
    sc.part = (long long *)ws->part;
    sc.flags = ws->flags;
    sc.pbuf = ws->pbuf;
    sc.max_per_cell = ws->max_per_cell;
    return forces_run(g, s, cell_start, coord, n, F, ew, precision, sc, st, ev, gather);
}

// ---------------------------------------------------------------------------
// a7: Verlet
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_kick_ke(double *__restrict__ vel,
                                                 const long long *__restrict__ F, int64_t n,
                                                 double hdt, int kick,
                                                 unsigned long long *__restrict__ part) {
    __shared__ long long s_w[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long q = 0;
    if (i < n) {
        double v[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * n + i;
            double x = vel[k];
            if (kick) {
                const double acc = (double)F[k] * (1.0 / 4294967296.0);
                x = x + hdt * acc;
                vel[k] = x;
            }
            v[d] = x;
        }
        double s = v[0] * v[0] + v[1] * v[1];
        s = s + v[2] * v[2];
        q = (long long)rint((s * 0.5) * 4294967296.0);
    }
    q = wave_sum64(q);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        atomicAdd(&part[blockIdx.x % kPartSlots], (unsigned long long)t);
    }
}

// The closing half kick of one step (with its kinetic energy, as k_kick_ke)
// fused with the opening half kick and drift of the next:
// both half kicks take the same forces, so one pass reads F, v, x and x_ref
// once.  Per particle the arithmetic is the two kernels' own, in their
// order, so the trajectory is bit-identical to running them one after the
// other.
__global__ __launch_bounds__(256) void k_kick_ke_drift(
    double *__restrict__ pos, double *__restrict__ vel, const long long *__restrict__ F, int64_t n,
    double hdt, double dt, int kick, const double *__restrict__ xref, double lim2, GridArgs ga,
    uint32_t *__restrict__ coord, uint32_t *__restrict__ flags,
    unsigned long long *__restrict__ part) {
    __shared__ long long s_w[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long q = 0;
    if (i < n) {
        double v[3], acc[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * n + i;
            acc[d] = (double)F[k] * (1.0 / 4294967296.0);
            double x = vel[k];
            if (kick) x = x + hdt * acc[d];
            v[d] = x;
        }
        double s = v[0] * v[0] + v[1] * v[1];
        s = s + v[2] * v[2];
        q = (long long)rint((s * 0.5) * 4294967296.0);
        double r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * n + i;
            const double w = v[d] + hdt * acc[d];
            double x = pos[k];
            x = x + dt * w;
            vel[k] = w;
            pos[k] = x;
            coord[k] = canon(x, ga.inv[d]);
            const double dd = x - xref[k];
            r2 += dd * dd;
        }
        if (r2 > lim2) atomicOr(flags, (uint32_t)LC_FLAG_DISP);
    }
    q = wave_sum64(q);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        atomicAdd(&part[blockIdx.x % kPartSlots], (unsigned long long)t);
    }
}

// k_kick_ke_drift for buffer + reduce schedules, with the gather folded in:
// each particle's forces are the sum of its cell's replica slots (as
// k_gather_partials sums them), read here instead of F, so the pass that
// would write F and the read of it are gone.  The first work-group sums the
// energy slots into ew (as the gather launch's extra work-group does); the
// kinetic energy goes to its own slots.
__global__ __launch_bounds__(256) void k_gather_kick_ke_drift(
    const long long *__restrict__ pbuf, const int *__restrict__ rcnt, int rmax, int64_t n,
    double *__restrict__ pos, double *__restrict__ vel, double hdt, double dt, int kick,
    const double *__restrict__ xref, double lim2, GridArgs ga, uint32_t *__restrict__ coord,
    uint32_t *__restrict__ flags, unsigned long long *__restrict__ kpart,
    long long *__restrict__ part, long long *__restrict__ ew) {
    if (blockIdx.x == 0) {
        reduce_parts_wg<3>(part, ew);
        return;
    }
    __shared__ long long s_w[4];
    const int64_t i = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
    long long q = 0;
    if (i < n) {
        long long f[3];
        sum_replicas(pbuf, n, i, min(rcnt[i], rmax), f);
        double v[3], acc[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * n + i;
            acc[d] = (double)f[d] * (1.0 / 4294967296.0);
            double x = vel[k];
            if (kick) x = x + hdt * acc[d];
            v[d] = x;
        }
        double s = v[0] * v[0] + v[1] * v[1];
        s = s + v[2] * v[2];
        q = (long long)rint((s * 0.5) * 4294967296.0);
        double r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const int64_t k = d * n + i;
            const double w = v[d] + hdt * acc[d];
            double x = pos[k];
            x = x + dt * w;
            vel[k] = w;
            pos[k] = x;
            coord[k] = canon(x, ga.inv[d]);
            const double dd = x - xref[k];
            r2 += dd * dd;
        }
        if (r2 > lim2) atomicOr(flags, (uint32_t)LC_FLAG_DISP);
    }
    q = wave_sum64(q);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        atomicAdd(&kpart[(blockIdx.x - 1) % kPartSlots], (unsigned long long)t);
    }
}

__global__ void k_copy64(const long long *__restrict__ src, long long *__restrict__ dst, int cnt) {
    if ((int)threadIdx.x < cnt) dst[threadIdx.x] = src[threadIdx.x];
}

__global__ void k_gather(const int *__restrict__ perm, int64_t n, const double *__restrict__ in,
                         double *__restrict__ out, const int *__restrict__ in_ids,
                         int *__restrict__ out_ids) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t s = perm[k];
    out[k] = in[s];
    out[n + k] = in[n + s];
    out[2 * n + k] = in[2 * n + s];
    if (in_ids) out_ids[k] = in_ids[s];
}

static int gather_impl(const int32_t *perm, int64_t n, const double *in3, double *out3,
                       const int32_t *in_ids, int32_t *out_ids, hipStream_t st) {
    if (n <= 0) return LC_OK;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm, n, in3,
                       out3, in_ids, out_ids);
    LAUNCHCHK("k_gather");
    return LC_OK;
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

// Stencil reach of a grid (grids filled before the field existed read 0).
static int grid_reach(const lc_grid *g) { return g->reach > 1 ? 2 : 1; }

extern "C" int lc_make_grid(const double box[3], double rc, double skin, int flags,
                            lc_grid *out) {
    if (!box || !out) return fail(LC_EINVAL, "lc_make_grid: null argument");
    if (!(rc > 0.0) || !(skin >= 0.0)) return fail(LC_EINVAL, "lc_make_grid: rc/skin");
    const bool flat = (flags & LC_GRID_2D) != 0;
    if (flat && (flags & LC_GRID_HALF))
        return fail(LC_EINVAL, "lc_make_grid: LC_GRID_2D with LC_GRID_HALF");
    lc_grid g;
    memset(&g, 0, sizeof g);
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (!(box[d] > 0.0)) return fail(LC_EINVAL, "lc_make_grid: box length");
        g.box[d] = box[d];
        g.inv_box[d] = 1.0 / box[d];
        const int reach = (flags & LC_GRID_HALF) ? 2 : 1;
        const double side = (rc * (1.0 + 1.0 / 4096.0) + skin) / reach;
        const double q = box[d] / side;
        if (!(q < 2147483647.0)) return fail(LC_EINVAL, "lc_make_grid: too many cells");
        int64_t k = (int64_t)q;
        if ((flags & LC_GRID_EVEN) && (k & 1)) k -= 1;
        if (flat && d == 2) k = 1;  // the flat axis: one cell
        else if (k < 2 * reach + 1)
            return fail(LC_EINVAL, "lc_make_grid: axis %d gets %lld cells (< %d)", d, (long long)k,
                        2 * reach + 1);
        g.nc[d] = (int32_t)k;
        ncell *= k;
        g.scale[d] = (float)(box[d] / 4294967296.0);
    }
    if (ncell >= 2147483647LL) return fail(LC_EINVAL, "lc_make_grid: too many cells");
    g.ncell = (int32_t)ncell;
    g.rc = rc;
    g.skin = skin;
    g.reach = (flags & LC_GRID_HALF) ? 2 : 1;
    g.rc2 = (float)(rc * rc);
    {
        float inv = 1.0f / g.rc2;
        float s6 = inv * inv;
        s6 = s6 * inv;
        float e = 4.0f * s6;
        g.ecut = e * (s6 - 1.0f);
    }
    *out = g;
    return LC_OK;
}


extern "C" void lc_workspace_destroy(lc_workspace *ws) {
    if (!ws) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ws->device);
    (void)hipFree(ws->counts);
    (void)hipFree(ws->flags);
    (void)hipFree(ws->ew);
    (void)hipFree(ws->part);
    (void)hipFree(ws->kpart);
    (void)hipFree(ws->ke);
    (void)hipFree(ws->xref);
    (void)hipFree(ws->tmp3);
    (void)hipFree(ws->tmpi);
    (void)hipFree(ws->df_sync);
    (void)hipFree(ws->df_ctl);
    (void)hipFree(ws->pbuf);
    (void)hipFree(ws->lb_status);
    (void)hipFree(ws->lb_done);
    (void)hipSetDevice(cur);
    delete ws;
}

extern "C" int lc_workspace_create(int64_t max_n, int64_t max_cells, lc_workspace **out) {
    if (!out || max_n < 0 || max_cells < 1 || max_cells >= 2147483647LL || max_n >= 2147483647LL)
        return fail(LC_EINVAL, "lc_workspace_create: bad sizes");
    lc_workspace *ws = new lc_workspace();
    HIPCHK(hipGetDevice(&ws->device));
    ws->max_n = max_n;
    ws->max_cells = max_cells;
    ws->lb_tiles = (max_cells + kLbTile - 1) / kLbTile;
    int rc = 0;
    if ((rc = dalloc(&ws->counts, max_cells)) ||
        (rc = dalloc(&ws->flags, 1)) || (rc = dalloc(&ws->ew, 3)) ||
        (rc = dalloc(&ws->part, 3 * kPartSlots)) || (rc = dalloc(&ws->kpart, kPartSlots)) ||
        (rc = dalloc(&ws->ke, 1)) ||
        (rc = dalloc(&ws->xref, 3 * max_n)) || (rc = dalloc(&ws->tmp3, 3 * max_n)) ||
        (rc = dalloc(&ws->tmpi, max_n)) ||
        (rc = dalloc(&ws->lb_status, (max_cells + kLbTile - 1) / kLbTile)) ||
        (rc = dalloc(&ws->lb_done, 1))) {
        lc_workspace_destroy(ws);
        return rc;
    }
    if (hipMemset(ws->flags, 0, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(ws->part, 0, 3 * kPartSlots * sizeof(int64_t)) != hipSuccess ||
        hipMemset(ws->kpart, 0, kPartSlots * sizeof(int64_t)) != hipSuccess ||
        hipMemset(ws->counts, 0, (size_t)max_cells * sizeof(int)) != hipSuccess ||
        hipMemset(ws->lb_status, 0,
                  (size_t)((max_cells + kLbTile - 1) / kLbTile) * sizeof(unsigned long long)) !=
            hipSuccess ||
        hipMemset(ws->lb_done, 0, sizeof(int32_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        lc_workspace_destroy(ws);
        return fail(LC_EHIP, "lc_workspace_create: clearing the workspace");
    }
    *out = ws;
    return LC_OK;
}

extern "C" int lc_workspace_set_tile_hint(lc_workspace *ws, int32_t max_per_cell) {
    if (!ws || max_per_cell < 0) return fail(LC_EINVAL, "lc_workspace_set_tile_hint");
    ws->max_per_cell = max_per_cell;
    return LC_OK;
}

extern "C" int lc_workspace_clear_status(lc_workspace *ws, void *stream) {
    if (!ws) return fail(LC_EINVAL, "null workspace");
    // also the energy slots, which a failed evaluation may have left dirty,
    // and the cell build's counters and scan status words, which an
    // abandoned scan may have left set
    hipStream_t st = (hipStream_t)stream;
    int rc = fill64((long long *)ws->part, 3 * kPartSlots, st);
    if (!rc) rc = fill64((long long *)ws->kpart, kPartSlots, st);
    if (!rc) rc = fill32((int *)ws->flags, 1, st);
    if (!rc) rc = fill32(ws->counts, ws->max_cells, st);
    if (!rc) rc = fill64((long long *)ws->lb_status, ws->lb_tiles, st);
    if (!rc) rc = fill32(ws->lb_done, 1, st);
    return rc;
}

extern "C" int lc_workspace_status(lc_workspace *ws, void *stream, uint32_t *flags) {
    if (!ws || !flags) return fail(LC_EINVAL, "null argument");
    uint32_t v = 0;
    HIPCHK(hipMemcpyAsync(&v, ws->flags, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    *flags = v;
    return LC_OK;
}

extern "C" int lc_workspace_check(lc_workspace *ws, void *stream) {
    uint32_t f = 0;
    int rc = lc_workspace_status(ws, stream, &f);
    if (rc) return rc;
    if (f & LC_FLAG_OVERFLOW)
        return fail(LC_EOVERFLOW, "a quantised pair term left the fixed-point range (or r2 == 0)");
    if (f & LC_FLAG_ABORT)
        return fail(LC_EABORT, "a dataflow wait expired: the evaluation was abandoned");
    if (f & LC_FLAG_DISP)
        return fail(LC_EDISP, "a particle moved more than skin / 2 since the last cell rebuild");
    return LC_OK;
}

static int check_ws(const lc_workspace *ws, int64_t n, int64_t ncell) {
    if (!ws) return fail(LC_EINVAL, "null workspace");
    if (n > ws->max_n || ncell > ws->max_cells)
        return fail(LC_ECAPACITY, "workspace too small: n %lld > %lld or cells %lld > %lld",
                    (long long)n, (long long)ws->max_n, (long long)ncell,
                    (long long)ws->max_cells);
    return LC_OK;
}

extern "C" int lc_build_cells(const lc_grid *g, const double *pos, int64_t n, int32_t *cell_start,
                              int32_t *perm, uint32_t *coord, lc_workspace *ws, void *stream) {
    if (!g || (n > 0 && (!pos || !perm || !coord)) || !cell_start)
        return fail(LC_EINVAL, "lc_build_cells: null argument");
    if (n < 0 || n >= 2147483647LL) return fail(LC_EINVAL, "lc_build_cells: bad n");
    int rc = check_ws(ws, n, g->ncell);
    if (rc) return rc;
    return build_cells_impl(g, pos, n, cell_start, perm, coord, ws, (hipStream_t)stream);
}

extern "C" int lc_gather(const int32_t *perm, int64_t n, const double *in3, double *out3,
                         const int32_t *in_ids, int32_t *out_ids, void *stream) {
    if (n > 0 && (!perm || !in3 || !out3 || in3 == out3))
        return fail(LC_EINVAL, "lc_gather: bad arguments");
    if ((in_ids == nullptr) != (out_ids == nullptr)) return fail(LC_EINVAL, "lc_gather: ids");
    return gather_impl(perm, n, in3, out3, in_ids, out_ids, (hipStream_t)stream);
}

extern "C" int lc_make_schedule(const lc_grid *g, int kind, const int8_t *offsets, int n,
                                lc_schedule **out) {
    return lc_make_schedule_ex(g, kind, offsets, n, nullptr, out);
}

static int make_schedule_impl(const lc_grid *g, int kind, const int8_t *offsets, int n,
                              const int32_t *block_min, const int32_t *cell_counts,
                              lc_schedule **out) {
    if (!g || !out) return fail(LC_EINVAL, "lc_make_schedule: null argument");
    if (kind < 0 || kind >= LC_SCHED_COUNT) return fail(LC_EINVAL, "unknown schedule kind %d", kind);
    lc_schedule *s = new lc_schedule();
    for (int d = 0; d < 3; ++d) s->nc[d] = g->nc[d];
    std::string err;
    int rc = lcs::build_schedule(g->nc, kind, offsets, n, s->h, err, block_min, grid_reach(g));
    if (rc) {
        delete s;
        return fail(rc, "lc_make_schedule: %s", err.c_str());
    }
    if (cell_counts) {
        for (int64_t c = 0; c < g->ncell; ++c)
            if (cell_counts[c] < 0) {
                delete s;
                return fail(LC_EINVAL, "lc_make_schedule_weighted: negative count in cell %lld",
                            (long long)c);
            }
        lcs::order_groups_by_work(s->h, cell_counts);
        const int ngrp = (int)s->h.grp_foot.size() - 1;
        for (int k = 0; k < ngrp; ++k) {
            int64_t np = 0;
            for (int f = s->h.grp_foot[k]; f < s->h.grp_foot[k + 1]; ++f)
                np += cell_counts[s->h.foot_cells[(size_t)f]];
            s->foot_max = std::max(s->foot_max, np);
        }
    }
    if (!lcs::validate(s->h, g->ncell, err)) {
        delete s;
        return fail(LC_ESCHED, "lc_make_schedule: %s", err.c_str());
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(LC_EHIP, "hipGetDevice");
    }
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device) ==
                hipSuccess &&
            ncu > 0)
            s->ncu = ncu;
    }
    auto up = [&](auto **dst, const auto &vec) -> int {
        int r = dalloc(dst, (int64_t)vec.size());
        if (r) return r;
        if (!vec.empty() && hipMemcpy(*dst, vec.data(), sizeof(vec[0]) * vec.size(),
                                      hipMemcpyHostToDevice) != hipSuccess)
            return fail(LC_EHIP, "schedule upload");
        return LC_OK;
    };
    if ((rc = up(&s->grp_task, s->h.grp_task)) || (rc = up(&s->grp_foot, s->h.grp_foot)) ||
        (rc = up(&s->foot_cells, s->h.foot_cells)) || (rc = up(&s->task_ab, s->h.task_ab)) ||
        (rc = up(&s->foot_rep, device_foot_rep(s->h)))) {
        lc_schedule_free(s);
        return rc;
    }
    {
        // fixed-stride copy of the group tables when the padding costs at
        // most half again the tables themselves (near-uniform groups)
        const lcs::HostSchedule &h = s->h;
        const size_t ng = h.grp_task.size() - 1;
        int tmax = 0, fmax = 0;
        for (size_t q = 0; q < ng; ++q) {
            tmax = std::max(tmax, h.grp_task[q + 1] - h.grp_task[q]);
            fmax = std::max(fmax, h.grp_foot[q + 1] - h.grp_foot[q]);
        }
        const size_t padded = ng * (size_t)(tmax + 2 * fmax);
        const size_t actual = h.task_ab.size() + 2 * h.foot_cells.size();
        if (ng > 0 && tmax > 0 && 2 * padded <= 3 * actual) {
            const std::vector<int32_t> drep = device_foot_rep(h);
            std::vector<uint32_t> ft(ng * (size_t)tmax, 0u);
            std::vector<int32_t> ff(ng * (size_t)fmax, -1), fr(ng * (size_t)fmax, 0), fc(2 * ng);
            for (size_t q = 0; q < ng; ++q) {
                const int t0 = h.grp_task[q], nt = h.grp_task[q + 1] - t0;
                const int f0 = h.grp_foot[q], nf = h.grp_foot[q + 1] - f0;
                for (int t = 0; t < nt; ++t) ft[q * tmax + t] = h.task_ab[(size_t)(t0 + t)];
                for (int f = 0; f < nf; ++f) {
                    ff[q * fmax + f] = h.foot_cells[(size_t)(f0 + f)];
                    if (!drep.empty()) fr[q * fmax + f] = drep[(size_t)(f0 + f)];
                }
                fc[2 * q] = nt;
                fc[2 * q + 1] = nf;
            }
            if ((rc = up(&s->fx_task, ft)) || (rc = up(&s->fx_foot, ff)) ||
                (rc = up(&s->fx_rep, fr)) || (rc = up(&s->fx_cnt, fc))) {
                lc_schedule_free(s);
                return rc;
            }
            s->fx_tmax = tmax;
            s->fx_fmax = fmax;
        }
    }
    if (!s->h.order_a.empty()) {  // creation-order kind: the dataflow task list
        const size_t nt = s->h.order_a.size();
        std::vector<int32_t> seen((size_t)g->ncell, 0), sa(nt), sb(nt);
        for (size_t t = 0; t < nt; ++t) {
            const int32_t a = s->h.order_a[t], b = s->h.order_b[t];
            sa[t] = seen[(size_t)a];
            sb[t] = seen[(size_t)b];
            seen[(size_t)a]++;
            if (b != a) seen[(size_t)b]++;
        }
        if ((rc = up(&s->df_a, s->h.order_a)) || (rc = up(&s->df_b, s->h.order_b)) ||
            (rc = up(&s->df_seqa, sa)) || (rc = up(&s->df_seqb, sb))) {
            lc_schedule_free(s);
            return rc;
        }
    }
    *out = s;
    return LC_OK;
}

extern "C" int lc_make_schedule_ex(const lc_grid *g, int kind, const int8_t *offsets, int n,
                                   const int32_t *block_min, lc_schedule **out) {
    return make_schedule_impl(g, kind, offsets, n, block_min, nullptr, out);
}

extern "C" int lc_make_schedule_weighted(const lc_grid *g, int kind, const int8_t *offsets, int n,
                                         const int32_t *block_min, const int32_t *cell_counts,
                                         lc_schedule **out) {
    if (!cell_counts) return fail(LC_EINVAL, "lc_make_schedule_weighted: null cell_counts");
    return make_schedule_impl(g, kind, offsets, n, block_min, cell_counts, out);
}

extern "C" int lc_schedule_group_work(const lc_schedule *s, const int32_t *cell_counts,
                                      double *work) {
    if (!s || !cell_counts || !work) return fail(LC_EINVAL, "lc_schedule_group_work: null argument");
    const std::vector<double> w = lcs::group_work(s->h, cell_counts);
    std::copy(w.begin(), w.end(), work);
    return LC_OK;
}

extern "C" void lc_schedule_free(lc_schedule *s) {
    if (!s) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    (void)hipFree(s->grp_task);
    (void)hipFree(s->grp_foot);
    (void)hipFree(s->foot_cells);
    (void)hipFree(s->task_ab);
    (void)hipFree(s->foot_rep);
    (void)hipFree(s->fx_task);
    (void)hipFree(s->fx_foot);
    (void)hipFree(s->fx_rep);
    (void)hipFree(s->fx_cnt);
    (void)hipFree(s->df_a);
    (void)hipFree(s->df_b);
    (void)hipFree(s->df_seqa);
    (void)hipFree(s->df_seqb);
    (void)hipSetDevice(cur);
    delete s;
}

extern "C" int lc_schedule_tasks(const lc_schedule *s, int32_t *A, int32_t *B, int64_t cap,
                                 int64_t *ntask) {
    if (!s || !ntask) return fail(LC_EINVAL, "lc_schedule_tasks: null argument");
    const int64_t t = (int64_t)s->h.order_a.size();
    *ntask = t;
    if (t == 0) return fail(LC_EINVAL, "lc_schedule_tasks: not a creation-order schedule");
    if (!A || !B || cap < t) return fail(LC_ECAPACITY, "lc_schedule_tasks: need %lld entries",
                                         (long long)t);
    std::copy(s->h.order_a.begin(), s->h.order_a.end(), A);
    std::copy(s->h.order_b.begin(), s->h.order_b.end(), B);
    return LC_OK;
}

extern "C" int lc_schedule_cell_footprints(const lc_schedule *s, int32_t *count, int64_t cap) {
    if (!s || !count) return fail(LC_EINVAL, "lc_schedule_cell_footprints: null argument");
    const int64_t ncell = (int64_t)s->nc[0] * s->nc[1] * s->nc[2];
    if (cap < ncell)
        return fail(LC_ECAPACITY, "lc_schedule_cell_footprints: need %lld entries", (long long)ncell);
    std::fill(count, count + ncell, 0);
    for (int32_t c : s->h.foot_cells) count[c]++;
    return LC_OK;
}

extern "C" int lc_schedule_info_get(const lc_schedule *s, lc_schedule_info *out) {
    if (!s || !out) return fail(LC_EINVAL, "null argument");
    memset(out, 0, sizeof *out);
    out->kind = s->h.kind;
    out->nphase = (int32_t)s->h.phase_grp.size() - 1;
    out->ntask = s->h.ntask;
    out->ngroup = (int64_t)s->h.grp_task.size() - 1;
    out->max_group_tasks = s->h.max_tasks;
    out->max_group_cells = s->h.max_cells;
    out->write_mode = s->h.write_mode;
    out->max_replicas = s->h.rmax;
    return LC_OK;
}

extern "C" int lc_schedule_plan(const lc_grid *g, int kind, const int8_t *offsets, int n,
                                lc_schedule_info *out) {
    return lc_schedule_plan_ex(g, kind, offsets, n, nullptr, out);
}

extern "C" int lc_schedule_plan_tasks(const lc_grid *g, int kind, const int8_t *offsets, int n,
                                      const int32_t *block_min, int32_t *A, int32_t *B,
                                      int32_t *grp, int32_t *phase, int64_t cap,
                                      int64_t *ntask) {
    if (!g || !ntask) return fail(LC_EINVAL, "lc_schedule_plan_tasks: null argument");
    if (kind < 0 || kind >= LC_SCHED_COUNT) return fail(LC_EINVAL, "unknown schedule kind %d", kind);
    lcs::HostSchedule h;
    std::string err;
    int rc = lcs::build_schedule(g->nc, kind, offsets, n, h, err, block_min, grid_reach(g));
    if (rc) return fail(rc, "lc_schedule_plan_tasks: %s", err.c_str());
    if (!lcs::validate(h, g->ncell, err))
        return fail(LC_ESCHED, "lc_schedule_plan_tasks: %s", err.c_str());
    *ntask = (int64_t)h.task_ab.size();
    if (cap < *ntask)
        return fail(LC_ECAPACITY, "lc_schedule_plan_tasks: need %lld entries", (long long)*ntask);
    const int ngrp = (int)h.grp_task.size() - 1;
    int p = 0;
    for (int k = 0; k < ngrp; ++k) {
        while (p + 1 < (int)h.phase_grp.size() && h.phase_grp[p + 1] <= k) ++p;
        const int32_t *fc = h.foot_cells.data() + h.grp_foot[k];
        for (int t = h.grp_task[k]; t < h.grp_task[k + 1]; ++t) {
            const uint32_t ab = h.task_ab[(size_t)t];
            if (A) A[t] = fc[ab & 0xffffu];
            if (B) B[t] = fc[ab >> 16];
            if (grp) grp[t] = k;
            if (phase) phase[t] = p;
        }
    }
    return LC_OK;
}

extern "C" int lc_schedule_plan_ex(const lc_grid *g, int kind, const int8_t *offsets, int n,
                                   const int32_t *block_min, lc_schedule_info *out) {
    if (!g || !out) return fail(LC_EINVAL, "lc_schedule_plan: null argument");
    if (kind < 0 || kind >= LC_SCHED_COUNT) return fail(LC_EINVAL, "unknown schedule kind %d", kind);
    lcs::HostSchedule h;
    std::string err;
    int rc = lcs::build_schedule(g->nc, kind, offsets, n, h, err, block_min, grid_reach(g));
    if (rc) return fail(rc, "lc_schedule_plan: %s", err.c_str());
    if (!lcs::validate(h, g->ncell, err)) return fail(LC_ESCHED, "lc_schedule_plan: %s", err.c_str());
    memset(out, 0, sizeof *out);
    out->kind = h.kind;
    out->nphase = (int32_t)h.phase_grp.size() - 1;
    out->ntask = h.ntask;
    out->ngroup = (int64_t)h.grp_task.size() - 1;
    out->max_group_tasks = h.max_tasks;
    out->max_group_cells = h.max_cells;
    out->write_mode = h.write_mode;
    out->max_replicas = h.rmax;
    return LC_OK;
}

extern "C" int lc_validate_phases(int64_t ncell, int32_t nphase, const int32_t *phase_grp,
                                  const int32_t *grp_foot, const int32_t *foot_cells) {
    if (ncell < 1 || nphase < 0 || !phase_grp || !grp_foot || (nphase > 0 && !foot_cells))
        return fail(LC_EINVAL, "lc_validate_phases: bad arguments");
    lcs::HostSchedule h;
    h.write_mode = 0;
    h.phase_grp.assign(phase_grp, phase_grp + nphase + 1);
    const int32_t ng = phase_grp[nphase];
    if (phase_grp[0] != 0 || ng < 0) return fail(LC_EINVAL, "lc_validate_phases: phase_grp");
    for (int p = 0; p < nphase; ++p)
        if (phase_grp[p + 1] < phase_grp[p]) return fail(LC_EINVAL, "lc_validate_phases: order");
    h.grp_foot.assign(grp_foot, grp_foot + ng + 1);
    for (int k = 0; k < ng; ++k)
        if (grp_foot[k + 1] < grp_foot[k]) return fail(LC_EINVAL, "lc_validate_phases: grp_foot");
    h.foot_cells.assign(foot_cells, foot_cells + grp_foot[ng]);
    std::string err;
    if (!lcs::validate(h, ncell, err)) return fail(LC_ESCHED, "%s", err.c_str());
    return LC_OK;
}

extern "C" int lc_serialization_degree(const int32_t dims[3], int kind, const int8_t *offsets,
                                       int n, int64_t *level_hist, int64_t hist_len,
                                       lc_sd_result *out) {
    if (!dims || !out) return fail(LC_EINVAL, "null argument");
    for (int d = 0; d < 3; ++d)
        if (dims[d] < 1) return fail(LC_EINVAL, "dims must be >= 1");
    const bool two_d = dims[2] == 1;
    std::vector<lcs::Offset> order;
    std::string err;
    if (kind != LC_SCHED_LEX && kind != LC_SCHED_OPT && kind != LC_SCHED_BEST &&
        kind != LC_SCHED_BAD && kind != LC_SCHED_LOOPEX && kind != LC_SCHED_CUSTOM)
        return fail(LC_EINVAL, "kind %d has no creation order", kind);
    if (!lcs::stencil_order(kind, two_d, offsets, n, order, err,
                            kind == LC_SCHED_CUSTOM ? lcs::order_reach(offsets, n) : 1))
        return fail(LC_EINVAL, "serialization_degree: %s", err.c_str());
    std::vector<int32_t> A, B, level;
    if (kind == LC_SCHED_LOOPEX) {
        if (!lcs::loopex_tasks(dims, order, A, B))
            return fail(LC_EINVAL, "loop exchange needs even dims");
    } else {
        lcs::basic_tasks(dims, order, A, B);
    }
    const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
    const int64_t cp = lcs::task_levels(ncell, A, B, level);
    memset(out, 0, sizeof *out);
    out->tasks = (int64_t)A.size();
    out->cp = cp;
    out->speedup = cp ? (double)out->tasks / (double)cp : 0.0;
    out->degree = out->tasks ? (double)cp / (double)out->tasks : 0.0;
    out->n = (int32_t)order.size();
    // loop exchange has no stencil displacement (Delta = 0): Eq. 2 then
    // gives k (every cell at once) and Eq. 3 diverges
    const int delta = kind == LC_SCHED_LOOPEX ? 0 : lcs::delta_rule(order);
    out->delta = delta;
    const double k = (double)ncell, nn = (double)order.size();
    out->s_eq2 = nn * k / (nn + delta * (k - 1.0));
    out->s_max = delta > 0 ? nn / delta : HUGE_VAL;
    if (level_hist) {
        for (int64_t l = 0; l < hist_len; ++l) level_hist[l] = 0;
        for (int32_t l : level)
            if (l - 1 < hist_len) level_hist[l - 1]++;
    }
    return LC_OK;
}

extern "C" int lc_serialization_degree_weighted(const int32_t dims[3], int kind,
                                                const int8_t *offsets, int n,
                                                const int32_t *cell_counts, lc_wsd_result *out) {
    if (!dims || !out || !cell_counts) return fail(LC_EINVAL, "null argument");
    for (int d = 0; d < 3; ++d)
        if (dims[d] < 1) return fail(LC_EINVAL, "dims must be >= 1");
    if (kind != LC_SCHED_LEX && kind != LC_SCHED_OPT && kind != LC_SCHED_BEST &&
        kind != LC_SCHED_BAD && kind != LC_SCHED_LOOPEX && kind != LC_SCHED_CUSTOM)
        return fail(LC_EINVAL, "kind %d has no creation order", kind);
    const bool two_d = dims[2] == 1;
    std::vector<lcs::Offset> order;
    std::string err;
    if (!lcs::stencil_order(kind, two_d, offsets, n, order, err,
                            kind == LC_SCHED_CUSTOM ? lcs::order_reach(offsets, n) : 1))
        return fail(LC_EINVAL, "serialization_degree_weighted: %s", err.c_str());
    std::vector<int32_t> A, B;
    if (kind == LC_SCHED_LOOPEX) {
        if (!lcs::loopex_tasks(dims, order, A, B))
            return fail(LC_EINVAL, "loop exchange needs even dims");
    } else {
        lcs::basic_tasks(dims, order, A, B);
    }
    std::vector<double> w(A.size());
    double work = 0.0;
    for (size_t t = 0; t < A.size(); ++t) {
        const double na = cell_counts[A[t]], nb = cell_counts[B[t]];
        w[t] = A[t] == B[t] ? 0.5 * na * (na - 1.0) : na * nb;
        work += w[t];
    }
    const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
    const double cp = lcs::task_levels_weighted(ncell, A, B, w);
    out->tasks = (int64_t)A.size();
    out->work = work;
    out->cp = cp;
    out->speedup = cp > 0.0 ? work / cp : 0.0;
    return LC_OK;
}

extern "C" int lc_compute_forces(const lc_grid *g, const lc_schedule *s, const int32_t *cell_start,
                                 const uint32_t *coord, int64_t n, int64_t *F, int64_t *ew,
                                 int precision, lc_workspace *ws, void *stream) {
    if (!g || !s || !cell_start || !F || !ew || (n > 0 && !coord))
        return fail(LC_EINVAL, "lc_compute_forces: null argument");
    if (precision != LC_PREC_FP32 && precision != LC_PREC_FP64)
        return fail(LC_EINVAL, "lc_compute_forces: precision");
    if (s->nc[0] != g->nc[0] || s->nc[1] != g->nc[1] || s->nc[2] != g->nc[2])
        return fail(LC_EINVAL, "lc_compute_forces: schedule built for another grid");
    if (n < 0 || n >= 2147483647LL) return fail(LC_EINVAL, "lc_compute_forces: bad n");
    int rc = check_ws(ws, 0, 0);
    if (rc) return rc;
    return forces_impl(g, s, cell_start, coord, n, F, ew, precision, ws, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Force evaluation without allocation: the scratch lives in a file-scope
// device array, one copy per device, held until the process ends.
// ---------------------------------------------------------------------------

// Layout: the spread energy slots (kPartSlots x 3 int64), the status word
// (one int64 slot), then the replica buffer of buffer + reduce.
constexpr int64_t kScratchPartElems = 3 * kPartSlots + 1;
constexpr int64_t kScratchPbufOff = 24832;  // bytes, 256-aligned, past the slots
static_assert(kScratchPartElems * 8 <= kScratchPbufOff && kScratchPbufOff % 256 == 0,
              "scratch layout");
static __device__ __align__(256) unsigned char scratch[LC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device

// The device address of the current device's `scratch` (looked up once per
// device, with that device current).
static int scratch_address(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LC_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LC_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LC_OK;
}

extern "C" int lc_compute_forces_noalloc(const lc_grid *g, const lc_schedule *s,
                                         const int32_t *cell_start, const uint32_t *coord,
                                         int64_t n, int64_t *F, int64_t *ew, int precision,
                                         uint32_t *flags, void *stream) {
    if (!g || !s || !cell_start || !F || !ew || (n > 0 && !coord))
        return fail(LC_EINVAL, "lc_compute_forces_noalloc: null argument");
    if (precision != LC_PREC_FP32 && precision != LC_PREC_FP64)
        return fail(LC_EINVAL, "lc_compute_forces_noalloc: precision");
    if (s->nc[0] != g->nc[0] || s->nc[1] != g->nc[1] || s->nc[2] != g->nc[2])
        return fail(LC_EINVAL, "lc_compute_forces_noalloc: schedule built for another grid");
    if (n < 0 || n >= 2147483647LL) return fail(LC_EINVAL, "lc_compute_forces_noalloc: bad n");
    const int64_t pbuf_bytes = s->h.write_mode == 3 ? 8 * pbuf_elems(s->h.rmax, n) : 0;
    if (pbuf_bytes > (int64_t)LC_NOALLOC_SCRATCH_BYTES - kScratchPbufOff)
        return fail(LC_ECAPACITY,
                    "lc_compute_forces_noalloc: the replica buffer needs %lld bytes, the static "
                    "scratch holds %lld",
                    (long long)pbuf_bytes, (long long)(LC_NOALLOC_SCRATCH_BYTES - kScratchPbufOff));
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    SweepScratch sc;
    sc.part = (long long *)base;
    sc.flags = flags ? flags : (uint32_t *)(sc.part + 3 * kPartSlots);
    sc.pbuf = (long long *)((unsigned char *)base + kScratchPbufOff);
    sc.max_per_cell = 0;
    // the slots and the status word keep what the last call left: clear them
    if ((rc = fill64(sc.part, kScratchPartElems, st))) return rc;
    return forces_run(g, s, cell_start, coord, n, F, ew, precision, sc, st, nullptr);
}

__global__ __launch_bounds__(256) void k_selftest_recip(uint32_t lo, uint32_t n,
                                                        unsigned long long *bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long cnt = 0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const float x = __uint_as_float(lo + (uint32_t)k);
        cnt += __float_as_uint(rcp_nr(x)) != __float_as_uint(1.0f / x) ? 1u : 0u;
    }
    if (cnt) atomicAdd(bad, cnt);
}

extern "C" int lc_selftest_recip(uint32_t lo_bits, uint32_t hi_bits, uint64_t *mismatches) {
    if (!mismatches || hi_bits <= lo_bits) return fail(LC_EINVAL, "lc_selftest_recip: range");
    unsigned long long *d = nullptr;
    int rc = dalloc(&d, 1);
    if (rc) return rc;
    unsigned long long h = 0;
    hipError_t e = hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const uint32_t n = hi_bits - lo_bits;
        hipLaunchKernelGGL(k_selftest_recip, dim3(4096), dim3(256), 0, 0, lo_bits, n, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(&h, d, sizeof(h), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(LC_EHIP, "lc_selftest_recip: %s", hipGetErrorString(e));
    *mismatches = (uint64_t)h;
    return LC_OK;
}

template <int MODE, int CELL>
static int launch_dataflow(const DfArgs &a, int ncu, hipStream_t st) {
    static int per_cu = 0;
    int res = per_cu;
    if (res == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(&k_dataflow<MODE, CELL>), 64, 0) ==
                hipSuccess &&
            nb >= 1)
            per_cu = res = nb;
        else
            res = 1;
    }
    // at most 10 runners per compute unit (what the 256-particle tiles allow):
    // more only add contention on the unit counter and the cell locks
    const int64_t grid = std::min<int64_t>(a.nunit, (int64_t)std::min(res, 10) * ncu);
    if (grid > 0) {
        hipLaunchKernelGGL((k_dataflow<MODE, CELL>), dim3((unsigned)grid), dim3(64), 0, st, a);
        LAUNCHCHK("k_dataflow");
    }
    return LC_OK;
}

extern "C" int lc_compute_forces_dataflow(const lc_grid *g, const lc_schedule *s, int mode,
                                          const int32_t *cell_start, const uint32_t *coord,
                                          int64_t n, int64_t *F, int64_t *ew, double limit_ms,
                                          lc_workspace *ws, void *stream) {
    return lc_compute_forces_dataflow_log(g, s, mode, cell_start, coord, n, F, ew, limit_ms,
                                          nullptr, ws, stream);
}

extern "C" int lc_compute_forces_dataflow_log(const lc_grid *g, const lc_schedule *s, int mode,
                                              const int32_t *cell_start, const uint32_t *coord,
                                              int64_t n, int64_t *F, int64_t *ew,
                                              double limit_ms, int32_t *log, lc_workspace *ws,
                                              void *stream) {
    if (!g || !s || !cell_start || !F || !ew || (n > 0 && !coord))
        return fail(LC_EINVAL, "lc_compute_forces_dataflow: null argument");
    if (mode < LC_DF_ORDERED || mode > LC_DF_NESTED)
        return fail(LC_EINVAL, "lc_compute_forces_dataflow: unknown mode %d", mode);
    if (s->nc[0] != g->nc[0] || s->nc[1] != g->nc[1] || s->nc[2] != g->nc[2])
        return fail(LC_EINVAL, "lc_compute_forces_dataflow: schedule built for another grid");
    if (!s->df_a)
        return fail(LC_EINVAL, "lc_compute_forces_dataflow: needs a creation-order schedule "
                               "(LEX, OPT, BEST, BAD, CUSTOM or LOOPEX)");
    if (mode == LC_DF_NESTED && s->h.chain <= 0)
        return fail(LC_EINVAL, "lc_compute_forces_dataflow: loop exchange has no per-cell chains");
    if (!(limit_ms >= 0.0) || limit_ms > 6.0e4)
        return fail(LC_EINVAL, "lc_compute_forces_dataflow: limit_ms must be in [0, 60000]");
    int rc = check_ws(ws, n, g->ncell);
    if (rc) return rc;
    if (ws->max_per_cell > kDfCell)
        return fail(LC_ECAPACITY, "lc_compute_forces_dataflow: cells of up to %d particles "
                                  "(tile hint %d)", kDfCell, ws->max_per_cell);
    hipStream_t st = (hipStream_t)stream;
    if (!ws->df_sync) {
        if ((rc = dalloc(&ws->df_sync, ws->max_cells)) || (rc = dalloc(&ws->df_ctl, 4))) return rc;
    }
    if ((rc = fill32(ws->df_sync, g->ncell, st)) || (rc = fill32(ws->df_ctl, 4, st)) ||
        (rc = fill64((long long *)F, 3 * n, st)))
        return rc;
    DfArgs a;
    a.ta = s->df_a;
    a.tb = s->df_b;
    a.seqa = s->df_seqa;
    a.seqb = s->df_seqb;
    const int64_t ntask = (int64_t)s->h.order_a.size();
    a.ntask = ntask;
    a.log = log;
    a.chain = mode == LC_DF_NESTED ? s->h.chain : 1;
    a.nunit = mode == LC_DF_NESTED ? ntask / s->h.chain : ntask;
    a.cell_start = cell_start;
    a.coord = coord;
    a.n = n;
    a.F = (long long *)F;
    a.part = (long long *)ws->part;
    a.sync = ws->df_sync;
    a.ctl = ws->df_ctl;
    a.flags = ws->flags;
    a.pp = pair_params(g);
    a.limit = (unsigned long long)(limit_ms * 1.0e5);  // s_memrealtime: 100 MHz
    // small cells (the tile hint, set by the cell build) take the runner
    // with 64-particle tiles: more runners per compute unit
    const bool small = ws->max_per_cell > 0 && ws->max_per_cell <= 64;
    if (mode == LC_DF_ORDERED)
        rc = small ? launch_dataflow<0, 64>(a, s->ncu, st) : launch_dataflow<0, 256>(a, s->ncu, st);
    else if (mode == LC_DF_MUTEX)
        rc = small ? launch_dataflow<1, 64>(a, s->ncu, st) : launch_dataflow<1, 256>(a, s->ncu, st);
    else
        rc = small ? launch_dataflow<2, 64>(a, s->ncu, st) : launch_dataflow<2, 256>(a, s->ncu, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_reduce_parts<3>, dim3(1), dim3(256), 0, st, (long long *)ws->part,
                       (long long *)ew, 0);
    LAUNCHCHK("k_reduce_parts");
    return LC_OK;
}

extern "C" int lc_compute_forces_profiled(const lc_grid *g, const lc_schedule *s,
                                          const int32_t *cell_start, const uint32_t *coord,
                                          int64_t n, int64_t *F, int64_t *ew, int precision,
                                          lc_workspace *ws, void *stream, double *sweep_ms,
                                          double *phase_ms) {
    if (!sweep_ms) return fail(LC_EINVAL, "lc_compute_forces_profiled: sweep_ms");
    if (!g || !s || !cell_start || !F || !ew || (n > 0 && !coord))
        return fail(LC_EINVAL, "lc_compute_forces_profiled: null argument");
    if (precision != LC_PREC_FP32 && precision != LC_PREC_FP64)
        return fail(LC_EINVAL, "lc_compute_forces_profiled: precision");
    if (s->nc[0] != g->nc[0] || s->nc[1] != g->nc[1] || s->nc[2] != g->nc[2])
        return fail(LC_EINVAL, "lc_compute_forces_profiled: schedule built for another grid");
    int rc = check_ws(ws, 0, 0);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int nphase = (int)s->h.phase_grp.size() - 1;
    std::vector<hipEvent_t> ev((size_t)2 * nphase + 2, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(LC_EHIP, "hipEventCreate");
        }
    rc = forces_impl(g, s, cell_start, coord, n, F, ew, precision, ws, st, ev.data());
    double total = 0.0;
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(LC_EHIP, "hipStreamSynchronize");
    for (int p = 0; p < nphase && !rc; ++p) {
        float ms = 0.0f;
        if (s->h.phase_grp[p + 1] > s->h.phase_grp[p]) {
            if (hipEventElapsedTime(&ms, ev[2 * p], ev[2 * p + 1]) != hipSuccess) {
                rc = fail(LC_EHIP, "hipEventElapsedTime");
                break;
            }
        }
        total += ms;
        if (phase_ms) phase_ms[p] = ms;
    }
    if (!rc && phase_ms) {  // the closing launch: gather (buffer + reduce) or the energy sums
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[2 * nphase], ev[2 * nphase + 1]) != hipSuccess)
            rc = fail(LC_EHIP, "hipEventElapsedTime");
        phase_ms[nphase] = ms;
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (!rc) *sweep_ms = total;
    return rc;
}

extern "C" int lc_kinetic_energy(const double *vel, int64_t n, int64_t *ke, lc_workspace *ws,
                                 void *stream) {
    if (!ke || (n > 0 && !vel)) return fail(LC_EINVAL, "lc_kinetic_energy: null argument");
    hipStream_t st = (hipStream_t)stream;
    if (!ws) return fail(LC_EINVAL, "lc_kinetic_energy: null workspace");
    if (n > 0) {
        hipLaunchKernelGGL(k_kick_ke, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           (double *)vel, (const long long *)nullptr, n, 0.0, 0,
                           (unsigned long long *)ws->kpart);
        LAUNCHCHK("k_kick_ke");
    }
    hipLaunchKernelGGL(k_reduce_parts<1>, dim3(1), dim3(256), 0, st, (long long *)ws->kpart,
                       (long long *)ke, 0);
    LAUNCHCHK("k_reduce_parts");
    return LC_OK;
}

static int rebuild(const lc_grid *g, double *pos, double *vel, int32_t *ids, int64_t n,
                   int32_t *cell_start, int32_t *perm, uint32_t *coord, lc_workspace *ws,
                   hipStream_t st) {
    int rc = build_cells_impl(g, pos, n, cell_start, perm, coord, ws, st);
    if (rc) return rc;
    const size_t b3 = sizeof(double) * 3 * (size_t)n;
    if ((rc = gather_impl(perm, n, pos, ws->tmp3, ids, ws->tmpi, st))) return rc;
    HIPCHK(hipMemcpyAsync(pos, ws->tmp3, b3, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(ws->xref, ws->tmp3, b3, hipMemcpyDeviceToDevice, st));
    if (ids) HIPCHK(hipMemcpyAsync(ids, ws->tmpi, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    if ((rc = gather_impl(perm, n, vel, ws->tmp3, nullptr, nullptr, st))) return rc;
    HIPCHK(hipMemcpyAsync(vel, ws->tmp3, b3, hipMemcpyDeviceToDevice, st));
    return LC_OK;
}

extern "C" int lc_verlet_step(const lc_grid *g, const lc_schedule *s, double *pos, double *vel,
                              int32_t *ids, int64_t n, int64_t *F, int32_t *cell_start,
                              int32_t *perm, uint32_t *coord, double dt, int nsteps,
                              int rebuild_every, int64_t *trace, lc_workspace *ws, void *stream) {
    if (!g || !s || !trace || !F || !cell_start || (n > 0 && (!pos || !vel || !perm || !coord)))
        return fail(LC_EINVAL, "lc_verlet_step: null argument");
    if (nsteps < 0 || rebuild_every < 1) return fail(LC_EINVAL, "lc_verlet_step: steps");
    int rc = check_ws(ws, n, g->ncell);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    GridArgs ga;
    for (int d = 0; d < 3; ++d) {
        ga.inv[d] = g->inv_box[d];
        ga.nc[d] = g->nc[d];
    }
    const double hdt = 0.5 * dt;
    const double lim = 0.5 * g->skin;
    const double lim2 = lim * lim;
    const unsigned nbk = (unsigned)((n + 255) / 256);
    // Step k: (rebuild), forces at x_k, the closing half kick to v_k with
    // its kinetic energy, and -- fused into the same pass while another
    // step follows -- the next step's opening half kick and drift to
    // x_{k+1}.  Buffer + reduce schedules sum their replica slots inside
    // that pass (no gather launch, no F round trip) except at the last step,
    // whose forces are returned in F.
    const bool fold = s->h.write_mode == 3 && n > 0;
    // step 0: sort into cells at the current positions, forces, energies
    if ((rc = rebuild(g, pos, vel, ids, n, cell_start, perm, coord, ws, st))) return rc;
    if ((rc = forces_impl(g, s, cell_start, coord, n, F, ws->ew, LC_PREC_FP32, ws, st, nullptr,
                          !(fold && nsteps > 0))))
        return rc;
    for (int step = 0; step <= nsteps; ++step) {
        if (step > 0) {
            if (step % rebuild_every == 0)
                if ((rc = rebuild(g, pos, vel, ids, n, cell_start, perm, coord, ws, st))) return rc;
            if ((rc = forces_impl(g, s, cell_start, coord, n, F, ws->ew, LC_PREC_FP32, ws, st,
                                  nullptr, !(fold && step < nsteps))))
                return rc;
        }
        long long *row = (long long *)trace + 2 * step;
        if (n > 0 && step < nsteps && fold) {
            hipLaunchKernelGGL(k_gather_kick_ke_drift, dim3(nbk + 1), dim3(256), 0, st,
                               (const long long *)ws->pbuf,
                               (const int *)rcnt_of(ws, s->h.rmax, n), s->h.rmax, n, pos,
                               vel, hdt, dt,
                               step > 0 ? 1 : 0, ws->xref, lim2, ga, coord, ws->flags,
                               (unsigned long long *)ws->kpart, (long long *)ws->part,
                               (long long *)ws->ew);
            LAUNCHCHK("k_gather_kick_ke_drift");
        } else if (n > 0 && step < nsteps) {
            hipLaunchKernelGGL(k_kick_ke_drift, dim3(nbk), dim3(256), 0, st, pos, vel,
                               (const long long *)F, n, hdt, dt, step > 0 ? 1 : 0, ws->xref,
                               lim2, ga, coord, ws->flags, (unsigned long long *)ws->kpart);
            LAUNCHCHK("k_kick_ke_drift");
        } else if (n > 0) {
            hipLaunchKernelGGL(k_kick_ke, dim3(nbk), dim3(256), 0, st, vel, (const long long *)F, n,
                               hdt, step > 0 ? 1 : 0, (unsigned long long *)ws->kpart);
            LAUNCHCHK("k_kick_ke");
        }
        hipLaunchKernelGGL(k_reduce_parts<1>, dim3(1), dim3(256), 0, st, (long long *)ws->kpart,
                           row, 0);
        LAUNCHCHK("k_reduce_parts");
        hipLaunchKernelGGL(k_copy64, dim3(1), dim3(64), 0, st, (const long long *)ws->ew, row + 1, 1);
        LAUNCHCHK("k_copy64");
    }
    return LC_OK;
}

// ---------------------------------------------------------------------------
// a8: batched boxes
// ---------------------------------------------------------------------------

struct BoxGeo {
    double inv[3];
    int nc[3];
    int cstart;
};

__device__ __forceinline__ int box_of(const int64_t *__restrict__ pstart, int nbox, int64_t i) {
    int lo = 0, hi = nbox;  // pstart[lo] <= i < pstart[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pstart[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_bin_batch(const double *__restrict__ pos, int64_t ntot,
                                                   const int64_t *__restrict__ pstart, int nbox,
                                                   const BoxGeo *__restrict__ geo,
                                                   int *__restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < ntot;
    int cc = 0;
    uint32_t u[3];
    if (act) {
        const BoxGeo gb = geo[box_of(pstart, nbox, i)];
        cc = gb.cstart + cell_and_fractions(pos, ntot, i, gb.inv, gb.nc, u);
    }
    const unsigned long long mine = wave_cell_group(act, cc);
    const int lane = threadIdx.x & 63;
    if (mine && !(mine & ((1ull << lane) - 1ull))) atomicAdd(&counts[cc], __popcll(mine));
}

__global__ __launch_bounds__(256) void k_scatter_batch(
    const double *__restrict__ pos, int64_t ntot, const int64_t *__restrict__ pstart, int nbox,
    const BoxGeo *__restrict__ geo, const int *__restrict__ cell_start, int *__restrict__ counts,
    int *__restrict__ perm, uint32_t *__restrict__ coord) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < ntot;
    int cc = 0;
    uint32_t u[3] = {0u, 0u, 0u};
    if (act) {
        const BoxGeo gb = geo[box_of(pstart, nbox, i)];
        cc = gb.cstart + cell_and_fractions(pos, ntot, i, gb.inv, gb.nc, u);
    }
    const int r = wave_cell_claim(act, cc, counts);
    if (!act) return;
    const int64_t dst = (int64_t)cell_start[cc] + r;
    perm[dst] = (int)i;
    for (int d = 0; d < 3; ++d) coord[d * ntot + dst] = u[d];
}

struct lc_batch {
    int device = 0;
    int ncu = 256;
    int nbox = 0;
    int nwhole = 0;
    int cap = 1024;
    bool ff = true;  // every box admits the integer candidate filter
    int wmode = 3;   // sweep write mode: 3 replica buffer + gather, 1 atomic write-back
    int64_t ntot = 0, ncell = 0;
    std::vector<int64_t> pstart, cstart;
    lcs::HostSchedule h;  // combined groups, global cell ids
    std::vector<int32_t> grp_box;
    std::vector<PairParams> ppar;
    std::vector<BoxGeo> geo;
    int32_t *d_grp_task = nullptr, *d_grp_foot = nullptr, *d_foot_cells = nullptr;
    int32_t *d_foot_rep = nullptr, *d_grp_box = nullptr;
    uint32_t *d_task_ab = nullptr;
    PairParams *d_ppar = nullptr;
    BoxGeo *d_geo = nullptr;
    int64_t *d_pstart = nullptr;
    int *d_ticket = nullptr;
};

struct lc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    lc_workspace *ws = nullptr;  // its replica buffer must not move while the graph lives
};

extern "C" void lc_batch_free(lc_batch *b) {
    if (!b) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(b->device);
    (void)hipFree(b->d_grp_task);
    (void)hipFree(b->d_grp_foot);
    (void)hipFree(b->d_foot_cells);
    (void)hipFree(b->d_foot_rep);
    (void)hipFree(b->d_grp_box);
    (void)hipFree(b->d_task_ab);
    (void)hipFree(b->d_ppar);
    (void)hipFree(b->d_geo);
    (void)hipFree(b->d_pstart);
    (void)hipFree(b->d_ticket);
    (void)hipSetDevice(cur);
    delete b;
}

template <typename T>
static int upload(T **dst, const std::vector<T> &v) {
    int rc = dalloc(dst, (int64_t)v.size());
    if (rc) return rc;
    if (!v.empty() &&
        hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(LC_EHIP, "batch upload");
    return LC_OK;
}

extern "C" int lc_batch_create(const lc_box_desc *boxes, int nbox, const int32_t *modes,
                               lc_batch **out) {
    return lc_batch_create_ex(boxes, nbox, modes, nullptr, out);
}

extern "C" int lc_batch_create_ex(const lc_box_desc *boxes, int nbox, const int32_t *modes,
                                  const lc_batch_opts *opts, lc_batch **out) {
    if (!boxes || nbox < 1 || !out) return fail(LC_EINVAL, "lc_batch_create: bad arguments");
    const int tile = opts && opts->tile ? opts->tile : 768;
    const int wm = opts ? opts->write_mode : LC_BATCH_WRITE_BUFFER;
    if (tile != 512 && tile != 768 && tile != 1024 && tile != 2048)
        return fail(LC_EINVAL, "lc_batch_create_ex: tile %d (512, 768, 1024 or 2048)", tile);
    if (wm != LC_BATCH_WRITE_BUFFER && wm != LC_BATCH_WRITE_ATOMIC)
        return fail(LC_EINVAL, "lc_batch_create_ex: write mode %d", wm);
    lc_batch *b = new lc_batch();
    b->wmode = wm == LC_BATCH_WRITE_ATOMIC ? 1 : 3;
    b->nbox = nbox;
    b->pstart.assign(1, 0);
    b->cstart.assign(1, 0);
    for (int k = 0; k < nbox; ++k) {
        if (boxes[k].n < 0 || boxes[k].grid.ncell < 27) {
            delete b;
            return fail(LC_EINVAL, "lc_batch_create: box %d", k);
        }
        if (grid_reach(&boxes[k].grid) != 1 || boxes[k].grid.nc[2] < 3) {
            delete b;
            return fail(LC_EINVAL, "lc_batch_create: box %d: batches take 3D grids of cells of "
                                   "side >= rc", k);
        }
        b->pstart.push_back(b->pstart.back() + boxes[k].n);
        b->cstart.push_back(b->cstart.back() + boxes[k].grid.ncell);
    }
    b->ntot = b->pstart.back();
    b->ncell = b->cstart.back();
    if (b->ntot >= 2147483647LL || b->ncell >= 2147483647LL) {
        delete b;
        return fail(LC_ECAPACITY, "lc_batch_create: more than 2^31 particles or cells");
    }
    // per-box group lists in global cell ids
    struct Grp {
        std::vector<int32_t> cells;  // footprint (global)
        std::vector<int32_t> rep;    // replica slot per footprint cell
        std::vector<uint32_t> ab;    // tasks (local footprint indices)
        int box;
        double est;                  // expected particles in the footprint
    };
    std::vector<Grp> groups;
    std::vector<int32_t> cell_rep((size_t)b->ncell, 0);
    double est_max = 0.0;
    bool filt = true;
    for (int k = 0; k < nbox; ++k) {
        const lc_grid &g = boxes[k].grid;
        const double dens = (double)boxes[k].n / (double)g.ncell;
        const int mode = modes ? modes[k] : LC_BATCH_AUTO;
        const bool whole = mode == LC_BATCH_WHOLE ||
                           (mode == LC_BATCH_AUTO && g.ncell <= 36 && boxes[k].n <= 768);
        const int32_t c0 = (int32_t)b->cstart[k];
        if (whole) {
            if (14 * (int64_t)g.ncell > lcs::kMaxGroupTasks || g.ncell > lcs::kMaxGroupCells) {
                lc_batch_free(b);
                return fail(LC_ECAPACITY, "box %d too large for one work-group", k);
            }
            std::vector<lcs::Offset> order;
            std::string err;
            lcs::stencil_order(LC_SCHED_LEX, false, nullptr, 0, order, err);
            std::vector<int32_t> A, B;
            lcs::basic_tasks(g.nc, order, A, B);
            Grp gr;
            gr.box = k;
            for (int32_t c = 0; c < g.ncell; ++c) {
                gr.cells.push_back(c0 + c);
                gr.rep.push_back(cell_rep[(size_t)(c0 + c)]++);
            }
            for (size_t t = 0; t < A.size(); ++t)
                gr.ab.push_back((uint32_t)A[t] | ((uint32_t)B[t] << 16));
            gr.est = (double)boxes[k].n;  // the footprint is the box: exact
            est_max = std::max(est_max, gr.est);
            groups.push_back(std::move(gr));
            b->nwhole++;
        } else {
            // the largest blocks whose footprint is expected (box density,
            // 35% headroom) to fit the tile (768 particles by default, which
            // runs three work-groups per CU); dense boxes take smaller blocks
            // (more replicas).  Footprints (corner grouping): 64, 48, 36, 32,
            // 18, 12 and 8 cells.
            static const int32_t kShapes[][3] = {{3, 3, 3}, {2, 3, 3}, {2, 2, 3}, {1, 3, 3},
                                                 {1, 2, 2}, {1, 1, 2}, {1, 1, 1}};
            lcs::HostSchedule hb;
            std::string err;
            int rc = 0;
            for (const auto &shape : kShapes) {
                rc = lcs::build_schedule(g.nc, LC_SCHED_BUFFER, nullptr, 0, hb, err, shape);
                if (rc || dens * hb.max_cells * 1.35 <= (double)tile) break;
            }
            if (rc) {
                lc_batch_free(b);
                return fail(rc, "box %d: %s", k, err.c_str());
            }
            const int ng = (int)hb.grp_task.size() - 1;
            for (int q = 0; q < ng; ++q) {
                Grp gr;
                gr.box = k;
                for (int f = hb.grp_foot[q]; f < hb.grp_foot[q + 1]; ++f) {
                    gr.cells.push_back(c0 + hb.foot_cells[f]);
                    gr.rep.push_back(hb.foot_rep[f]);
                }
                for (int t = hb.grp_task[q]; t < hb.grp_task[q + 1]; ++t) gr.ab.push_back(hb.task_ab[t]);
                gr.est = dens * (double)gr.cells.size() * 1.35;
                est_max = std::max(est_max, gr.est);
                groups.push_back(std::move(gr));
            }
            for (int32_t c = 0; c < g.ncell; ++c) cell_rep[(size_t)(c0 + c)] = hb.cell_rep[(size_t)c];
        }
        PairParams pp;
        for (int d = 0; d < 3; ++d) {
            pp.s[d] = g.scale[d];
            pp.sd[d] = g.box[d] / 4294967296.0;
        }
        pp.rc2 = g.rc2;
        pp.thr16 = filter16_bound(g.box, g.rc2);
        if (pp.thr16 == 0 || dens > 0.5 * kFFCell) filt = false;
        pp.ecut = g.ecut;
        pp.rc2d = g.rc * g.rc;
        const double ic = 1.0 / pp.rc2d, s6 = ic * ic * ic;
        pp.ecutd = 4.0 * s6 * (s6 - 1.0);
        b->ppar.push_back(pp);
        BoxGeo gg;
        for (int d = 0; d < 3; ++d) {
            gg.inv[d] = g.inv_box[d];
            gg.nc[d] = g.nc[d];
        }
        gg.cstart = c0;
        b->geo.push_back(gg);
    }
    // one launch, heaviest groups first: a group's pair work grows with its
    // task count times the square of its box's particles per cell
    std::stable_sort(groups.begin(), groups.end(), [&](const Grp &x, const Grp &y) {
        const double dx = (double)boxes[x.box].n / (double)boxes[x.box].grid.ncell;
        const double dy = (double)boxes[y.box].n / (double)boxes[y.box].grid.ncell;
        return (double)x.ab.size() * dx * dx > (double)y.ab.size() * dy * dy;
    });
    lcs::HostSchedule &h = b->h;
    h.write_mode = b->wmode;
    h.grp_task.assign(1, 0);
    h.grp_foot.assign(1, 0);
    h.phase_grp = {0};
    for (auto &gr : groups) {
        h.foot_cells.insert(h.foot_cells.end(), gr.cells.begin(), gr.cells.end());
        h.foot_rep.insert(h.foot_rep.end(), gr.rep.begin(), gr.rep.end());
        h.task_ab.insert(h.task_ab.end(), gr.ab.begin(), gr.ab.end());
        h.grp_task.push_back((int32_t)h.task_ab.size());
        h.grp_foot.push_back((int32_t)h.foot_cells.size());
        h.max_tasks = std::max(h.max_tasks, (int)gr.ab.size());
        h.max_cells = std::max(h.max_cells, (int)gr.cells.size());
        h.ntask += (int64_t)gr.ab.size();
        b->grp_box.push_back(gr.box);
    }
    h.phase_grp.push_back((int32_t)groups.size());
    h.cell_rep = cell_rep;
    for (int32_t r : cell_rep) h.rmax = std::max(h.rmax, r);
    const double need = est_max;
    b->cap = need <= 768 ? 768 : need <= 1024 ? 1024 : (need <= 2048 ? 2048 : 3072);
    if (filt && need <= 512) b->cap = 512;  // the filtered kernel has a 512 tile
    b->ff = filt && b->cap <= 2048;

    int rc = 0;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return fail(LC_EHIP, "hipGetDevice");
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess &&
        ncu > 0)
        b->ncu = ncu;
    std::vector<int64_t> ps(b->pstart);
    if ((rc = upload(&b->d_grp_task, h.grp_task)) || (rc = upload(&b->d_grp_foot, h.grp_foot)) ||
        (rc = upload(&b->d_foot_cells, h.foot_cells)) ||
        (rc = upload(&b->d_foot_rep, device_foot_rep(h))) ||
        (rc = upload(&b->d_grp_box, b->grp_box)) ||
        (rc = upload(&b->d_task_ab, h.task_ab)) || (rc = upload(&b->d_ppar, b->ppar)) ||
        (rc = upload(&b->d_geo, b->geo)) || (rc = upload(&b->d_pstart, ps)) ||
        (rc = dalloc(&b->d_ticket, 1))) {
        lc_batch_free(b);
        return rc;
    }
    *out = b;
    return LC_OK;
}

extern "C" int lc_batch_info_get(const lc_batch *b, lc_batch_info *out) {
    if (!b || !out) return fail(LC_EINVAL, "null argument");
    memset(out, 0, sizeof *out);
    out->nbox = b->nbox;
    out->nwhole = b->nwhole;
    out->ntot = b->ntot;
    out->ncell = b->ncell;
    out->ngroup = (int64_t)b->grp_box.size();
    out->ntask = b->h.ntask;
    out->max_replicas = b->h.rmax;
    out->lds_tile = b->cap;
    return LC_OK;
}

extern "C" int lc_batch_offsets(const lc_batch *b, int64_t *pstart, int64_t *cstart) {
    if (!b || !pstart || !cstart) return fail(LC_EINVAL, "null argument");
    for (int k = 0; k <= b->nbox; ++k) {
        pstart[k] = b->pstart[k];
        cstart[k] = b->cstart[k];
    }
    return LC_OK;
}

extern "C" int lc_batch_build_cells(const lc_batch *b, const double *pos, int32_t *cell_start,
                                    int32_t *perm, uint32_t *coord, lc_workspace *ws,
                                    void *stream) {
    if (!b || !cell_start || (b->ntot > 0 && (!pos || !perm || !coord)))
        return fail(LC_EINVAL, "lc_batch_build_cells: null argument");
    int rc = check_ws(ws, b->ntot, b->ncell);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t m = b->ncell, n = b->ntot;
    // the cell counters are clear (see build_cells_impl)
    if (n > 0) {
        hipLaunchKernelGGL(k_bin_batch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n,
                           (const int64_t *)b->d_pstart, b->nbox, (const BoxGeo *)b->d_geo,
                           ws->counts);
        LAUNCHCHK("k_bin_batch");
    }
    if ((rc = scan_counts(ws, m, cell_start, st))) return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter_batch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos,
                           n, (const int64_t *)b->d_pstart, b->nbox, (const BoxGeo *)b->d_geo,
                           cell_start, ws->counts, perm, coord);
        LAUNCHCHK("k_scatter_batch");
    }
    return LC_OK;
}


static int batch_forces_impl(const lc_batch *b, const int32_t *cell_start, const uint32_t *coord,
                             int64_t *F, int64_t *ew, int persistent, lc_workspace *ws,
                             hipStream_t st) {
    int rc = fill64((long long *)ew, 3 * (int64_t)b->nbox, st);
    if (rc) return rc;
    const bool atomic = b->wmode == 1;  // adds into F: clear it first
    if (atomic && (rc = fill64((long long *)F, 3 * b->ntot, st))) return rc;
    const int ng = (int)b->grp_box.size();
    SweepArgs a;
    memset(&a, 0, sizeof a);
    a.grp_task = b->d_grp_task;
    a.grp_foot = b->d_grp_foot;
    a.foot_cells = b->d_foot_cells;
    a.task_ab = b->d_task_ab;
    a.grp_base = 0;
    a.cell_start = cell_start;
    a.coord = coord;
    a.n = b->ntot;
    a.F = (long long *)F;
    a.foot_rep = b->d_foot_rep;
    a.pbuf = atomic ? nullptr : ws->pbuf;
    a.rcnt = atomic ? nullptr : rcnt_of(ws, b->h.rmax, b->ntot);
    a.fx_task = nullptr;
    a.fx_foot = a.fx_rep = a.fx_cnt = nullptr;
    a.fx_tmax = a.fx_fmax = 0;
    a.part = (long long *)ws->part;
    a.flags = ws->flags;
    a.pp = b->ppar[0];
    a.grp_box = b->d_grp_box;
    a.ppar = b->d_ppar;
    a.ew_box = (long long *)ew;
    a.ngroups = ng;
    int *tk = nullptr;
    if (persistent) {
        if ((rc = fill32(b->d_ticket, 1, st))) return rc;
        tk = b->d_ticket;
    }
    if (ng > 0 && (rc = launch_sweep(b->cap, b->wmode, false, b->ff, a, ng, b->ncu, tk, st)))
        return rc;
    if (!atomic && b->ntot > 0) {
        hipLaunchKernelGGL(k_gather_partials, dim3((unsigned)((b->ntot + 255) / 256)), dim3(256), 0,
                           st, (const long long *)ws->pbuf, (const int *)a.rcnt, b->h.rmax,
                           b->ntot, (long long *)F, (long long *)nullptr, (long long *)nullptr);
        LAUNCHCHK("k_gather_partials");
    }
    return LC_OK;
}

extern "C" int lc_batch_forces(const lc_batch *b, const int32_t *cell_start, const uint32_t *coord,
                               int64_t *F, int64_t *ew, int persistent, lc_workspace *ws,
                               void *stream) {
    if (!b || !cell_start || !F || !ew || (b->ntot > 0 && !coord))
        return fail(LC_EINVAL, "lc_batch_forces: null argument");
    int rc = check_ws(ws, b->ntot, b->ncell);
    if (rc) return rc;
    if (b->wmode == 3 && (rc = ensure_pbuf(ws, pbuf_elems(b->h.rmax, b->ntot)))) return rc;
    return batch_forces_impl(b, cell_start, coord, F, ew, persistent, ws, (hipStream_t)stream);
}

extern "C" int lc_batch_graph_create(const lc_batch *b, const int32_t *cell_start,
                                     const uint32_t *coord, int64_t *F, int64_t *ew,
                                     int persistent, lc_workspace *ws, void *stream,
                                     lc_graph **out) {
    if (!b || !out || !stream) return fail(LC_EINVAL, "lc_batch_graph_create: bad arguments");
    int rc = check_ws(ws, b->ntot, b->ncell);
    if (rc) return rc;
    if (b->wmode == 3 && (rc = ensure_pbuf(ws, pbuf_elems(b->h.rmax, b->ntot))))
        return rc;  // outside capture
    hipStream_t st = (hipStream_t)stream;
    lc_graph *gr = new lc_graph();
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = batch_forces_impl(b, cell_start, coord, F, ew, persistent, ws, st);
    hipError_t e = hipStreamEndCapture(st, &gr->graph);
    if (rc || e != hipSuccess) {
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        delete gr;
        return rc ? rc : fail(LC_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr->graph);
        delete gr;
        return fail(LC_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    gr->ws = ws;
    ws->live_graphs++;
    *out = gr;
    return LC_OK;
}

// One force evaluation captured into a graph (the launches of
// lc_compute_forces, in order).  Like the batch graph it pins the
// workspace's replica buffer while it lives.
extern "C" int lc_forces_graph_create(const lc_grid *g, const lc_schedule *s,
                                      const int32_t *cell_start, const uint32_t *coord, int64_t n,
                                      int64_t *F, int64_t *ew, int precision, lc_workspace *ws,
                                      void *stream, lc_graph **out) {
    if (!g || !s || !cell_start || !F || !ew || (n > 0 && !coord) || !out || !stream)
        return fail(LC_EINVAL, "lc_forces_graph_create: bad arguments");
    if (precision != LC_PREC_FP32 && precision != LC_PREC_FP64)
        return fail(LC_EINVAL, "lc_forces_graph_create: precision");
    if (s->nc[0] != g->nc[0] || s->nc[1] != g->nc[1] || s->nc[2] != g->nc[2])
        return fail(LC_EINVAL, "lc_forces_graph_create: schedule built for another grid");
    if (n < 0 || n >= 2147483647LL) return fail(LC_EINVAL, "lc_forces_graph_create: bad n");
    int rc = check_ws(ws, 0, 0);
    if (rc) return rc;
    if (s->h.write_mode == 3 && (rc = ensure_pbuf(ws, pbuf_elems(s->h.rmax, n))))
        return rc;  // outside capture
    hipStream_t st = (hipStream_t)stream;
    lc_graph *gr = new lc_graph();
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = forces_impl(g, s, cell_start, coord, n, F, ew, precision, ws, st);
    hipError_t e = hipStreamEndCapture(st, &gr->graph);
    if (rc || e != hipSuccess) {
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        delete gr;
        return rc ? rc : fail(LC_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr->graph);
        delete gr;
        return fail(LC_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    gr->ws = ws;
    ws->live_graphs++;
    *out = gr;
    return LC_OK;
}

extern "C" int lc_graph_launch(lc_graph *gr, void *stream) {
    if (!gr) return fail(LC_EINVAL, "null graph");
    HIPCHK(hipGraphLaunch(gr->exec, (hipStream_t)stream));
    return LC_OK;
}

extern "C" void lc_graph_free(lc_graph *gr) {
    if (!gr) return;
    if (gr->ws) gr->ws->live_graphs--;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
}
