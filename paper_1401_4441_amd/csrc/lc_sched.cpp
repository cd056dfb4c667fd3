// Host-side cell-task scheduler (see sched.h).
#include "lc_sched.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <unordered_map>

#include "lc.h"

namespace lcs {

namespace {

Offset mk(int x, int y, int z) {
    Offset o;
    o.d[0] = (int8_t)x;
    o.d[1] = (int8_t)y;
    o.d[2] = (int8_t)z;
    return o;
}

bool same(const Offset &a, const Offset &b) {
    return a.d[0] == b.d[0] && a.d[1] == b.d[1] && a.d[2] == b.d[2];
}

bool is_zero(const Offset &a) { return !a.d[0] && !a.d[1] && !a.d[2]; }

int64_t wrap(int64_t a, int64_t m) {
    a %= m;
    return a < 0 ? a + m : a;
}

// (dz, dy, dx) ascending: the linear-index order of the offsets.
bool lin_less(const Offset &a, const Offset &b) {
    if (a.d[2] != b.d[2]) return a.d[2] < b.d[2];
    if (a.d[1] != b.d[1]) return a.d[1] < b.d[1];
    return a.d[0] < b.d[0];
}

}  // namespace

std::vector<Offset> half_stencil(bool two_d) {
    std::vector<Offset> h;
    if (two_d) {
        h = {mk(0, -1, 0), mk(1, -1, 0), mk(1, 0, 0), mk(1, 1, 0)};
        return h;
    }
    for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) h.push_back(mk(1, a, b));
    for (int a = -1; a <= 1; ++a) h.push_back(mk(0, a, 1));
    h.push_back(mk(0, -1, 0));
    return h;
}

std::vector<Offset> half_shell(int reach) {
    if (reach <= 1) return half_stencil(false);
    std::vector<Offset> h;
    const int r = reach;
    for (int dx = 1; dx <= r; ++dx)
        for (int dz = -r; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy) h.push_back(mk(dx, dy, dz));
    for (int dz = 1; dz <= r; ++dz)
        for (int dy = -r; dy <= r; ++dy) h.push_back(mk(0, dy, dz));
    for (int dy = -1; dy >= -r; --dy) h.push_back(mk(0, dy, 0));
    return h;
}

int order_reach(const int8_t *offsets, int n) {
    int r = 1;
    for (int k = 0; offsets && k < 3 * n; ++k) r = std::max(r, std::abs((int)offsets[k]));
    return r;
}

bool stencil_order(int kind, bool two_d, const int8_t *offsets, int n,
                   std::vector<Offset> &order, std::string &err, int reach) {
    order.clear();
    const Offset intra = mk(0, 0, 0), ex = mk(1, 0, 0);
    if (reach < 1 || reach > 2 || (two_d && reach != 1)) {
        err = "stencil reach must be 1 or 2 (3D)";
        return false;
    }
    if (kind == LC_SCHED_CUSTOM) {
        if (!offsets || n <= 0) {
            err = "custom order needs offsets";
            return false;
        }
        for (int k = 0; k < n; ++k)
            order.push_back(mk(offsets[3 * k], offsets[3 * k + 1], offsets[3 * k + 2]));
        // validate: intra once, and one of d / -d for every neighbour
        const int r = reach, w = 2 * r + 1;
        int nz = 0;
        const int want = two_d ? w * w : w * w * w;
        std::vector<int> seen((size_t)(w * w * w), 0);
        for (auto &o : order) {
            for (int d = 0; d < 3; ++d)
                if (o.d[d] < -r || o.d[d] > r) {
                    err = r == 1 ? "offset component outside [-1, 1]"
                                 : "offset component outside [-2, 2]";
                    return false;
                }
            if (two_d && o.d[2]) {
                err = "2D order with nonzero dz";
                return false;
            }
            int k1 = (o.d[0] + r) + w * (o.d[1] + r) + w * w * (o.d[2] + r);
            int k2 = (-o.d[0] + r) + w * (-o.d[1] + r) + w * w * (-o.d[2] + r);
            if (seen[k1] || (k1 != k2 && seen[k2])) {
                err = "offset or its mirror repeated";
                return false;
            }
            seen[k1] = 1;
            nz += is_zero(o) ? 1 : 2;
        }
        if (nz != want) {
            err = "order is not a complete half shell plus intra";
            return false;
        }
        return true;
    }
    if (reach == 2) {
        switch (kind) {
            case LC_SCHED_LEX:
            case LC_SCHED_LOOPEX:
            case LC_SCHED_BLOCK8:
            case LC_SCHED_ATOMIC_TILE:
            case LC_SCHED_ATOMIC_PAIR:
            case LC_SCHED_BUFFER: {
                std::vector<Offset> h2 = half_shell(2);
                std::sort(h2.begin(), h2.end(), lin_less);
                order.push_back(intra);
                for (auto &o : h2) order.push_back(o);
                return true;
            }
            default:
                err = "this kind has no reach-2 preset order (pass the offsets)";
                return false;
        }
    }
    std::vector<Offset> h = half_stencil(two_d);
    std::sort(h.begin(), h.end(), lin_less);
    if (two_d) {
        const Offset bl = mk(0, -1, 0), lr = mk(1, -1, 0), ur = mk(1, 1, 0);
        switch (kind) {
            case LC_SCHED_LEX:  // Fig. 5(a)
            case LC_SCHED_LOOPEX:
            case LC_SCHED_BLOCK8:
            case LC_SCHED_ATOMIC_TILE:
            case LC_SCHED_ATOMIC_PAIR:
            case LC_SCHED_BUFFER: order = {intra, bl, lr, ex, ur}; return true;
            case LC_SCHED_BAD: order = {intra, bl, lr, ur, ex}; return true;   // 5(b)
            case LC_SCHED_OPT: order = {ex, lr, ur, bl, intra}; return true;   // 5(c)
            case LC_SCHED_BEST: order = {intra, ex, lr, ur, bl}; return true;
            default: err = "kind has no 2D order"; return false;
        }
    }
    std::vector<Offset> dx1, dx0;
    for (auto &o : h) {
        if (same(o, ex)) continue;
        (o.d[0] == 1 ? dx1 : dx0).push_back(o);
    }
    switch (kind) {
        case LC_SCHED_LEX:
        case LC_SCHED_LOOPEX:
        case LC_SCHED_BLOCK8:
        case LC_SCHED_ATOMIC_TILE:
        case LC_SCHED_ATOMIC_PAIR:
        case LC_SCHED_BUFFER:
            order.push_back(intra);
            for (auto &o : h) order.push_back(o);
            return true;
        case LC_SCHED_OPT:
            order.push_back(ex);
            for (auto &o : dx1) order.push_back(o);
            for (auto &o : dx0) order.push_back(o);
            order.push_back(intra);
            return true;
        case LC_SCHED_BEST:
            order.push_back(intra);
            order.push_back(ex);
            for (auto &o : dx1) order.push_back(o);
            for (auto &o : dx0) order.push_back(o);
            return true;
        case LC_SCHED_BAD:
            order.push_back(intra);
            for (auto &o : h)
                if (!same(o, ex)) order.push_back(o);
            order.push_back(ex);
            return true;
        default: err = "unknown schedule kind"; return false;
    }
}

void basic_tasks(const int32_t dims[3], const std::vector<Offset> &order,
                 std::vector<int32_t> &A, std::vector<int32_t> &B) {
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    A.clear();
    B.clear();
    A.reserve((size_t)(nx * ny * nz) * order.size());
    B.reserve(A.capacity());
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int32_t a = (int32_t)(x + nx * (y + ny * z));
                for (const Offset &o : order) {
                    A.push_back(a);
                    B.push_back((int32_t)(wrap(x + o.d[0], nx) +
                                          nx * (wrap(y + o.d[1], ny) +
                                                ny * wrap(z + o.d[2], nz))));
                }
            }
}

bool loopex_tasks(const int32_t dims[3], const std::vector<Offset> &order,
                  std::vector<int32_t> &A, std::vector<int32_t> &B, int stride) {
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const bool flat = nz == 1;
    const int s = stride;
    if ((nx % s) || (ny % s) || (!flat && (nz % s))) return false;
    A.clear();
    B.clear();
    const int zc = flat ? 1 : s, zs = flat ? 1 : s;
    for (const Offset &o : order)
        for (int c = 0; c < s * s * zc; ++c) {
            const int cx = c % s, cy = (c / s) % s, cz = c / (s * s);
            for (int64_t z = cz; z < nz; z += zs)
                for (int64_t y = cy; y < ny; y += s)
                    for (int64_t x = cx; x < nx; x += s) {
                        A.push_back((int32_t)(x + nx * (y + ny * z)));
                        B.push_back((int32_t)(wrap(x + o.d[0], nx) +
                                              nx * (wrap(y + o.d[1], ny) +
                                                    ny * wrap(z + o.d[2], nz))));
                    }
        }
    return true;
}

int64_t task_levels(int64_t ncell, const std::vector<int32_t> &A,
                    const std::vector<int32_t> &B,
                    std::vector<int32_t> &level) {
    std::vector<int32_t> last((size_t)ncell, 0);
    level.resize(A.size());
    int64_t cp = 0;
    for (size_t t = 0; t < A.size(); ++t) {
        const int32_t l = 1 + std::max(last[A[t]], last[B[t]]);
        level[t] = l;
        last[A[t]] = l;
        last[B[t]] = l;
        cp = std::max<int64_t>(cp, l);
    }
    return cp;
}

double task_levels_weighted(int64_t ncell, const std::vector<int32_t> &A,
                            const std::vector<int32_t> &B, const std::vector<double> &w) {
    std::vector<double> last((size_t)ncell, 0.0);
    double cp = 0.0;
    for (size_t t = 0; t < A.size(); ++t) {
        const double f = w[t] + std::max(last[(size_t)A[t]], last[(size_t)B[t]]);
        last[(size_t)A[t]] = f;
        last[(size_t)B[t]] = f;
        cp = std::max(cp, f);
    }
    return cp;
}

int delta_rule(const std::vector<Offset> &order) {
    auto pos = [&](const Offset &o) -> int {
        for (size_t k = 0; k < order.size(); ++k)
            if (same(order[k], o)) return (int)k + 1;
        return 0;
    };
    int delta = pos(mk(1, 0, 0));
    for (const Offset &d : order) {
        Offset back = mk(d.d[0] - 1, d.d[1], d.d[2]);
        int pb = pos(back);
        if (pb) delta = std::max(delta, pos(d) - pb + 1);
    }
    return delta;
}

namespace {

// Assemble one work-group from a task list: footprint = distinct cells in
// order of first appearance.
bool add_group(HostSchedule &hs, const std::vector<int32_t> &A,
               const std::vector<int32_t> &B, std::string &err) {
    std::vector<int32_t> cells;
    auto local = [&](int32_t c) -> int {
        for (size_t k = 0; k < cells.size(); ++k)
            if (cells[k] == c) return (int)k;
        cells.push_back(c);
        return (int)cells.size() - 1;
    };
    for (size_t t = 0; t < A.size(); ++t) {
        const int a = local(A[t]), b = local(B[t]);
        hs.task_ab.push_back((uint32_t)a | ((uint32_t)b << 16));
    }
    if ((int)A.size() > kMaxGroupTasks || (int)cells.size() > kMaxGroupCells) {
        err = "work-group exceeds task/cell limits";
        return false;
    }
    hs.foot_cells.insert(hs.foot_cells.end(), cells.begin(), cells.end());
    hs.grp_task.push_back((int32_t)hs.task_ab.size());
    hs.grp_foot.push_back((int32_t)hs.foot_cells.size());
    hs.max_tasks = std::max(hs.max_tasks, (int)A.size());
    hs.max_cells = std::max(hs.max_cells, (int)cells.size());
    hs.ntask += (int64_t)A.size();
    return true;
}

// n cells cut into ceil(n / maxsize) near-equal blocks of at most maxsize
// (the uncoloured block kinds: no parity or spacing constraint).  Returns
// block start offsets with n appended.
std::vector<int> axis_blocks_max(int n, int maxsize) {
    const int m = (n + maxsize - 1) / maxsize;
    const int base = n / m, extra = n % m;
    std::vector<int> s(1, 0);
    int pos = 0;
    for (int b = 0; b < m; ++b) {
        pos += base + (b < extra ? 1 : 0);
        s.push_back(pos);
    }
    return s;
}

// n cells cut into an even number m of near-equal blocks for the 2-colouring
// of BLOCK8: m = ceil(n / maxsize) rounded up to even, then fewer by twos
// while a block would be narrower than `reach`.  Same-coloured blocks are
// then separated by a whole block, which keeps their write footprints apart
// since a footprint reaches `reach` cells past its block (towards + only,
// under corner grouping).  A single block (no colours along this axis) when
// maxsize covers the axis or two blocks do not fit.  Returns block start
// offsets with n appended.
std::vector<int> axis_blocks(int n, int maxsize, int reach) {
    int m = (n + maxsize - 1) / maxsize;
    if (m <= 1) return {0, n};
    if (m & 1) m += 1;
    while (m >= 2 && n < m * reach) m -= 2;
    if (m < 2) return {0, n};
    const int base = n / m, extra = n % m;
    std::vector<int> s(1, 0);
    int pos = 0;
    for (int b = 0; b < m; ++b) {
        pos += base + (b < extra ? 1 : 0);
        s.push_back(pos);
    }
    return s;
}

// The tasks of one block of cells (block bx, by, bz of the partition bs),
// offset-major: for each stencil offset, every cell of the block in x-fastest
// order.  Consecutive tasks then have distinct cells A and distinct cells B,
// so the 64 lanes of a wave, which cover about five consecutive tasks, spread
// their force additions over several cells' particles instead of piling them
// onto one cell A.
//
// corner = false: the block's cells are the tasks' cells A (the stencil task
// of cell A with offset o couples A and A + o); the footprint is the block
// grown by the reach towards +x and both ways along y and z.
// corner = true: a task joins the block that holds its lower corner, the
// cell C = A + min(o, 0) (per axis the smaller of the two cells' coordinates,
// the periodic wrap taken on the side the pair reaches across).  For a block
// cell C and offset o the task couples C + max(-o, 0) and C + max(o, 0): the
// stencil task of cell A = C + max(-o, 0), the same (A, B) pair, so the task
// set is the stencil's and each pair is kept once.  Both cells lie in C +
// {0..reach}^3, so the footprint is the block grown by the reach towards +x,
// +y and +z only -- (bx + r)(by + r)(bz + r) cells against about
// (bx + r)(by + 2r)(bz + 2r).
void block_tasks(const int32_t nc[3], const std::vector<int> bs[3], int bx, int by, int bz,
                 const std::vector<Offset> &offs, std::vector<int32_t> &A,
                 std::vector<int32_t> &B, bool corner = false) {
    auto cell = [&](int x, int y, int z) -> int32_t {
        return (int32_t)(wrap(x, nc[0]) + nc[0] * (wrap(y, nc[1]) + nc[1] * wrap(z, nc[2])));
    };
    for (const Offset &o : offs) {
        int sa[3], sb[3];  // cell A and cell B relative to the block cell
        for (int d = 0; d < 3; ++d) {
            sa[d] = corner ? std::max(-(int)o.d[d], 0) : 0;
            sb[d] = sa[d] + o.d[d];
        }
        for (int z = bs[2][bz]; z < bs[2][bz + 1]; ++z)
            for (int y = bs[1][by]; y < bs[1][by + 1]; ++y)
                for (int x = bs[0][bx]; x < bs[0][bx + 1]; ++x) {
                    A.push_back(cell(x + sa[0], y + sa[1], z + sa[2]));
                    B.push_back(cell(x + sb[0], y + sb[1], z + sb[2]));
                }
    }
}

}  // namespace

int build_schedule(const int32_t nc[3], int kind, const int8_t *offsets,
                   int n, HostSchedule &hs, std::string &err, const int32_t *block_min,
                   int reach) {
    if (reach != 1 && reach != 2) {
        err = "stencil reach must be 1 or 2";
        return LC_EINVAL;
    }
    // a flat grid (one cell along z): the 2D stencil and orders
    const bool flat = nc[2] == 1;
    if (flat && reach != 1) {
        err = "flat grids take the reach-1 2D stencil";
        return LC_EINVAL;
    }
    if (kind == LC_SCHED_CUSTOM && order_reach(offsets, n) != reach) {
        err = "custom offsets must reach as far as the grid's stencil";
        return LC_EINVAL;
    }
    // Block sizes are upper bounds for every block kind.  (The tiled
    // Newton-3 kinds group tasks by their lower corner cell, so a block's
    // footprint grows by the reach towards +x, +y and +z only: BLOCK8's
    // same-coloured blocks stay apart when every block spans at least the
    // reach, which its partition ensures.)
    const bool coloured = kind == LC_SCHED_BLOCK8;  // FULLSHELL: uncoloured
    // defaults: blocks of at most 1 x 3 x 3 cells; at reach 2, 2 x 2 x 2 for
    // BLOCK8 and 1 x 2 x 2 for the uncoloured kinds (63 tasks per cell)
    int32_t bmin[3] = {1, 3, 3};
    if (reach == 2) {
        bmin[0] = coloured ? 2 : 1;
        bmin[1] = bmin[2] = 2;
    }
    if (block_min) {
        for (int d = 0; d < 3; ++d) bmin[d] = block_min[d];
        if (bmin[0] < 1 || bmin[1] < 1 || bmin[2] < 1 || bmin[0] > 64 || bmin[1] > 64 ||
            bmin[2] > 64) {
            err = "block sizes must be >= 1 and <= 64";
            return LC_EINVAL;
        }
    }
    hs = HostSchedule();
    hs.kind = kind;
    hs.grp_task.push_back(0);
    hs.grp_foot.push_back(0);
    hs.phase_grp.push_back(0);
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];

    if (kind == LC_SCHED_FULLSHELL) {
        // Blocks of home cells (sizes as upper bounds; default 1 x 2 x 2),
        // each home cell with its intra task and its 26 full-shell
        // neighbours; foot_rep marks the home cells (1), which alone are
        // written.
        // (default 1 x 1 x 1 at reach 2: a 125-cell footprint)
        static const int32_t dflt[3] = {1, 2, 2}, dflt2[3] = {1, 1, 1};
        const int32_t *sz = block_min ? bmin : (reach == 2 ? dflt2 : dflt);
        std::vector<int> bs[3];
        for (int d = 0; d < 3; ++d) bs[d] = axis_blocks_max(nc[d], sz[d]);
        std::vector<Offset> shell(1, Offset{{0, 0, 0}});
        const int rz = flat ? 0 : reach;
        for (int dz = -rz; dz <= rz; ++dz)
            for (int dy = -reach; dy <= reach; ++dy)
                for (int dx = -reach; dx <= reach; ++dx)
                    if (dx || dy || dz) shell.push_back(Offset{{(int8_t)dx, (int8_t)dy, (int8_t)dz}});
        hs.write_mode = 4;
        struct G {
            std::vector<int32_t> A, B;
        };
        std::vector<G> groups;
        for (size_t bz = 0; bz + 1 < bs[2].size(); ++bz)
            for (size_t by = 0; by + 1 < bs[1].size(); ++by)
                for (size_t bx = 0; bx + 1 < bs[0].size(); ++bx) {
                    G gr;
                    block_tasks(nc, bs, (int)bx, (int)by, (int)bz, shell, gr.A, gr.B);
                    groups.push_back(std::move(gr));
                }
        std::stable_sort(groups.begin(), groups.end(),
                         [](const G &x, const G &y) { return x.A.size() > y.A.size(); });
        for (const G &gr : groups) {
            const size_t f0 = hs.foot_cells.size();
            if (!add_group(hs, gr.A, gr.B, err)) return LC_ECAPACITY;
            for (size_t f = f0; f < hs.foot_cells.size(); ++f)
                hs.foot_rep.push_back(
                    std::find(gr.A.begin(), gr.A.end(), hs.foot_cells[f]) != gr.A.end() ? 1 : 0);
        }
        hs.phase_grp.push_back((int32_t)(hs.grp_task.size() - 1));
        return LC_OK;
    }

    std::vector<Offset> order;
    if (!stencil_order(kind, flat, offsets, n, order, err, reach)) return LC_EINVAL;

    if (kind == LC_SCHED_BLOCK8 || kind == LC_SCHED_ATOMIC_TILE || kind == LC_SCHED_BUFFER) {
        hs.write_mode = kind == LC_SCHED_BLOCK8 ? 0 : (kind == LC_SCHED_ATOMIC_TILE ? 1 : 3);
        std::vector<int> bs[3];
        for (int d = 0; d < 3; ++d)
            // (uncoloured kinds at reach 2 default to blocks of at most
            // 1 x 2 x 2: their footprints stay inside the work-group limits)
            bs[d] = (!coloured && (block_min || reach == 2)) ? axis_blocks_max(nc[d], bmin[d])
                                                             : axis_blocks(nc[d], bmin[d], reach);
        const int nb[3] = {(int)bs[0].size() - 1, (int)bs[1].size() - 1,
                           (int)bs[2].size() - 1};
        const int ncol[3] = {nb[0] > 1 ? 2 : 1, nb[1] > 1 ? 2 : 1, nb[2] > 1 ? 2 : 1};
        {
            // footprint extent per axis: the largest block plus the stencil
            // reach (corner grouping: towards + only)
            hs.compact = true;
            for (int d = 0; d < 3; ++d) {
                int big = 0;
                for (int b = 0; b < nb[d]; ++b) big = std::max(big, bs[d][b + 1] - bs[d][b]);
                const int extent = big + reach;
                if (2 * extent >= nc[d]) hs.compact = false;
            }
        }
        const int nphase_col = ncol[0] * ncol[1] * ncol[2];
        for (int ph = 0; ph < nphase_col; ++ph) {
            const int col[3] = {ph % ncol[0], (ph / ncol[0]) % ncol[1],
                                ph / (ncol[0] * ncol[1])};
            // groups of this phase, launched largest first (longest-
            // processing-time order: the big blocks start early and the
            // phase tail is short)
            std::vector<std::pair<std::vector<int32_t>, std::vector<int32_t>>> groups;
            for (int bz = 0; bz < nb[2]; ++bz)
                for (int by = 0; by < nb[1]; ++by)
                    for (int bx = 0; bx < nb[0]; ++bx) {
                        if ((bx % ncol[0]) != col[0] || (by % ncol[1]) != col[1] ||
                            (bz % ncol[2]) != col[2])
                            continue;
                        std::vector<int32_t> A, B;
                        block_tasks(nc, bs, bx, by, bz, order, A, B, true);
                        groups.emplace_back(std::move(A), std::move(B));
                    }
            std::stable_sort(groups.begin(), groups.end(), [](const auto &x, const auto &y) {
                return x.first.size() > y.first.size();
            });
            for (auto &gr : groups)
                if (!add_group(hs, gr.first, gr.second, err)) return LC_ECAPACITY;
            if (kind == LC_SCHED_BLOCK8)
                hs.phase_grp.push_back((int32_t)(hs.grp_task.size() - 1));
        }
        if (kind != LC_SCHED_BLOCK8)
            hs.phase_grp.push_back((int32_t)(hs.grp_task.size() - 1));
        if (kind == LC_SCHED_BUFFER) {
            // replica slot r of (group, cell): the r-th group whose footprint
            // holds the cell writes slot r of its particles
            hs.cell_rep.assign((size_t)ncell, 0);
            hs.foot_rep.resize(hs.foot_cells.size());
            for (size_t k = 0; k < hs.foot_cells.size(); ++k) {
                hs.foot_rep[k] = hs.cell_rep[(size_t)hs.foot_cells[k]]++;
                hs.rmax = std::max(hs.rmax, hs.cell_rep[(size_t)hs.foot_cells[k]]);
            }
        }
        return LC_OK;
    }

    if (kind == LC_SCHED_ATOMIC_PAIR) {
        hs.write_mode = 2;
        // footprint of a home cell: 1 + reach cells along x, 1 + 2 reach
        // along y and z
        hs.compact = 2 * (1 + reach) < nc[0] && 2 * (1 + 2 * reach) < nc[1] &&
                     2 * (1 + 2 * reach) < nc[2];
        std::vector<int32_t> A, B;
        basic_tasks(nc, order, A, B);
        const size_t per = order.size();
        for (size_t c = 0; c < (size_t)ncell; ++c) {
            std::vector<int32_t> a(A.begin() + c * per, A.begin() + (c + 1) * per);
            std::vector<int32_t> b(B.begin() + c * per, B.begin() + (c + 1) * per);
            if (!add_group(hs, a, b, err)) return LC_ECAPACITY;
        }
        hs.phase_grp.push_back((int32_t)(hs.grp_task.size() - 1));
        return LC_OK;
    }

    // Creation-order kinds: execute the DAG level by level.
    std::vector<int32_t> A, B;
    if (kind == LC_SCHED_LOOPEX) {
        if (!loopex_tasks(nc, order, A, B, reach + 1)) {
            err = reach == 1 ? "loop-exchange colouring needs even cell counts"
                             : "loop-exchange colouring at reach 2 needs cell counts divisible by 3";
            return LC_EINVAL;
        }
    } else {
        basic_tasks(nc, order, A, B);
    }
    std::vector<int32_t> level;
    const int64_t cp = task_levels(ncell, A, B, level);
    hs.cp = cp;
    // the creation order itself, for the dataflow executors
    hs.order_a = A;
    hs.order_b = B;
    hs.chain = kind == LC_SCHED_LOOPEX ? 0 : (int)order.size();
    // bucket tasks by level, keeping creation order inside a level
    std::vector<int64_t> cnt((size_t)cp + 2, 0);
    for (int32_t l : level) cnt[(size_t)l + 1]++;
    for (size_t l = 1; l < cnt.size(); ++l) cnt[l] += cnt[l - 1];
    std::vector<int32_t> byl(A.size());
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end());
        for (size_t t = 0; t < A.size(); ++t) byl[(size_t)fill[(size_t)level[t]]++] = (int32_t)t;
    }
    hs.write_mode = 0;
    for (int64_t l = 1; l <= cp; ++l) {
        for (int64_t k = cnt[(size_t)l]; k < cnt[(size_t)l + 1]; k += kLevelGroupTasks) {
            const int64_t e = std::min<int64_t>(k + kLevelGroupTasks, cnt[(size_t)l + 1]);
            std::vector<int32_t> a, b;
            for (int64_t q = k; q < e; ++q) {
                a.push_back(A[(size_t)byl[(size_t)q]]);
                b.push_back(B[(size_t)byl[(size_t)q]]);
            }
            if (!add_group(hs, a, b, err)) return LC_ECAPACITY;
        }
        hs.phase_grp.push_back((int32_t)(hs.grp_task.size() - 1));
    }
    return LC_OK;
}

std::vector<double> group_work(const HostSchedule &hs, const int32_t *cell_counts) {
    const size_t ng = hs.grp_task.empty() ? 0 : hs.grp_task.size() - 1;
    std::vector<double> w(ng, 0.0);
    for (size_t g = 0; g < ng; ++g) {
        const int32_t *fc = hs.foot_cells.data() + hs.grp_foot[g];
        for (int t = hs.grp_task[g]; t < hs.grp_task[g + 1]; ++t) {
            const uint32_t ab = hs.task_ab[(size_t)t];
            const int la = (int)(ab & 0xffffu), lb = (int)(ab >> 16);
            const double na = cell_counts[fc[la]], nb = cell_counts[fc[lb]];
            w[g] += la == lb ? na * (na - 1.0) * 0.5 : na * nb;
        }
    }
    return w;
}

void order_groups_by_work(HostSchedule &hs, const int32_t *cell_counts) {
    const std::vector<double> w = group_work(hs, cell_counts);
    const size_t ng = w.size();
    std::vector<int32_t> perm(ng);
    for (size_t g = 0; g < ng; ++g) perm[g] = (int32_t)g;
    const int nphase = (int)hs.phase_grp.size() - 1;
    for (int p = 0; p < nphase; ++p)
        std::stable_sort(perm.begin() + hs.phase_grp[p], perm.begin() + hs.phase_grp[p + 1],
                         [&](int32_t a, int32_t b) { return w[(size_t)a] > w[(size_t)b]; });
    HostSchedule out = hs;
    out.grp_task.assign(1, 0);
    out.grp_foot.assign(1, 0);
    out.task_ab.clear();
    out.foot_cells.clear();
    out.foot_rep.clear();
    for (int32_t g : perm) {
        out.task_ab.insert(out.task_ab.end(), hs.task_ab.begin() + hs.grp_task[g],
                           hs.task_ab.begin() + hs.grp_task[g + 1]);
        out.foot_cells.insert(out.foot_cells.end(), hs.foot_cells.begin() + hs.grp_foot[g],
                              hs.foot_cells.begin() + hs.grp_foot[g + 1]);
        if (!hs.foot_rep.empty())
            out.foot_rep.insert(out.foot_rep.end(), hs.foot_rep.begin() + hs.grp_foot[g],
                                hs.foot_rep.begin() + hs.grp_foot[g + 1]);
        out.grp_task.push_back((int32_t)out.task_ab.size());
        out.grp_foot.push_back((int32_t)out.foot_cells.size());
    }
    if (out.write_mode == 3) {  // replica slot r: the r-th group, in launch order
        std::fill(out.cell_rep.begin(), out.cell_rep.end(), 0);
        out.rmax = 0;
        for (size_t k = 0; k < out.foot_cells.size(); ++k) {
            out.foot_rep[k] = out.cell_rep[(size_t)out.foot_cells[k]]++;
            out.rmax = std::max(out.rmax, out.cell_rep[(size_t)out.foot_cells[k]]);
        }
    }
    hs = std::move(out);
}

bool validate(const HostSchedule &hs, int64_t ncell, std::string &err) {
    if (hs.write_mode == 4) {
        // full shell: every cell is the home (written) cell of exactly one
        // work-group
        std::vector<int32_t> home((size_t)ncell, 0);
        for (size_t f = 0; f < hs.foot_cells.size(); ++f) {
            const int32_t c = hs.foot_cells[f];
            if (c < 0 || c >= ncell || f >= hs.foot_rep.size()) {
                err = "footprint cell out of range";
                return false;
            }
            if (hs.foot_rep[f]) home[(size_t)c]++;
        }
        for (int64_t c = 0; c < ncell; ++c)
            if (home[(size_t)c] != 1) {
                err = "cell " + std::to_string(c) + " is the home cell of " +
                      std::to_string(home[(size_t)c]) + " work-groups";
                return false;
            }
        return true;
    }
    if (hs.write_mode != 0) return true;  // atomic write-back needs no colouring
    std::vector<int32_t> owner((size_t)ncell, -1);
    std::vector<int32_t> stamp((size_t)ncell, -1);
    const int nphase = (int)hs.phase_grp.size() - 1;
    for (int p = 0; p < nphase; ++p)
        for (int g = hs.phase_grp[p]; g < hs.phase_grp[p + 1]; ++g)
            for (int f = hs.grp_foot[g]; f < hs.grp_foot[g + 1]; ++f) {
                const int32_t c = hs.foot_cells[f];
                if (c < 0 || c >= ncell) {
                    err = "footprint cell out of range";
                    return false;
                }
                if (stamp[c] == p && owner[c] != g) {
                    err = "phase " + std::to_string(p) + ": cell " + std::to_string(c) +
                          " written by two work-groups";
                    return false;
                }
                stamp[c] = p;
                owner[c] = g;
            }
    return true;
}

}  // namespace lcs
