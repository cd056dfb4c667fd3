// Host-side cell-task scheduler: creation orders, task DAG levels, phase and
// work-group construction, validation, and the serialisation-degree model.
// Pure C++ (no HIP); the device upload lives in lc.hip.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace lcs {

struct Offset {
    int8_t d[3];
};

// Fig. 3 half stencils.  3D: the whole +x layer (9), the three +z cells of
// the centre layer, the cell below the centre (axes read from the drawing as
// depth = z, right = x, up = y).  2D: below, and the three cells of the +x
// column.
std::vector<Offset> half_stencil(bool two_d);

// The 3D half shell of a stencil reaching `reach` cells (1 or 2; cells of side
// >= rc / reach): the same construction as the reach-1 one above -- every
// offset with dx > 0, those with dx = 0 and dz > 0, and those with dx = dz = 0
// and dy < 0 -- so 13 offsets at reach 1 (the Fig. 3 set) and 62 at reach 2.
std::vector<Offset> half_shell(int reach);

// Stencil evaluation order (intra = (0,0,0) included) of a preset kind
// (LC_SCHED_LEX/OPT/BEST/BAD/LOOPEX), or the caller's order for CUSTOM.
// reach: the stencil's reach in cells (1, or 2 for cells of side >= rc/2;
// at reach 2 the presets are the linear-index order of half_shell(2), and
// OPT/BEST/BAD have none).  A CUSTOM order must be a complete half shell of
// the same reach.  Returns false with `err` set when the order is not a valid
// half shell.
bool stencil_order(int kind, bool two_d, const int8_t *offsets, int n,
                   std::vector<Offset> &order, std::string &err, int reach = 1);

// The reach of a CUSTOM order: the largest offset component (1 or 2).
int order_reach(const int8_t *offsets, int n);

// Tasks (cellA, cellB) in creation order.
//   basic:  for z, for y, for x: for each entry of `order`
//   loopex: for each entry of `order`: for each colour in {0,1}^D (x
//           fastest): for each cell of that colour (x fastest)
void basic_tasks(const int32_t dims[3], const std::vector<Offset> &order,
                 std::vector<int32_t> &A, std::vector<int32_t> &B);
// Loop exchange colours cells with stride `stride` along each axis
// (stride^D colours; stride = reach + 1 keeps a colour's tasks of one offset
// disjoint); every cell count must be a multiple of the stride.
bool loopex_tasks(const int32_t dims[3], const std::vector<Offset> &order,
                  std::vector<int32_t> &A, std::vector<int32_t> &B, int stride = 2);

// DAG level of every task under the inout rule, by the last-writer
// recurrence: level[t] = 1 + max(last[A_t], last[B_t]), then both cells'
// last = level[t].  Returns the critical path (max level).
int64_t task_levels(int64_t ncell, const std::vector<int32_t> &A,
                    const std::vector<int32_t> &B,
                    std::vector<int32_t> &level);

// Weighted version: finish[t] = w[t] + max(finish of the last task on A,
// on B); returns the largest finish time.
double task_levels_weighted(int64_t ncell, const std::vector<int32_t> &A,
                            const std::vector<int32_t> &B, const std::vector<double> &w);

// Stencil displacement Delta of an evaluation order over a periodic row.
// Stencils at x and x + e_x are both full chains through their centre cell;
// stencil x+1 touches cell x+d (d in stencil, d - e_x in stencil) with its
// task at position pos(d - e_x), after stencil x touched it at pos(d); and
// its first task touches its own centre, which stencil x wrote at pos(e_x).
// Hence Delta = max(pos(e_x), max_d [pos(d) - pos(d - e_x) + 1]).
int delta_rule(const std::vector<Offset> &order);

// Device-ready schedule in host memory.
struct HostSchedule {
    int kind = 0;
    int write_mode = 0;  // 0 plain, 1 atomic tile, 2 atomic pair, 3 replicas, 4 home only
    std::vector<int32_t> phase_grp;   // nphase + 1
    std::vector<int32_t> grp_task;    // ngroup + 1 (index into task_ab)
    std::vector<int32_t> grp_foot;    // ngroup + 1 (index into foot_cells)
    std::vector<int32_t> foot_cells;  // global cell id per footprint slot
    std::vector<uint32_t> task_ab;    // local a | (local b << 16)
    int64_t ntask = 0;
    int max_tasks = 0;
    int max_cells = 0;
    // every group's footprint spans less than half the box along each axis
    // (group-relative float coordinates then reproduce minimum images)
    bool compact = false;
    // buffer + reduce: replica slot of every footprint entry (parallel to
    // foot_cells), replica count per cell, and its maximum; full shell
    // (write mode 4): foot_rep = 1 for the group's home cells
    std::vector<int32_t> foot_rep;
    std::vector<int32_t> cell_rep;
    int rmax = 0;
    // creation-order kinds: the tasks in creation order (cell A, cell B),
    // the critical path, and the per-cell chain length of the basic
    // traversal (tasks [c * chain, (c + 1) * chain) are cell c's stencil;
    // 0 for loop exchange, whose order has no per-cell chains)
    std::vector<int32_t> order_a, order_b;
    int64_t cp = 0;
    int chain = 0;
};

constexpr int kMaxGroupTasks = 512;
constexpr int kMaxGroupCells = 128;
constexpr int kLevelGroupTasks = 16;

// Build the schedule of `kind` on grid `nc` (LC_SCHED_*).  Returns 0 or a
// negative LC_E* code with `err` set.
// block_min (may be NULL): smallest block per axis for the block kinds
// (default {1, 2, 2}; at least 1 along x and 2 along y and z, the stencil's
// reach on each side).  reach: 1, or 2 on grids of cells of side >= rc/2
// (no BLOCK8 there: its blocks would exceed the work-group limits).
int build_schedule(const int32_t nc[3], int kind, const int8_t *offsets,
                   int n, HostSchedule &hs, std::string &err,
                   const int32_t *block_min = nullptr, int reach = 1);

// Every phase's work-groups write pairwise disjoint cells (required for
// plain read-modify-write).  Returns true when valid.
bool validate(const HostSchedule &hs, int64_t ncell, std::string &err);

// Estimated work of every work-group, in launch order: the sum over its
// tasks of n_A n_B (n_A (n_A - 1) / 2 for an intra task) from per-cell
// particle counts -- the task weights of the weighted critical path.
std::vector<double> group_work(const HostSchedule &hs, const int32_t *cell_counts);

// Reorder the work-groups of every phase by group_work, largest first
// (longest-processing-time order: the heavy groups start early and the
// launch ends on light ones).  Replica slots (buffer + reduce) are
// reassigned in the new order.  Tasks inside a group keep their order.
void order_groups_by_work(HostSchedule &hs, const int32_t *cell_counts);

}  // namespace lcs
