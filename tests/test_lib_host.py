"""Host-side checks of the HIP library (no GPU needed): the shared library
loads and exports every function include/lc.h declares; the grid, the
serialisation-degree calculation (last-writer recurrence) and the Delta rule
agree with the oracle's independent definitions; the schedule validator
rejects a phase with shared writes."""
import itertools
import os
import re

import numpy as np
import pytest

import oracle as O

lc = pytest.importorskip("paper_1401_4441_amd.lc")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "lc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(lc_[a-z_0-9]+)\s*\(", hdr))
    assert len(declared) >= 15
    L = lc.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(lc.SYMBOLS), declared ^ set(lc.SYMBOLS)


def test_grid_dims_match_oracle():
    for L, rc, skin, even in ((17.0998, 2.5, 0.0, False), (68.399, 2.5, 0.0, True),
                             (170.998, 2.5, 0.6, True), (7.6, 2.5, 0.0, False)):
        g = lc.Grid((L, L, L), rc, skin, even)
        want = O.grid_dims((L, L, L), rc, skin, even)
        assert g.nc == tuple(int(x) for x in want)
    assert lc.Grid((68.399,) * 3, 2.5, even=True).nc == (26, 26, 26)
    assert lc.Grid((170.998,) * 3, 2.5, 0.6, even=True).nc == (54, 54, 54)
    with pytest.raises(lc.LCError):
        lc.Grid((7.4, 20, 20), 2.5)  # 2 cells along x


@pytest.mark.parametrize("dims", [(5, 5, 1), (6, 4, 1), (7, 3, 1), (4, 4, 4),
                                  (6, 6, 6), (5, 3, 4)])
@pytest.mark.parametrize("kind", ["lex", "opt", "best", "bad"])
def test_cp_matches_oracle(dims, kind):
    two_d = dims[2] == 1
    order = {("lex", True): O.ORDER2_NAIVE, ("opt", True): O.ORDER2_OPT,
             ("bad", True): O.ORDER2_BAD,
             ("best", True): [O.INTRA, (1, 0, 0), (1, -1, 0), (1, 1, 0), (0, -1, 0)],
             ("lex", False): O.ORDER3_LEX, ("opt", False): O.ORDER3_OPT,
             ("best", False): O.ORDER3_BEST, ("bad", False): O.ORDER3_BAD}[(kind, two_d)]
    r = lc.serialization_degree(dims, kind)
    o = O.serialization_degree(dims, order)
    assert (r["tasks"], r["cp"]) == (o["T"], o["cp"])
    assert r["speedup"] == pytest.approx(o["S"])


def test_cp_loopex_matches_oracle():
    for dims, order in (((6, 4, 1), O.ORDER2_NAIVE), ((6, 6, 6), O.ORDER3_LEX),
                        ((4, 6, 8), O.ORDER3_LEX)):
        r = lc.serialization_degree(dims, "loopex")
        o = O.serialization_degree(dims, order, loopex=True)
        assert (r["tasks"], r["cp"]) == (o["T"], o["cp"])
        # no stencil displacement: Eq. 2 at Delta = 0 is k, Eq. 3 diverges
        k = dims[0] * dims[1] * dims[2]
        assert r["delta"] == 0
        assert r["s_eq2"] == pytest.approx(O.speedup_eq2(0, k, r["n"])) == k
        assert r["s_max"] == float("inf")


def test_batch_options_rejected_on_host():
    g = lc.Grid((17.1, 17.1, 17.1), 2.5)
    for kw in ({"tile": 999}, {"tile": 256}):
        with pytest.raises(lc.LCError) as e:
            lc.Batch([g], [100], **kw)
        assert e.value.code == -1
    with pytest.raises(KeyError):
        lc.Batch([g], [100], write="nope")


def test_custom_orders_delta_rule_vs_dag():
    """The closed-form Delta rule equals the slope of the exact critical path
    for all 24 intra-first 2D orders."""
    inter = [(0, -1, 0), (1, -1, 0), (1, 0, 0), (1, 1, 0)]
    for p in itertools.permutations(inter):
        order = [O.INTRA] + list(p)
        r = lc.serialization_degree((10, 3, 1), "custom", offsets=order)
        c1 = O.serialization_degree((60, 3, 1), order)["cp"]
        c2 = O.serialization_degree((120, 3, 1), order)["cp"]
        assert r["delta"] == (c2 - c1) / (60 * 3), order
        assert r["s_max"] == pytest.approx(5 / r["delta"])


def test_3d_presets_delta_and_eq2():
    for kind, delta in (("lex", 7), ("opt", 1), ("best", 2), ("bad", 14)):
        r = lc.serialization_degree((30, 10, 10), kind)
        assert r["delta"] == delta and r["n"] == 14
        k = 3000
        assert r["s_eq2"] == pytest.approx(O.speedup_eq2(delta, k, 14))
        assert r["s_max"] == pytest.approx(14 / delta)
    # the paper's 3D domain: exact S sits below the Eq. 2 model, approaching it
    r = lc.serialization_degree((30, 10, 10), "opt")
    assert r["speedup"] < r["s_eq2"] <= 14


def test_level_histogram():
    r = lc.serialization_degree((6, 6, 6), "loopex", hist_len=40)
    h = r["level_hist"]
    assert h.sum() == r["tasks"] and (h[:r["cp"]] > 0).all() and (h[r["cp"]:] == 0).all()
    assert h[0] == 216  # all intra tasks are independent


def test_custom_order_rejects_non_half_shell():
    with pytest.raises(lc.LCError):
        lc.serialization_degree((6, 6, 1), "custom",
                                offsets=[O.INTRA, (1, 0, 0), (-1, 0, 0), (1, 1, 0), (0, 1, 0)])


@pytest.mark.parametrize("kind,nphase", [("loopex", 27), ("block8", 8), ("buffer", 1),
                                         ("atomic_tile", 1), ("atomic_pair", 1)])
def test_schedule_plan_shapes(kind, nphase):
    g = lc.Grid((68.399,) * 3, 2.5, even=True)
    info = lc.schedule_plan(g, kind)
    assert info["nphase"] == nphase
    assert info["ntask"] == 14 * g.ncell
    assert info["max_group_tasks"] <= 512 and info["max_group_cells"] <= 128


def test_schedule_plan_lex_levels_equal_cp():
    g = lc.Grid((17.0998,) * 3, 2.5)
    info = lc.schedule_plan(g, "lex")
    assert info["nphase"] == lc.serialization_degree(g.nc, "lex")["cp"]
    assert info["ntask"] == 14 * 216


def test_block8_on_odd_and_small_grids():
    for L in (17.0998, 20.0, 8.0, 12.5):
        g = lc.Grid((L, L, L), 2.5)
        info = lc.schedule_plan(g, "block8")
        assert info["ntask"] == 14 * g.ncell


@pytest.mark.parametrize("kind", ["buffer", "atomic_tile"])
def test_uncoloured_block_sizes_are_upper_bounds(kind):
    """Uncoloured block kinds cut each axis into ceil(n / size) near-equal
    blocks of at most `size` cells (down to single cells); every task is
    kept.  Tasks join the block of their lower corner cell (per axis the
    smaller coordinate of the two cells), so the footprint of a single-cell
    block is the 2 x 2 x 2 cube above it: 8 cells, and every cell lies in 8
    single-cell footprints."""
    g = lc.Grid((7 * 2.6,) * 3, 2.5)  # 7 cells per axis
    assert tuple(g.nc) == (7, 7, 7)
    one = lc.schedule_plan(g, kind, block=(1, 1, 1))
    assert one["ngroup"] == 343 and one["ntask"] == 14 * 343
    assert one["max_group_cells"] == 8 and one["max_group_tasks"] == 14
    two = lc.schedule_plan(g, kind, block=(1, 1, 2))
    assert two["ngroup"] == 7 * 7 * 4 and two["ntask"] == 14 * 343
    big = lc.schedule_plan(g, kind, block=(2, 3, 3))
    assert big["ngroup"] == 4 * 3 * 3 and big["ntask"] == 14 * 343
    assert big["max_group_cells"] == 3 * 4 * 4  # (2 + 1)(3 + 1)(3 + 1)
    if kind == "buffer":
        assert one["max_replicas"] == 8


def test_fullshell_plan():
    """Full shell: 27 tasks per cell in one phase, home cells written only
    (every cell the home of exactly one group, checked by the validator)."""
    g = lc.Grid((7 * 2.6,) * 3, 2.5)
    info = lc.schedule_plan(g, "fullshell")
    assert info["nphase"] == 1 and info["write_mode"] == 4
    assert info["ntask"] == 27 * 343
    one = lc.schedule_plan(g, "fullshell", block=(1, 1, 1))
    assert one["ngroup"] == 343 and one["max_group_cells"] == 27
    assert one["max_group_tasks"] == 27
    big = lc.schedule_plan(g, "fullshell", block=(2, 2, 2))
    assert big["ngroup"] == 4 * 4 * 4 and big["max_group_cells"] == 64


def test_block8_sizes_are_upper_bounds():
    """BLOCK8 block sizes are upper bounds like the other block kinds: an
    axis of n cells is cut into ceil(n / size) blocks rounded up to an even
    count (the 2-colouring), fewer by twos while a block would be narrower
    than the stencil's reach -- corner grouping grows a footprint by the
    reach towards +x, +y and +z only, so single cells colour at reach 1 and
    blocks of two cells at reach 2."""
    g = lc.Grid((8 * 2.6,) * 3, 2.5)  # 8 cells per axis
    assert g.nc == (8, 8, 8)
    with pytest.raises(lc.LCError):
        lc.schedule_plan(g, "block8", block=(0, 1, 1))
    for blk, ngroup, cells in (((1, 1, 1), 512, 8), ((1, 2, 2), 8 * 4 * 4, 2 * 3 * 3),
                               ((2, 3, 3), 4 * 4 * 4, 3 * 3 * 3)):
        info = lc.schedule_plan(g, "block8", block=blk)
        assert info["nphase"] == 8 and info["ntask"] == 14 * 512, blk
        assert info["ngroup"] == ngroup and info["max_group_cells"] == cells, blk
    # a size covering an axis leaves one block there, and no colours along
    # it: columns of 1 x 1 x 8 cells in 2 x 2 = 4 phases
    cols = lc.schedule_plan(g, "block8", block=(1, 1, 8))
    assert cols["nphase"] == 4 and cols["ngroup"] == 64 and cols["max_group_cells"] == 2 * 2 * 8
    g7 = lc.Grid((7 * 2.6,) * 3, 2.5)  # 7 = 2+2+2+1: ceil(7/2) = 4 blocks, even
    info = lc.schedule_plan(g7, "block8", block=(2, 2, 2))
    assert info["ngroup"] == 4 ** 3 and info["max_group_cells"] == 3 ** 3
    h = lc.Grid((8 * 2.6,) * 3, 2.5, half=True)  # 16 cells per axis, reach 2
    assert h.nc == (16, 16, 16) and h.reach == 2
    for blk in ((1, 1, 1), (2, 2, 2)):  # blocks of one cell would be too narrow
        info = lc.schedule_plan(h, "block8", block=blk)
        assert info["nphase"] == 8 and info["ntask"] == 63 * 16 ** 3
        assert info["ngroup"] == 8 ** 3 and info["max_group_cells"] == 4 ** 3
        assert info["max_group_tasks"] == 63 * 8


def test_validator_rejects_shared_write():
    # phase 0: groups {0,1} and {2,3}; phase 1: {1,2}
    lc.validate_phases(4, [0, 2, 3], [0, 2, 4, 6], [0, 1, 2, 3, 1, 2])
    with pytest.raises(lc.LCError) as e:
        lc.validate_phases(4, [0, 2, 3], [0, 2, 4, 6], [0, 1, 1, 3, 1, 2])
    assert e.value.code == -4


def test_loopex_needs_even_grid():
    g = lc.Grid((17.0998 * 7 / 6,) * 3, 2.5)  # 7 cells per axis
    with pytest.raises(lc.LCError):
        lc.schedule_plan(g, "loopex")


def test_weighted_cp_matches_oracle():
    """Library weighted critical path == the oracle's definition, for random
    cell occupancies."""
    rng = np.random.default_rng(4)
    for dims, kind, order, loopex in (((6, 4, 1), "lex", O.ORDER2_NAIVE, False),
                                      ((5, 4, 3), "opt", O.ORDER3_OPT, False),
                                      ((4, 4, 4), "loopex", O.ORDER3_LEX, True)):
        counts = rng.integers(0, 30, size=int(np.prod(dims))).astype(np.int32)
        r = lc.serialization_degree_weighted(dims, kind, counts)
        A, B = O.lc_tasks(dims, order, loopex)
        w = np.where(A == B, 0.5 * counts[A] * (counts[A] - 1.0),
                     counts[A].astype(float) * counts[B])
        _, cp = O.dag_lc_weighted(A, B, w)
        assert r["cp"] == pytest.approx(cp)
        assert r["work"] == pytest.approx(w.sum())


# ---- cells of side rc/2: the stencil reaches two cells ----------------------

def _half_shell2():
    """The reach-2 half shell, built here from its definition (every offset
    in [-2, 2]^3 with dx > 0, or dx = 0 and dz > 0, or dx = dz = 0 and
    dy < 0), independently of the library's construction."""
    r = range(-2, 3)
    return [(x, y, z) for z in r for y in r for x in r
            if x > 0 or (x == 0 and z > 0) or (x == 0 and z == 0 and y < 0)]


def test_half_shell2_is_a_half_shell():
    h = _half_shell2()
    assert len(h) == 62 and len(set(h)) == 62
    full = {d for d in itertools.product(range(-2, 3), repeat=3) if d != (0, 0, 0)}
    assert {d for d in h} | {tuple(-c for c in d) for d in h} == full


def test_half_grid_dims():
    g = lc.Grid((17.0998,) * 3, 2.5, half=True)
    assert g.reach == 2 and lc.Grid((17.0998,) * 3, 2.5).reach == 1
    # two cells cover rc with the FP32 margin: floor(2 L / (rc (1 + 2^-12)))
    assert g.nc == (13, 13, 13)
    assert lc.Grid((17.0998,) * 3, 2.5, 0.6, half=True).nc == (11, 11, 11)
    with pytest.raises(lc.LCError):
        lc.Grid((6.0, 20, 20), 2.5, half=True)  # 4 cells: a +-2 stencil wraps


def test_half_grid_plans():
    g = lc.Grid((17.0998,) * 3, 2.5, half=True)
    n = g.ncell
    for kind, per_cell in (("buffer", 63), ("atomic_tile", 63), ("atomic_pair", 63),
                           ("fullshell", 125), ("lex", 63)):
        info = lc.schedule_plan(g, kind)
        assert info["ntask"] == per_cell * n, kind
        assert info["max_group_tasks"] <= 512 and info["max_group_cells"] <= 128, kind
    assert lc.schedule_plan(g, "lex")["nphase"] == lc.serialization_degree(
        g.nc, "custom", offsets=[O.INTRA] + sorted(_half_shell2(), key=lambda d: (d[2], d[1], d[0])))["cp"]
    for kind in ("block8", "opt", "best", "bad"):
        with pytest.raises(lc.LCError):
            lc.schedule_plan(g, kind)
    with pytest.raises(lc.LCError):  # 13 cells: no stride-3 colouring
        lc.schedule_plan(g, "loopex")
    g12 = lc.Grid((15.6,) * 3, 2.5, half=True)
    assert g12.nc == (12, 12, 12)
    info = lc.schedule_plan(g12, "loopex")  # 27 colours x 63 offsets, levels validated
    assert info["ntask"] == 63 * g12.ncell and info["nphase"] <= 27 * 63
    # a reach-1 order on a reach-2 grid (or the reverse) is refused
    with pytest.raises(lc.LCError):
        lc.schedule_plan(g, "custom", offsets=O.ORDER3_LEX)
    with pytest.raises(lc.LCError):
        lc.schedule_plan(lc.Grid((17.0998,) * 3, 2.5), "custom",
                         offsets=[O.INTRA] + _half_shell2())


def test_reach2_cp_matches_oracle():
    """The critical path of a reach-2 creation order (library recurrence vs
    the oracle's task list and DAG)."""
    order = [O.INTRA] + sorted(_half_shell2(), key=lambda d: (d[2], d[1], d[0]))
    rev = [O.INTRA] + [tuple(-c for c in d) for d in order[1:]][::-1]
    for dims in ((5, 5, 5), (6, 5, 7)):
        for o in (order, rev):
            r = lc.serialization_degree(dims, "custom", offsets=o)
            want = O.serialization_degree(dims, o)
            assert (r["tasks"], r["cp"]) == (want["T"], want["cp"])
    with pytest.raises(lc.LCError):  # not a complete reach-2 half shell
        lc.serialization_degree((5, 5, 5), "custom", offsets=order[:-1])


# ---- flat (2D) systems: one cell along z, the Fig. 3a stencil ---------------

def test_flat_grid_plans_follow_the_2d_closed_forms():
    """On a flat grid the creation orders are the 2D ones of Fig. 5: their
    level counts are the periodic closed forms (naive (4Nx+1)Ny, bad
    (5Nx-1)Ny+1, opt (Nx+2)Ny+2), loop exchange has 2n - 1 = 9 levels, and
    the tile kinds cover each of the 5 stencil entries per cell once."""
    g = lc.Grid((65.465, 65.465, 10.0), 2.5, flat=True)
    nx, ny, nz = g.nc
    assert (nx, ny, nz) == (26, 26, 1)
    assert lc.schedule_plan(g, "lex")["nphase"] == (4 * nx + 1) * ny
    assert lc.schedule_plan(g, "bad")["nphase"] == (5 * nx - 1) * ny + 1
    assert lc.schedule_plan(g, "opt")["nphase"] == (nx + 2) * ny + 2
    assert lc.schedule_plan(g, "loopex")["nphase"] == 9
    info = lc.schedule_plan(g, "block8", block=(4, 4, 1))
    assert info["nphase"] == 4 and info["ntask"] == 5 * g.ncell
    for kind in ("buffer", "atomic_tile", "atomic_pair"):
        assert lc.schedule_plan(g, kind)["ntask"] == 5 * g.ncell, kind
    assert lc.schedule_plan(g, "fullshell")["ntask"] == 9 * g.ncell
    # blocks of at most 8 x 12: 26 = 7+7+6+6 along x, 9+9+8 along y; tasks
    # join the block of their lower corner cell, so the largest, 7 x 9,
    # reaches (7 + 1) x (9 + 1) cells
    info = lc.schedule_plan(g, "buffer", block=(8, 12, 1))
    assert info["max_group_cells"] == 8 * 10 and info["max_group_tasks"] == 5 * 7 * 9
    with pytest.raises(lc.LCError):
        lc.Grid((65.465, 65.465, 10.0), 2.5, half=True, flat=True)


def test_batch_refuses_half_and_flat_grids():
    """Batched boxes use the 3D rc-cell stencil (their whole-box groups
    too): a box on a half-cell or flat grid is refused before any device
    work."""
    for g in (lc.Grid((17.0998,) * 3, 2.5, half=True),
              lc.Grid((65.465, 65.465, 10.0), 2.5, flat=True)):
        with pytest.raises(lc.LCError, match="3D grids"):
            lc.Batch([lc.Grid((17.0998,) * 3, 2.5), g], [4000, 4000])


def test_new_entry_points_reject_bad_arguments():
    """Argument checks that run before any device work."""
    with pytest.raises(lc.LCError):
        lc.selftest_recip(0x43000000, 0x3E800000)  # empty range
    g = lc.Grid((17.0998,) * 3, 2.5)
    with pytest.raises(lc.LCError):  # wrong number of cell counts
        lc.Schedule(g, "buffer", cell_counts=np.zeros(g.ncell - 1, dtype=np.int32))


def _concurrent_rmw(ncell, phases):
    """Run phases of groups the way a plain read-modify-write kernel does
    when its work-groups run at once: every group reads its cells at the
    start of the phase, adds its tasks' contributions (one unit per cell a
    task writes) and stores the cells back, later groups over earlier ones."""
    F = np.zeros(ncell, dtype=np.int64)
    for groups in phases:
        snap = F.copy()
        for tasks in groups:
            cells = sorted({c for t in tasks for c in set(t)})
            acc = {c: int(snap[c]) for c in cells}
            for t in tasks:
                for c in set(t):
                    acc[c] += 1
            for c in cells:
                F[c] = acc[c]
    return F


def _as_phase_arrays(phases):
    pg, gf, fc = [0], [0], []
    for groups in phases:
        for tasks in groups:
            fc.extend(sorted({c for t in tasks for c in set(t)}))
            gf.append(len(fc))
        pg.append(len(gf) - 1)
    return pg, gf, fc


def test_race_canary():
    """The loop-exchange phases of Sec. VI (for every stencil offset, the
    cells of one parity class, one task per group) pass the validator and a
    concurrent plain read-modify-write gives the sequential sums; merging two
    parity classes into one phase is rejected by the validator (LC_ESCHED),
    and run anyway it loses updates (the race canary)."""
    dims = (4, 4, 4)
    nx, ny, nz = dims
    ncell = nx * ny * nz
    cid = lambda x, y, z: (x % nx) + nx * ((y % ny) + ny * (z % nz))
    offsets = [(0, 0, 0)] + [tuple(d) for d in O.H3]
    seq = np.zeros(ncell, dtype=np.int64)
    good, bad = [], []
    for d in offsets:
        classes = []
        for par in itertools.product((0, 1), repeat=3):
            tasks = []
            for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
                if (x % 2, y % 2, z % 2) == par:
                    t = (cid(x, y, z), cid(x + d[0], y + d[1], z + d[2]))
                    tasks.append(t)
                    for c in set(t):
                        seq[c] += 1
            classes.append([[t] for t in tasks])
        good.extend(classes)
        # two classes one cell apart along x in one phase
        bad.extend([classes[0] + classes[1]] + classes[2:])
    lc.validate_phases(ncell, *_as_phase_arrays(good))
    assert (_concurrent_rmw(ncell, good) == seq).all()
    with pytest.raises(lc.LCError) as e:
        lc.validate_phases(ncell, *_as_phase_arrays(bad))
    assert e.value.code == -4
    lost = seq - _concurrent_rmw(ncell, bad)
    assert (lost >= 0).all() and lost.sum() > 0


def _stencil_tasks(nc, offsets):
    """Every (A, A + o) of the half stencil plus the intra task, by definition."""
    nx, ny, nz = nc
    out = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                a = x + nx * (y + ny * z)
                for o in [(0, 0, 0)] + list(offsets):
                    b = ((x + o[0]) % nx) + nx * (((y + o[1]) % ny) + ny * ((z + o[2]) % nz))
                    out.append((a, b))
    return sorted(out)


def _half_shell(reach):
    r = range(-reach, reach + 1)
    return [(dx, dy, dz) for dz in r for dy in r for dx in r
            if dx > 0 or (dx == 0 and dz > 0) or (dx == 0 and dz == 0 and dy < 0)]


def _coords(c, nc):
    return np.stack([c % nc[0], (c // nc[0]) % nc[1], c // (nc[0] * nc[1])], axis=-1)


@pytest.mark.parametrize("ncell_axis,reach,kind,block", [
    (7, 1, "buffer", (2, 2, 3)), (7, 1, "atomic_tile", (1, 1, 1)), (8, 1, "block8", (1, 1, 1)),
    (8, 1, "block8", (1, 2, 2)), (8, 1, "block8", (1, 1, 8)), (7, 1, "block8", (2, 2, 2)),
    (9, 1, "buffer", (3, 3, 3)), (12, 2, "buffer", (2, 2, 2)),
    (12, 2, "block8", (2, 2, 2)), (13, 2, "atomic_tile", (1, 2, 3))])
def test_tile_tasks_by_corner_cell(ncell_axis, reach, kind, block):
    """The tile kinds keep the stencil's tasks exactly (each (A, A + o) once,
    compared with the stencil written out here), and a task runs in the
    work-group of its lower corner cell C (per axis A + min(o, 0)): every
    cell is the corner of all its tasks in one group, a group's corners form
    a box of at most the block's size, its footprint lies in the box grown
    by the reach towards +, and the groups of one phase touch disjoint
    cells."""
    side = 2.6 if reach == 1 else 1.3
    g = lc.Grid((ncell_axis * side,) * 3, 2.5, half=reach == 2)
    nc = g.nc
    assert nc == (ncell_axis,) * 3 and g.reach == reach
    A, B, G, P = lc.schedule_plan_tasks(g, kind, block=block)
    offs = O.H3 if reach == 1 else _half_shell(2)
    assert len(offs) == (13 if reach == 1 else 62)
    assert sorted(zip(A.tolist(), B.tolist())) == _stencil_tasks(nc, offs)
    n = np.array(nc)
    a, b = _coords(A, nc), _coords(B, nc)
    d = (b - a + reach) % n - reach  # the offset, in [-reach, reach]
    corner = (a + np.minimum(d, 0)) % n
    cid = corner[:, 0] + nc[0] * (corner[:, 1] + nc[1] * corner[:, 2])
    owner = {}
    for c, gg in zip(cid.tolist(), G.tolist()):
        assert owner.setdefault(c, gg) == gg  # one group per corner cell
    assert len(owner) == g.ncell
    for gg in np.unique(G):
        sel = G == gg
        cs = np.unique(cid[sel])
        cc = _coords(cs, nc)
        ext = []
        for ax in range(3):
            vals = sorted(set(cc[:, ax].tolist()))
            # a cyclic interval: the gaps between consecutive values are 1
            # except one wrap-around gap
            gaps = [(vals[(k + 1) % len(vals)] - vals[k]) % nc[ax] for k in range(len(vals))]
            assert len(vals) == nc[ax] or sum(x != 1 for x in gaps) <= 1
            ext.append(len(vals))
        assert len(cs) == ext[0] * ext[1] * ext[2]  # a box
        lim = block if kind != "block8" else tuple(2 * x + 1 for x in block)
        assert all(e <= m for e, m in zip(ext, lim)), (ext, block)
        foot = np.unique(np.concatenate([A[sel], B[sel]]))
        assert len(foot) <= np.prod([e + reach for e in ext])
    if kind == "block8":
        for p in np.unique(P):
            seen = {}
            for gg in np.unique(G[P == p]):
                sel = G == gg
                for c in np.unique(np.concatenate([A[sel], B[sel]])).tolist():
                    assert seen.setdefault(c, gg) == gg, (p, c)
