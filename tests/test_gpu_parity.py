"""GPU parity: the HIP path (through the C-ABI binding) against the oracle.

Bar: forces, energies, virials and pair counts are int64 and must be
bit-exact against the oracle's fixed-point link-cell sweep for every
schedule; cell_start must match exactly and cell membership as sets; the
FP64-arithmetic variant must sit within 2e-7 normwise of the FP64 oracle
(their only difference is the box-fraction quantisation of the positions,
a step of L * 2^-32 = 4e-9 at L = 17.1; the LJ force changes by a factor
of about 14 / r ~ 15 per unit relative displacement near contact, giving
~6e-8, with a margin of 3); the FP32 path within 1e-5 normwise and per particle within
1e-5 * sum_j |f_ij| of FP64; Verlet trajectories bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import synth

pytestmark = pytest.mark.gpu

lc = pytest.importorskip("paper_1401_4441_amd.lc")

DEV = torch.device("cuda:0")
KINDS = ["block8", "buffer", "atomic_tile", "atomic_pair", "loopex", "opt", "lex", "fullshell"]


def _say(*a):
    print(*a, flush=True)


class Setup:
    def __init__(self, box, skin=0.0, even=False, half=False, flat=False):
        self.box = box
        self.g = lc.Grid(box.L, box.rc, skin, even, half=half, flat=flat)
        self.ws = lc.Workspace(box.n, self.g.ncell)
        self.pos = torch.from_numpy(box.pos).to(DEV)
        self.cs, self.perm, self.coord = lc.build_cells(self.g, self.pos, self.ws)
        self.perm_h = self.perm.cpu().numpy()
        self.u = O.canonical(box.pos, box.L)

    def unsort(self, F):
        Fh = F.cpu().numpy()
        out = np.empty_like(Fh)
        out[:, self.perm_h] = Fh
        return out

    def forces(self, kind, precision="fp32", block=None, offsets=None):
        s = lc.Schedule(self.g, kind, offsets=offsets, block=block)
        self.ws.clear_status()
        F, ew = lc.compute_forces(self.g, s, self.cs, self.coord, self.ws, precision)
        torch.cuda.synchronize()
        return self.unsort(F), [int(x) for x in ew.cpu().numpy()], self.ws.status()


_c1 = None


def c1():
    global _c1
    if _c1 is None:
        _c1 = Setup(synth.fcc(4000, 0.8, rc=2.5, seed=1001))
    return _c1


def test_build_cells_c1():
    S = c1()
    _say("build_cells fcc4k nc", S.g.nc)
    cs = S.cs.cpu().numpy()
    assert (cs == O.cell_start(S.u, S.g.nc)).all()
    perm = S.perm_h
    assert np.array_equal(np.sort(perm), np.arange(S.box.n))
    # slot k lies in the cell whose range contains k (membership as sets)
    cid = O.cell_ids(S.u, S.g.nc)
    slot_cell = np.repeat(np.arange(S.g.ncell), np.diff(cs))
    assert (cid[perm] == slot_cell).all()
    coord = S.coord.cpu().numpy().view(np.uint32)
    assert (coord == S.u[:, perm]).all()


def test_cell_build_reuses_workspace_counters():
    """Each scan leaves the per-cell counters and its tile status words
    cleared for the next build: builds on one workspace that alternate a
    grid of one scan tile (6^3 cells) and one of 17 tiles (41^3 = 68,921
    cells) all match the oracle's cell table."""
    small = synth.fcc(4000, 0.8, rc=2.5, seed=51)
    big = synth.fcc(20000, 0.0185, rc=2.5, seed=52)
    gs, gb = lc.Grid(small.L, small.rc), lc.Grid(big.L, big.rc)
    assert gs.ncell <= 65536 < gb.ncell
    ws = lc.Workspace(big.n, gb.ncell)
    for box, g in ((small, gs), (big, gb), (small, gs), (big, gb), (big, gb)):
        _say("cell build", g.nc)
        cs, perm, coord = lc.build_cells(g, torch.from_numpy(box.pos).to(DEV), ws)
        u = O.canonical(box.pos, box.L)
        csh = cs.cpu().numpy()
        assert (csh == O.cell_start(u, g.nc)).all()
        slot_cell = np.repeat(np.arange(g.ncell), np.diff(csh))
        assert (O.cell_ids(u, g.nc)[perm.cpu().numpy()] == slot_cell).all()


def _check_build(box, g, cs, perm, coord):
    u = O.canonical(box.pos, box.L)
    csh = cs.cpu().numpy()
    assert (csh == O.cell_start(u, g.nc)).all()
    ph = perm.cpu().numpy()
    assert np.array_equal(np.sort(ph), np.arange(box.n))
    slot_cell = np.repeat(np.arange(g.ncell), np.diff(csh))
    assert (O.cell_ids(u, g.nc)[ph] == slot_cell).all()
    assert (coord.cpu().numpy().view(np.uint32) == u[:, ph]).all()


def test_cell_build_sizes_and_orders():
    """The cell build gives the oracle's cell table, a permutation with the
    oracle's cell membership and the matching box fractions: ragged sizes,
    one particle, a shuffled order, 256k in lattice order, and builds that
    alternate sizes on one workspace (counters and the bin pass's completion
    counter reset)."""
    cases = [synth.fcc(1, 0.8, rc=2.5, seed=61), synth.fcc(1234, 0.8, rc=2.5, seed=62),
             synth.fcc(4000, 0.8, rc=2.5, seed=63), synth.fcc(256000, 0.8, rc=2.5, seed=1002)]
    cases[0].L = np.array([8.0, 8.0, 8.0])  # one particle in a 3^3 grid
    sh = synth.fcc(70001, 0.7, rc=2.5, seed=64)
    sh.pos = np.ascontiguousarray(sh.pos[:, np.random.default_rng(5).permutation(sh.n)])
    cases.append(sh)
    grids = [lc.Grid(b.L, b.rc) for b in cases]
    ws = lc.Workspace(max(b.n for b in cases), max(g.ncell for g in grids))
    for b, g in list(zip(cases, grids)) + list(zip(cases, grids))[::-1]:
        _say("cell build", b.n, g.nc)
        cs, perm, coord = lc.build_cells(g, torch.from_numpy(b.pos).to(DEV), ws)
        _check_build(b, g, cs, perm, coord)
    assert ws.status() == 0


def test_cell_build_two_million():
    """The 2M slab (dense and dilute cells, 64^3 = 262,144 cells: the
    64 scan tiles)."""
    box = synth.workload("slab2m")
    g = lc.Grid(box.L, box.rc)
    ws = lc.Workspace(box.n, g.ncell)
    _say("cell build slab2m", g.nc)
    cs, perm, coord = lc.build_cells(g, torch.from_numpy(box.pos).to(DEV), ws)
    _check_build(box, g, cs, perm, coord)
    assert ws.status() == 0


@pytest.mark.parametrize("kind", KINDS)
def test_forces_bit_exact_c1(kind):
    S = c1()
    _say("forces fcc4k", kind)
    F, ew, st = S.forces(kind)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, S.box.L, S.box.rc, S.g.nc)
    assert st & lc.FLAG_OVERFLOW == 0
    assert (F == Fo).all()
    assert ew == [Eo, Wo, npo]


def test_fp64_variant_and_fp32_error_c1():
    S = c1()
    _say("fp64 variant fcc4k")
    F64g, ew64, _ = S.forces("block8", "fp64")
    F32g, ew32, _ = S.forces("block8", "fp32")
    F, mag, U, W, npairs = O.forces_brute_f64(S.box.pos, S.box.L, S.box.rc, u=S.u)
    assert ew64[2] == ew32[2] == npairs
    err64 = np.linalg.norm(F64g / lc.SCALE - F) / np.linalg.norm(F)
    assert err64 <= 2e-7
    Fx = F32g / lc.SCALE
    err32 = np.linalg.norm(Fx - F) / np.linalg.norm(F)
    assert err32 <= 1e-5
    assert (np.abs(Fx - F).max(axis=0) <= 1e-5 * mag).all()
    assert ew32[0] / lc.SCALE == pytest.approx(U, rel=1e-5)


def test_footprint_counts_and_profiled_phases_c1():
    """Per-cell footprint counts of buffer + reduce are its replica slots (at
    least one per cell, at most max_replicas), and the profiled evaluation
    times every phase and the closing gather."""
    S = c1()
    s = lc.Schedule(S.g, "buffer")
    fp = s.cell_footprints()
    assert fp.shape == (S.g.ncell,) and fp.min() >= 1
    assert fp.max() == s.info()["max_replicas"]
    F, ew, tot, ph = lc.compute_forces_profiled(S.g, s, S.cs, S.coord, S.ws)
    assert len(ph) == s.info()["nphase"] + 1 and tot > 0 and ph[-1] > 0
    assert (S.unsort(F) == O.forces_lc_fx(S.u, S.box.L, S.box.rc, S.g.nc)[0]).all()


def test_momentum_exact_c1():
    S = c1()
    F, _, _ = S.forces("block8")
    assert (F.sum(axis=1) == 0).all()


def test_c2_full_size_all_schedules():
    """256k particles, 26^3 cells: every schedule bit-exact vs the oracle."""
    box = synth.fcc(256000, 0.8, rc=2.5, seed=1002)
    S = Setup(box, even=True)
    _say("fcc256k nc", S.g.nc)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
    for kind in ["block8", "buffer", "atomic_tile", "atomic_pair", "loopex", "lex", "fullshell"]:
        _say("  fcc256k", kind)
        F, ew, st = S.forces(kind)
        assert (F == Fo).all(), kind
        assert ew == [Eo, Wo, npo], kind
        assert st == 0, (kind, st)


def test_c2_fp32_against_fp64_oracle():
    """256k particles: the FP32 pair arithmetic (int64 sums) of the headline
    schedule against the FP64 serial link-cell oracle, normwise <= 1e-5 in
    the forces and <= 1e-5 relative in the energy.  The FP64 oracle takes
    its pair set from the FP64 r^2 < rc^2 test; pairs within an FP32 ulp of
    the cutoff (about one expected here) may differ, which moves the norm
    by ~1e-8."""
    box = synth.fcc(256000, 0.8, rc=2.5, seed=1002)
    S = Setup(box)
    _say("fcc256k fp32 vs fp64 oracle, nc", S.g.nc)
    F, ew, st = S.forces("buffer", block=(2, 2, 3))
    F64, U64, W64, np64 = O.forces_lc_f64(box.pos, S.u, box.L, box.rc, S.g.nc)
    Fx = F / lc.SCALE
    err = np.linalg.norm(Fx - F64) / np.linalg.norm(F64)
    _say("  normwise", err, "pairs", ew[2], np64)
    assert st == 0
    assert err <= 1e-5
    assert abs(ew[2] - np64) <= 10
    assert abs(ew[0] / lc.SCALE - U64) <= 1e-5 * abs(U64)
    assert abs(ew[1] / lc.SCALE - W64) <= 1e-5 * abs(W64)


def test_c2_headline_configurations():
    """256k particles on the natural 27^3 grid with the block shapes the
    autotuner picks there (BUFFER and ATOMIC_TILE up to 1x4x4 and 2x2x3,
    FULLSHELL, BLOCK8 on odd counts), and on the rc/2 grid: bit-exact."""
    box = synth.fcc(256000, 0.8, rc=2.5, seed=1002)
    S = Setup(box)
    assert S.g.nc == (27, 27, 27)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
    for kind, block in (("buffer", (1, 3, 3)), ("buffer", (1, 3, 4)), ("buffer", (1, 4, 4)),
                        ("buffer", (2, 2, 3)), ("atomic_tile", (1, 3, 4)),
                        ("fullshell", (1, 2, 2)), ("block8", (1, 2, 2))):
        _say("  fcc256k 27^3", kind, block)
        F, ew, st = S.forces(kind, block=block)
        assert st == 0 and (F == Fo).all() and ew == [Eo, Wo, npo], (kind, block)
    H = Setup(box, half=True)
    assert H.g.nc == (54, 54, 54)
    for kind, block in (("buffer", (1, 2, 3)), ("atomic_tile", (1, 2, 2))):
        _say("  fcc256k 54^3", kind, block)
        F, ew, st = H.forces(kind, block=block)
        assert st == 0 and (F == Fo).all() and ew == [Eo, Wo, npo], (kind, block)


def test_ragged_and_vacancies():
    """N not a multiple of the lattice or of 64; odd cell counts."""
    for n, rho, seed in ((1234, 0.8, 3), (777, 0.6, 4), (5003, 0.85, 5)):
        box = synth.fcc(n, rho, rc=2.5, seed=seed)
        S = Setup(box)
        _say("ragged", n, rho, S.g.nc)
        Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
        for kind in ("block8", "buffer", "atomic_pair", "opt", "fullshell"):
            F, ew, _ = S.forces(kind)
            assert (F == Fo).all() and ew == [Eo, Wo, npo], (n, kind)


def test_minimum_grid_and_empty_cells():
    """3 cells per axis (the smallest grid) and a dilute box with many empty
    cells."""
    cases = [synth.fcc(108, 0.15, rc=2.5, seed=7),   # L = 8.96: 3^3 cells
             synth.fcc(200, 0.05, rc=2.5, seed=8)]   # dilute: many empty cells
    for box in cases:
        S = Setup(box)
        _say("small", box.n, S.g.nc)
        Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
        for kind in ("block8", "buffer", "atomic_tile", "atomic_pair", "lex", "fullshell"):
            F, ew, _ = S.forces(kind)
            assert (F == Fo).all() and ew == [Eo, Wo, npo], kind


def test_lds_overflow_falls_back_exactly():
    """A cutoff so large that a work-group footprint exceeds the LDS tile:
    the global-memory path takes over and stays bit-exact."""
    box = synth.fcc(4000, 0.8, rc=5.6, seed=9)  # 3^3 cells of 5.7
    S = Setup(box)
    _say("fallback nc", S.g.nc)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
    for kind in ("block8", "buffer", "atomic_tile", "fullshell"):
        F, ew, st = S.forces(kind)
        assert st & lc.FLAG_FALLBACK
        assert (F == Fo).all() and ew == [Eo, Wo, npo], kind


def test_dense_cells_take_the_tiled_path():
    """A skin grid of 4^3 cells holding 62.5 particles each on average (73
    at most): beyond what the 16-bit filter stages, so the unfiltered tiled
    kernel runs (27-cell footprints of at most 1971 particles fit its
    2048-particle tile) and no work-group falls back to global memory."""
    box = synth.fcc(4000, 0.8, rc=2.5, seed=1001)
    S = Setup(box, skin=0.6, even=True)
    assert S.g.nc == (4, 4, 4)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
    for kind in ("block8", "buffer", "atomic_tile", "fullshell"):
        _say("dense", kind)
        F, ew, st = S.forces(kind)
        if kind != "fullshell":  # 48-cell footprints may exceed the tile
            assert st == 0, (kind, st)
        assert st & lc.FLAG_OVERFLOW == 0
        assert (F == Fo).all() and ew == [Eo, Wo, npo], kind


@pytest.mark.parametrize("kind", ["buffer", "atomic_tile", "fullshell"])
def test_block_shapes_bit_exact(kind):
    """Uncoloured kinds over block shapes from single cells to blocks
    larger than half the grid, on a ragged box with odd cell counts."""
    box = synth.fcc(5003, 0.85, rc=2.5, seed=5)
    S = Setup(box)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
    for block in ((1, 1, 1), (1, 2, 3), (2, 2, 2), (1, 4, 4)):
        _say("shape", kind, block, S.g.nc)
        F, ew, st = S.forces(kind, block=block)
        assert st & lc.FLAG_OVERFLOW == 0
        assert (F == Fo).all() and ew == [Eo, Wo, npo], (kind, block)


def test_block8_corner_colourings_bit_exact():
    """BLOCK8 over the shapes corner grouping admits: single cells (each
    colour class a 2 x 2 x 2 stride of cells, the paper's colouring with
    each cell's 14 tasks in one work-group) and 1 x 1 x 2 and 2 x 2 x 2
    blocks, on the 6^3 grid of 4,000 particles and an 8^3 grid."""
    for n, seed in ((4000, 1001), (9000, 7)):
        box = synth.fcc(n, 0.8, rc=2.5, seed=seed)
        S = Setup(box)
        Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
        for block in ((1, 1, 1), (1, 1, 2), (2, 2, 2)):
            _say("block8 corner", n, block, S.g.nc)
            F, ew, st = S.forces("block8", block=block)
            assert st & lc.FLAG_OVERFLOW == 0
            assert (F == Fo).all() and ew == [Eo, Wo, npo], (n, block)


def test_fast_reciprocal_is_ieee_on_its_range():
    """The FP32 sweep takes 1/r^2 for 0.3 <= r^2 < 128 from the hardware
    estimate plus one Newton-Raphson step; it must equal IEEE division for
    every float of [0.25, 128) (75.5M values, checked exhaustively)."""
    lo, hi = lc.RECIP_RANGE
    assert np.float32(np.uint32(lo).view(np.float32)) == 0.25
    assert np.float32(np.uint32(hi).view(np.float32)) == 128.0
    assert lc.selftest_recip(lo, hi) == 0


def test_overflow_flag():
    """Two particles 0.05 apart: the force exceeds the fixed-point range;
    the oracle refuses too."""
    box = synth.fcc(500, 0.8, rc=2.5, seed=10)
    box.pos[:, 1] = box.pos[:, 0] + np.array([0.05, 0.0, 0.0])
    S = Setup(box)
    _, _, st = S.forces("block8")
    assert st & lc.FLAG_OVERFLOW
    with pytest.raises(lc.LCError) as e:  # the flag as a status code
        S.ws.check()
    assert e.value.code == -5
    S.ws.clear_status()
    S.ws.check()
    with pytest.raises(O.OracleError):
        O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)


def _verlet_gpu(box, vel, dt, steps, rebuild, skin, chunks=(None,), check=False, kind="block8"):
    g = lc.Grid(box.L, box.rc, skin)
    ws = lc.Workspace(box.n, g.ncell)
    s = lc.Schedule(g, kind)
    pos = torch.from_numpy(box.pos).to(DEV)
    v = torch.from_numpy(vel).to(DEV)
    ids = torch.arange(box.n, dtype=torch.int32, device=DEV)
    traces = []
    for c in chunks:
        tr, F = lc.verlet_step(g, s, pos, v, ids, ws, dt, c or steps, rebuild)
        traces.append(tr.cpu().numpy())
    torch.cuda.synchronize()
    idh = ids.cpu().numpy()
    P = np.empty((3, box.n))
    V = np.empty((3, box.n))
    P[:, idh] = pos.cpu().numpy()
    V[:, idh] = v.cpu().numpy()
    _verlet_gpu.last_F = np.empty((3, box.n), dtype=np.int64)
    _verlet_gpu.last_F[:, idh] = F.cpu().numpy()
    if check:
        try:
            ws.check()
        except lc.LCError as e:
            return P, V, traces, e.code
        return P, V, traces, 0
    return P, V, traces, ws.status()


_verlet_oracle = {}


@pytest.mark.parametrize("kind", ["block8", "buffer", "atomic_tile"])
def test_verlet_bit_exact_vs_oracle(kind):
    """Config 1 (4,000 particles) with thermal velocities: 100 kick-drift-kick
    steps at dt = 0.005, cells rebuilt every 10 steps (skin 0.6), bit-exact
    positions, velocities and energy trace against the oracle -- under
    BLOCK8, under buffer + reduce (whose replica slots the kick pass sums
    itself, without a gather launch) and under tile atomics."""
    box = synth.fcc(4000, 0.8, rc=2.5, seed=1001)
    vel = synth.maxwell_boltzmann(box.n, 1.0, seed=2001)
    _say("verlet fcc4k 100 steps", kind)
    P, V, (tr,), st = _verlet_gpu(box, vel, 0.005, 100, 10, 0.6, kind=kind)
    if "ref" not in _verlet_oracle:
        _verlet_oracle["ref"] = O.verlet_fx(box.pos, vel, box.L, box.rc, 0.005, 100)
    Po, Vo, Fo, tro = _verlet_oracle["ref"]
    assert st & lc.FLAG_DISP == 0
    assert (P == Po).all() and (V == Vo).all()
    assert (tr == tro).all()
    assert (_verlet_gpu.last_F == Fo).all()  # the forces returned for the last step


@pytest.mark.parametrize("kind", ["block8", "buffer"])
def test_verlet_resume_is_bit_exact(kind):
    """Twice 10 steps give the bits of 20 (and with buffer + reduce the
    returned forces of the last step are the gathered ones)."""
    box = synth.fcc(2048, 0.8, rc=2.5, seed=12)
    vel = synth.maxwell_boltzmann(box.n, 1.0, seed=13)
    P1, V1, _, _ = _verlet_gpu(box, vel, 0.005, 20, 10, 0.6, kind=kind)
    P2, V2, trs, _ = _verlet_gpu(box, vel, 0.005, 20, 10, 0.6, chunks=(10, 10), kind=kind)
    assert (P1 == P2).all() and (V1 == V2).all()


def test_displacement_flag():
    """Cells kept far longer than the skin allows must raise the flag."""
    box = synth.fcc(2048, 0.8, rc=2.5, seed=14)
    vel = synth.maxwell_boltzmann(box.n, 1.0, seed=15)
    _, _, _, st = _verlet_gpu(box, vel, 0.005, 120, 1000, 0.1)
    assert st & lc.FLAG_DISP
    # and as a status code from the check call
    _, _, _, code = _verlet_gpu(box, vel, 0.005, 120, 1000, 0.1, check=True)
    assert code == -6


def _half_shell2():
    r = range(-2, 3)
    return [(x, y, z) for z in r for y in r for x in r
            if x > 0 or (x == 0 and z > 0) or (x == 0 and z == 0 and y < 0)]


def test_half_cells_bit_exact():
    """Cells of side rc/2 (13^3, reach-2 stencil of 62 offsets + intra): every
    schedule kind defined there gives the bits of the oracle's rc-cell sweep
    (the pair set does not depend on the cell size)."""
    box = synth.fcc(4000, 0.8, rc=2.5, seed=41)
    S = Setup(box, half=True)
    assert S.g.nc == (13, 13, 13) and S.g.reach == 2
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, O.grid_dims(box.L, box.rc))
    order = [O.INTRA] + [tuple(-c for c in d) for d in _half_shell2()][::-1]
    cases = [("buffer", None, None), ("buffer", (1, 1, 1), None), ("buffer", (2, 1, 1), None),
             ("atomic_tile", None, None), ("atomic_pair", None, None),
             ("fullshell", None, None), ("lex", None, None), ("custom", None, order)]
    for kind, block, offs in cases:
        _say("half", kind, block)
        F, ew, st = S.forces(kind, block=block, offsets=offs)
        assert st & lc.FLAG_OVERFLOW == 0
        assert (F == Fo).all() and ew == [Eo, Wo, npo], (kind, block)
    for mode in ("ordered", "nested"):
        _say("half dataflow", mode)
        s = lc.Schedule(S.g, "lex")
        S.ws.clear_status()
        F, ew = lc.compute_forces_dataflow(S.g, s, S.cs, S.coord, S.ws, mode)
        torch.cuda.synchronize()
        assert S.ws.status() == 0
        assert (S.unsort(F) == Fo).all() and [int(x) for x in ew.cpu()] == [Eo, Wo, npo], mode


def test_half_cells_loopex_27_colours():
    """Loop exchange at reach 2 colours cells with stride 3 (27 colours): a
    12^3 half-cell grid, level by level, bit-exact; BLOCK8, buffer + reduce
    and tile atomics with 2 x 2 x 2 blocks on the same grid."""
    box = synth.fcc(3000, 0.8, rc=2.5, seed=42)
    S = Setup(box, half=True)
    assert S.g.nc == (12, 12, 12)
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, O.grid_dims(box.L, box.rc))
    F, ew, st = S.forces("loopex")
    assert st & lc.FLAG_OVERFLOW == 0
    assert (F == Fo).all() and ew == [Eo, Wo, npo]
    # 2-cell blocks colour at reach 2 (footprints grow two cells towards +)
    for kind in ("block8", "buffer", "atomic_tile"):
        _say("half 2x2x2", kind)
        F, ew, st = S.forces(kind, block=(2, 2, 2))
        assert st & lc.FLAG_OVERFLOW == 0
        assert (F == Fo).all() and ew == [Eo, Wo, npo], kind


def test_flat_2d_bit_exact():
    """A flat LJ system (square lattice with jitter, all particles at z = 0)
    on a 26 x 26 x 1 grid: the 2D stencil, every schedule kind and the
    paper's 2D orders, bit-exact against the oracle's brute force."""
    box = synth.square2d(3000, 0.7, rc=2.5, seed=43)
    S = Setup(box, flat=True)
    assert S.g.nc == (26, 26, 1)
    Fo, Eo, Wo, npo = O.forces_brute_fx(S.u, box.L, box.rc)
    assert npo > 15000
    cases = [("block8", (4, 4, 1)), ("block8", None), ("buffer", (8, 8, 1)), ("buffer", None),
             ("atomic_tile", (4, 8, 1)), ("atomic_pair", None), ("fullshell", (4, 4, 1)),
             ("lex", None), ("opt", None), ("bad", None), ("loopex", None)]
    for kind, block in cases:
        _say("flat", kind, block)
        F, ew, st = S.forces(kind, block=block)
        assert st & lc.FLAG_OVERFLOW == 0
        assert (F == Fo).all() and ew == [Eo, Wo, npo], (kind, block)


def test_load_aware_group_order():
    """Load-aware schedules (groups launched heaviest first, weights n_A n_B
    from the cell counts) on a slab: the estimated work is non-increasing
    inside every phase, the total is unchanged, and the forces keep the
    oracle's bits."""
    box = synth.slab(60000, seed=44)
    S = Setup(box)
    counts = lc.cell_counts_of(S.cs)
    assert int(counts.sum()) == box.n
    Fo, Eo, Wo, npo = O.forces_lc_fx(S.u, box.L, box.rc, S.g.nc)
    for kind, block in (("buffer", (1, 2, 2)), ("block8", None), ("atomic_tile", (1, 3, 3)),
                        ("fullshell", None)):
        _say("load-aware", kind)
        plain = lc.Schedule(S.g, kind, block=block)
        s = lc.Schedule(S.g, kind, block=block, cell_counts=counts)
        w0, w = plain.group_work(counts), s.group_work(counts)
        assert np.isclose(w0.sum(), w.sum()) and sorted(w0) == sorted(w)
        ph = s.info()["nphase"]
        if ph == 1:
            assert (np.diff(w) <= 0).all(), kind
        S.ws.clear_status()
        F, ew = lc.compute_forces(S.g, s, S.cs, S.coord, S.ws)
        torch.cuda.synchronize()
        assert S.ws.status() & lc.FLAG_OVERFLOW == 0
        assert (S.unsort(F) == Fo).all() and [int(x) for x in ew.cpu()] == [Eo, Wo, npo], kind


def test_weighted_schedule_rejects_negative_counts():
    g = lc.Grid((17.0998,) * 3, 2.5)
    counts = np.ones(g.ncell, dtype=np.int32)
    counts[5] = -1
    with pytest.raises(lc.LCError, match="negative"):
        lc.Schedule(g, "buffer", cell_counts=counts)
