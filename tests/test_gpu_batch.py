"""GPU parity of the batched path: many independent boxes of uneven size and
density in one launch, bit-exact per box against the oracle; persistent and
one-group-per-work-group launches, whole-box and block splits, and HIP graph
replays all give the same bits."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import synth

pytestmark = pytest.mark.gpu

lc = pytest.importorskip("paper_1401_4441_amd.lc")
DEV = torch.device("cuda:0")


def _batch_inputs(count, n_lo, n_hi, seed):
    boxes = synth.boxes(count, n_lo, n_hi, 0.5, 0.9, rc=2.5, seed=seed)
    grids = [lc.Grid(b.L, b.rc) for b in boxes]
    pos = np.concatenate([b.pos for b in boxes], axis=1)
    return boxes, grids, np.ascontiguousarray(pos)


def _oracle(boxes, grids):
    out = []
    for b, g in zip(boxes, grids):
        u = O.canonical(b.pos, b.L)
        out.append(O.forces_lc_fx(u, b.L, b.rc, g.nc))
    return out


def _check(batch, boxes, grids, cs, perm, coord, ws, want, persistent):
    F, ew = batch.forces(cs, coord, ws, persistent=persistent)
    torch.cuda.synchronize()
    Fh = F.cpu().numpy()
    ph = perm.cpu().numpy()
    Fu = np.empty_like(Fh)
    Fu[:, ph] = Fh  # back to input order
    ps, _ = batch.offsets()
    ewh = ew.cpu().numpy()
    for k, (Fo, Eo, Wo, npo) in enumerate(want):
        assert (Fu[:, ps[k]:ps[k + 1]] == Fo).all(), k
        assert [int(x) for x in ewh[k]] == [Eo, Wo, npo], k
    return F.clone(), ew.clone()


def test_batch_bit_exact_modes():
    boxes, grids, pos = _batch_inputs(12, 500, 4000, seed=5)
    print("batch sizes", [b.n for b in boxes], flush=True)
    want = _oracle(boxes, grids)
    posd = torch.from_numpy(pos).to(DEV)
    results = []
    for modes in (None, ["blocks"] * len(boxes)):
        batch = lc.Batch(grids, [b.n for b in boxes], modes)
        info = batch.info()
        print("batch info", modes is None, info, flush=True)
        ws = lc.Workspace(info["ntot"], info["ncell"])
        cs, perm, coord = batch.build_cells(posd, ws)
        for persistent in (True, False):
            results.append(_check(batch, boxes, grids, cs, perm, coord, ws, want, persistent))
        assert ws.status() & lc.FLAG_OVERFLOW == 0
    assert any(lc.Batch(grids, [b.n for b in boxes]).info()["nwhole"] > 0 for _ in [0])


def test_batch_build_cells_matches_oracle():
    boxes, grids, pos = _batch_inputs(6, 500, 3000, seed=7)
    batch = lc.Batch(grids, [b.n for b in boxes])
    info = batch.info()
    ws = lc.Workspace(info["ntot"], info["ncell"])
    cs, perm, coord = batch.build_cells(torch.from_numpy(pos).to(DEV), ws)
    csh = cs.cpu().numpy()
    ps, cst = batch.offsets()
    for k, (b, g) in enumerate(zip(boxes, grids)):
        u = O.canonical(b.pos, b.L)
        loc = csh[cst[k]:cst[k + 1] + 1] - ps[k]
        assert (loc == O.cell_start(u, g.nc)).all(), k


def test_batch_many_cells_three_pass_scan():
    """Dilute boxes whose cells total more than 65,536 (many scan tiles
    looking back over each other): cell tables and forces bit-exact per box,
    twice on one workspace (the counters are left cleared between builds)."""
    boxes = synth.boxes(30, 1500, 3000, 0.04, 0.08, rc=2.5, seed=13)
    grids = [lc.Grid(b.L, b.rc) for b in boxes]
    pos = np.ascontiguousarray(np.concatenate([b.pos for b in boxes], axis=1))
    batch = lc.Batch(grids, [b.n for b in boxes])
    info = batch.info()
    print("batch cells", info["ncell"], flush=True)
    assert info["ncell"] > 65536
    want = _oracle(boxes, grids)
    ws = lc.Workspace(info["ntot"], info["ncell"])
    posd = torch.from_numpy(pos).to(DEV)
    ps, cst = batch.offsets()
    for _ in range(2):
        cs, perm, coord = batch.build_cells(posd, ws)
        csh = cs.cpu().numpy()
        for k, (b, g) in enumerate(zip(boxes, grids)):
            loc = csh[cst[k]:cst[k + 1] + 1] - ps[k]
            assert (loc == O.cell_start(O.canonical(b.pos, b.L), g.nc)).all(), k
        _check(batch, boxes, grids, cs, perm, coord, ws, want, persistent=False)


def test_batch_graph_replays_bit_identical():
    boxes, grids, pos = _batch_inputs(8, 500, 3000, seed=9)
    want = _oracle(boxes, grids)
    batch = lc.Batch(grids, [b.n for b in boxes])
    info = batch.info()
    ws = lc.Workspace(info["ntot"], info["ncell"])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        cs, perm, coord = batch.build_cells(torch.from_numpy(pos).to(DEV), ws, stream=side)
        F = torch.empty((3, info["ntot"]), dtype=torch.int64, device=DEV)
        ew = torch.empty((len(boxes), 3), dtype=torch.int64, device=DEV)
        batch.forces(cs, coord, ws, F, ew, stream=side)  # eager reference
    side.synchronize()
    F0, ew0 = F.clone(), ew.clone()
    gr = batch.graph(cs, coord, F, ew, ws, side)
    for rep in range(3):
        F.zero_()
        ew.zero_()
        torch.cuda.synchronize()
        gr.launch(side)
        side.synchronize()
        assert torch.equal(F, F0) and torch.equal(ew, ew0), rep
    ph = perm.cpu().numpy()
    Fu = np.empty((3, info["ntot"]), dtype=np.int64)
    Fu[:, ph] = F.cpu().numpy()
    ps, _ = batch.offsets()
    for k, (Fo, Eo, Wo, npo) in enumerate(want):
        assert (Fu[:, ps[k]:ps[k + 1]] == Fo).all(), k
    gr.close()


def test_batch_512_boxes_full_size():
    """The evaluated batch itself: 512 boxes, N ~ U{500..20000}, density ~
    U[0.5, 0.9] (the seeded set the benchmark times), in one persistent
    launch, a one-group-per-work-group launch and a graph replay.  Every box:
    exact momentum conservation, and sampled particles bit-exact against the
    oracle's brute-force fixed-point sum over all partners; the four largest
    and the four densest boxes: every particle, energy, virial and pair count
    bit-exact against the oracle's link-cell sweep."""
    boxes = synth.boxes(512, 500, 20000, 0.5, 0.9, rc=2.5, seed=777)
    grids = [lc.Grid(b.L, b.rc) for b in boxes]
    ns = [b.n for b in boxes]
    pos = np.ascontiguousarray(np.concatenate([b.pos for b in boxes], axis=1))
    batch = lc.Batch(grids, ns)
    info = batch.info()
    print("batch512 info", info, flush=True)
    ws = lc.Workspace(info["ntot"], info["ncell"])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        cs, perm, coord = batch.build_cells(torch.from_numpy(pos).to(DEV), ws, stream=side)
        F = torch.empty((3, info["ntot"]), dtype=torch.int64, device=DEV)
        ew = torch.empty((len(boxes), 3), dtype=torch.int64, device=DEV)
        batch.forces(cs, coord, ws, F, ew, persistent=True, stream=side)
    side.synchronize()
    F0, ew0 = F.clone(), ew.clone()
    with torch.cuda.stream(side):
        batch.forces(cs, coord, ws, F, ew, persistent=False, stream=side)
    side.synchronize()
    assert torch.equal(F, F0) and torch.equal(ew, ew0)
    gr = batch.graph(cs, coord, F, ew, ws, side, True)
    for rep in range(2):
        F.zero_()
        ew.zero_()
        torch.cuda.synchronize()
        gr.launch(side)
        side.synchronize()
        assert torch.equal(F, F0) and torch.equal(ew, ew0), rep
    gr.close()
    assert ws.status() & lc.FLAG_OVERFLOW == 0
    ph = perm.cpu().numpy()
    Fu = np.empty((3, info["ntot"]), dtype=np.int64)
    Fu[:, ph] = F0.cpu().numpy()
    ewh = ew0.cpu().numpy()
    ps, _ = batch.offsets()
    rng = np.random.default_rng(17)
    for k, b in enumerate(boxes):
        Fb = Fu[:, ps[k]:ps[k + 1]]
        assert (Fb.sum(axis=1) == 0).all(), k
        idx = rng.choice(b.n, 3, replace=False)
        Fo, _ = O.forces_subset_fx(O.canonical(b.pos, b.L), b.L, b.rc, idx)
        assert (Fb[:, idx] == Fo).all(), k
    big = sorted(range(len(boxes)), key=lambda k: -boxes[k].n)[:4]
    dense = sorted(range(len(boxes)), key=lambda k: -boxes[k].n / np.prod(boxes[k].L))[:4]
    for k in big + dense:
        b = boxes[k]
        print("batch512 full box", k, b.n, grids[k].nc, flush=True)
        Fo, Eo, Wo, npo = O.forces_lc_fx(O.canonical(b.pos, b.L), b.L, b.rc, grids[k].nc)
        assert (Fu[:, ps[k]:ps[k + 1]] == Fo).all(), k
        assert [int(x) for x in ewh[k]] == [Eo, Wo, npo], k


def test_batch_atomic_write_and_tiles_same_bits():
    """The batch with tile-atomic write-back, and with blocks sized for the
    larger LDS tiles, gives the buffer + reduce batch's bits."""
    boxes, grids, pos = _batch_inputs(10, 500, 6000, seed=21)
    want = _oracle(boxes, grids)
    posd = torch.from_numpy(pos).to(DEV)
    for tile, write in ((512, "buffer"), (768, "atomic"), (1024, "buffer"), (2048, "buffer"),
                        (2048, "atomic")):
        print("batch tile", tile, write, flush=True)
        batch = lc.Batch(grids, [b.n for b in boxes], tile=tile, write=write)
        info = batch.info()
        ws = lc.Workspace(info["ntot"], info["ncell"])
        cs, perm, coord = batch.build_cells(posd, ws)
        for persistent in (True, False):
            _check(batch, boxes, grids, cs, perm, coord, ws, want, persistent)
        assert ws.status() & lc.FLAG_OVERFLOW == 0


def test_graph_pins_the_replica_buffer():
    """While a graph captured with a workspace lives, a call that would grow
    the workspace's replica buffer is refused (the graph holds its address);
    after the graph is freed the call goes through.  No replay needed."""
    boxes, grids, pos = _batch_inputs(4, 500, 1500, seed=23)
    batch = lc.Batch(grids, [b.n for b in boxes])
    info = batch.info()
    big = synth.fcc(32000, 0.8, rc=2.5, seed=24)
    gbig = lc.Grid(big.L, big.rc)
    ws = lc.Workspace(max(info["ntot"], big.n), max(info["ncell"], gbig.ncell))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        cs, perm, coord = batch.build_cells(torch.from_numpy(pos).to(DEV), ws, stream=side)
        F = torch.empty((3, info["ntot"]), dtype=torch.int64, device=DEV)
        ew = torch.empty((len(boxes), 3), dtype=torch.int64, device=DEV)
    side.synchronize()
    gr = batch.graph(cs, coord, F, ew, ws, side)
    cb, _, cob = lc.build_cells(gbig, torch.from_numpy(big.pos).to(DEV), ws)
    s = lc.Schedule(gbig, "buffer")
    with pytest.raises(lc.LCError) as e:
        lc.compute_forces(gbig, s, cb, cob, ws)
    assert e.value.code == -7
    with pytest.raises(lc.LCError):  # the binding keeps the workspace too
        ws.close()
    gr.close()
    lc.compute_forces(gbig, s, cb, cob, ws)
    torch.cuda.synchronize()
