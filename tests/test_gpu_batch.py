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
    """Dilute boxes whose cells total more than 65,536, so the batched cell
    build takes the three-pass scan: cell tables and forces bit-exact per box,
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
