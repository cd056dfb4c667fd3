"""GPU: one force evaluation captured into a HIP graph (lc_forces_graph_create)
replays bit-identically to lc_compute_forces and to the oracle.

Every replay is checked, with eager evaluations on another stream and host
synchronisations between the replays, and the output buffers overwritten
before each replay, so that a replay that skipped work or reused stale
values would show.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import synth

pytestmark = pytest.mark.gpu

lc = pytest.importorskip("paper_1401_4441_amd.lc")

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("n,seed", [(4000, 1001), (32000, 61)])
def test_forces_graph_replays_bit_exact(n, seed):
    box = synth.fcc(n, 0.8, rc=2.5, seed=seed)
    g = lc.Grid(box.L, box.rc)
    ws = lc.Workspace(box.n, g.ncell)
    cs, perm, coord = lc.build_cells(g, torch.from_numpy(box.pos).to(DEV), ws)
    torch.cuda.synchronize()
    perm_h = perm.cpu().numpy()
    Fo, Eo, Wo, npo = O.forces_lc_fx(O.canonical(box.pos, box.L), box.L, box.rc, g.nc)
    cc = lc.cell_counts_of(cs)
    side = torch.cuda.Stream()
    for kind, block, weighted in (("buffer", (2, 2, 3), True), ("block8", (1, 2, 2), False),
                                  ("atomic_tile", (1, 2, 2), True), ("fullshell", None, False),
                                  ("lex", None, False)):
        print("graph", n, kind, block, weighted, flush=True)
        s = lc.Schedule(g, kind, block=block, cell_counts=cc if weighted else None)
        Fe, ewe = lc.compute_forces(g, s, cs, coord, ws)
        torch.cuda.synchronize()
        Fg = torch.empty((3, box.n), dtype=torch.int64, device=DEV)
        ewg = torch.empty(3, dtype=torch.int64, device=DEV)
        with torch.cuda.stream(side):
            gr = lc.forces_graph(g, s, cs, coord, ws, Fg, ewg, side)
        for rep in range(3):
            Fg.fill_(-1)
            ewg.fill_(-1)
            torch.cuda.synchronize()
            gr.launch(side)
            side.synchronize()
            assert torch.equal(Fg, Fe) and torch.equal(ewg, ewe), (kind, rep)
            lc.compute_forces(g, s, cs, coord, ws)  # eager work between replays
            torch.cuda.synchronize()
        Fu = np.empty((3, box.n), dtype=np.int64)
        Fu[:, perm_h] = Fg.cpu().numpy()
        assert (Fu == Fo).all() and [int(x) for x in ewg.cpu()] == [Eo, Wo, npo], kind
        with pytest.raises(lc.LCError):  # the graph holds the schedule
            s.close()
        gr.close()
        s.close()
        assert ws.status() == 0
