"""GPU check of lc_compute_forces_noalloc (the force evaluation whose scratch
is a static device array, for callers that cannot allocate): bit-identical
to lc_compute_forces on two calls in a row, the second on a smaller system,
for buffer + reduce (replica buffer in the static scratch) and the coloured
blocks; oversized replica buffers are refused before anything runs."""
import numpy as np
import pytest
import torch

from paper_1401_4441_amd import synth

pytestmark = pytest.mark.gpu

lc = pytest.importorskip("paper_1401_4441_amd.lc")
DEV = torch.device("cuda:0")


def _system(n, seed):
    box = synth.fcc(n, 0.8, rc=2.5, seed=seed)
    g = lc.Grid(box.L, box.rc, 0.0, True)
    ws = lc.Workspace(box.n, g.ncell)
    cs, perm, coord = lc.build_cells(g, torch.from_numpy(box.pos).to(DEV), ws)
    return g, ws, cs, coord


@pytest.mark.parametrize("kind,prec", [("buffer", "fp32"), ("block8", "fp32"),
                                       ("atomic_tile", "fp32"), ("buffer", "fp64")])
def test_noalloc_matches_workspace_path(kind, prec):
    # the larger system first, then a smaller one: the second call reuses the
    # scratch the first left behind
    for n, seed in ((32000, 71), (4000, 72)):
        print(f"noalloc {kind} {prec} n={n} seed={seed}", flush=True)
        g, ws, cs, coord = _system(n, seed)
        s = lc.Schedule(g, kind)
        F0, ew0 = lc.compute_forces(g, s, cs, coord, ws, prec)
        F1 = torch.full((3, coord.shape[1]), 7, dtype=torch.int64, device=DEV)
        ew1 = torch.full((3,), 7, dtype=torch.int64, device=DEV)
        flags = torch.zeros(1, dtype=torch.int32, device=DEV)
        lc.compute_forces_noalloc(g, s, cs, coord, F1, ew1, prec, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(F0, F1), (kind, n)
        assert torch.equal(ew0, ew1), (kind, n, ew0.tolist(), ew1.tolist())
        assert int(flags.item()) & lc.FLAG_OVERFLOW == 0
        # again without a flags word (status bits go to the scratch)
        F1.fill_(-1)
        lc.compute_forces_noalloc(g, s, cs, coord, F1, ew1, prec)
        torch.cuda.synchronize()
        assert torch.equal(F0, F1) and torch.equal(ew0, ew1), (kind, n)


def test_noalloc_refuses_oversized_replica_buffer():
    # a 3M-particle replica buffer does not fit the static scratch; the call
    # must fail on the host before enqueuing anything (the cells are empty
    # and the buffers are never read)
    print("noalloc capacity refusal", flush=True)
    g, ws, cs, coord = _system(4000, 73)
    s = lc.Schedule(g, "buffer")
    n = 3_000_000
    csz = torch.zeros(g.ncell + 1, dtype=torch.int32, device=DEV)
    cz = torch.zeros((3, n), dtype=torch.int32, device=DEV)
    F = torch.zeros((3, n), dtype=torch.int64, device=DEV)
    ew = torch.zeros(3, dtype=torch.int64, device=DEV)
    with pytest.raises(lc.LCError) as e:
        lc.compute_forces_noalloc(g, s, csz, cz, F, ew)
    assert e.value.code == -7
    torch.cuda.synchronize()
    assert int(F.abs().sum().item()) == 0
