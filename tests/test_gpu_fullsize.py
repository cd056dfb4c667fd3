"""GPU checks at the full sizes of the evaluated configurations, on sampled
particles the oracle computes one by one (brute force over all partners),
plus properties that hold at any size (exact momentum conservation, no
flags).  Sizes: the 4,000,000-particle crystal on its rebuild grid (cells
of rc + skin, 54^3) and on plain rc cells (68^3); the 2,000,000-particle
inhomogeneous slab (rc = 3.0, 64^3 cells, plain and load-aware launch
order; 131^3 cells of side rc/2)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import synth

pytestmark = pytest.mark.gpu

lc = pytest.importorskip("paper_1401_4441_amd.lc")
DEV = torch.device("cuda:0")

_cache = {}


def _box(name):
    if name not in _cache:
        _cache[name] = synth.workload(name)
    return _cache[name]


def _check(box, skin, even, kinds, idx, half=False, weighted=False):
    g = lc.Grid(box.L, box.rc, skin, even, half=half)
    print("grid", g.nc, "n", box.n, flush=True)
    ws = lc.Workspace(box.n, g.ncell)
    pos = torch.from_numpy(box.pos).to(DEV)
    cs, perm, coord = lc.build_cells(g, pos, ws)
    perm_h = perm.cpu().numpy()
    inv = np.empty_like(perm_h)
    inv[perm_h] = np.arange(box.n, dtype=perm_h.dtype)
    u = O.canonical(box.pos, box.L)
    Fo, nn = O.forces_subset_fx(u, box.L, box.rc, idx)
    results = []
    counts = lc.cell_counts_of(cs) if weighted else None
    for kind in kinds:
        print("  kind", kind, flush=True)
        s = lc.Schedule(g, kind, cell_counts=counts)
        ws.clear_status()
        F, ew = lc.compute_forces(g, s, cs, coord, ws)
        torch.cuda.synchronize()
        st = ws.status()
        Fs = F[:, torch.from_numpy(inv[idx].astype(np.int64)).to(DEV)].cpu().numpy()
        assert (Fs == Fo).all(), kind
        assert (F.sum(dim=1) == 0).all(), kind
        assert st & lc.FLAG_OVERFLOW == 0, (kind, st)
        # in input order: separate builds may order particles inside a cell
        # differently (atomic ranks)
        results.append((F[:, torch.from_numpy(inv.astype(np.int64)).to(DEV)].clone(), ew.clone(),
                        st))
    for F, ew, _ in results[1:]:
        assert torch.equal(F, results[0][0]) and torch.equal(ew, results[0][1])
    return results


def test_fcc4m_rebuild_grid():
    box = _box("fcc4m")
    idx = np.random.default_rng(1).choice(box.n, 24, replace=False)
    res = _check(box, 0.6, True, ["buffer", "block8"], idx)
    assert all(st == 0 for _, _, st in res)


def test_fcc4m_rc_grid():
    box = _box("fcc4m")
    idx = np.random.default_rng(2).choice(box.n, 24, replace=False)
    _check(box, 0.0, True, ["buffer", "atomic_tile"], idx)


def test_slab2m():
    box = _box("slab2m")
    z = box.pos[2]
    L = box.L[2]
    dense = np.flatnonzero((z >= L / 3) & (z < 2 * L / 3))
    gas = np.flatnonzero((z < L / 3) | (z >= 2 * L / 3))
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(dense, 16, replace=False),
                          rng.choice(gas, 16, replace=False)])
    res = _check(box, 0.0, True, ["buffer", "block8"], idx)
    assert all(st & lc.FLAG_FALLBACK == 0 for _, _, st in res)
    # the load-aware launch order, and cells of side rc/2 (131^3)
    res2 = _check(box, 0.0, True, ["buffer", "block8"], idx, weighted=True)
    assert torch.equal(res2[0][0], res[0][0]) and torch.equal(res2[0][1], res[0][1])
    _check(box, 0.0, False, ["atomic_tile"], idx, half=True)
