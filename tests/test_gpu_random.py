"""Seeded randomized parity: random boxes (particle count, density, cutoff),
grid variants (cells of side rc, even counts, a Verlet skin, side rc/2, a
flat 2D system), schedule kinds, block shapes and the dataflow executor's
modes, every combination
bit-exact against the oracle's fixed-point brute force (which depends on no
cell decomposition).  Every other case shuffles its particles first, so the
cell build also sees waves of particles from many different cells.  The cases are drawn from a fixed seed, so a failure
names a reproducible configuration."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import synth

pytestmark = pytest.mark.gpu
lc = pytest.importorskip("paper_1401_4441_amd.lc")
DEV = torch.device("cuda:0")

KINDS_3D = ("block8", "buffer", "atomic_tile", "atomic_pair", "fullshell", "lex", "opt", "loopex")
KINDS_HALF = ("buffer", "atomic_tile", "atomic_pair", "fullshell", "lex", "loopex")


def _cases(count=40, seed=20261202):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        variant = ("natural", "even", "skin", "half", "flat")[k % 5]
        rc = float(rng.uniform(1.6, 3.2))
        rho = float(rng.uniform(0.35, 0.95))
        n = int(rng.integers(150, 6000))
        kinds = KINDS_HALF if variant == "half" else KINDS_3D
        kind = kinds[int(rng.integers(len(kinds)))]
        block = None
        if kind in ("buffer", "atomic_tile", "fullshell") and rng.random() < 0.7:
            if variant == "flat":
                block = (int(rng.integers(1, 7)), int(rng.integers(1, 9)), 1)
            elif variant == "half":
                block = (1, int(rng.integers(1, 3)), int(rng.integers(1, 3)))
            else:
                block = (int(rng.integers(1, 3)), int(rng.integers(1, 4)), int(rng.integers(1, 4)))
        if kind == "block8" and rng.random() < 0.5:
            block = (1, 2, 2) if variant != "flat" else (2, 4, 1)
        even = variant == "even" or kind == "loopex"  # loop exchange colours even counts
        flow = None
        if kind in ("lex", "opt") and rng.random() < 0.75:
            flow = ("ordered", "mutex", "nested")[int(rng.integers(3))]
        out.append((k, variant, even, n, rho, rc, kind, block, flow, int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-{c[1]}-{c[6]}")
def test_random_configuration_bit_exact(case):
    k, variant, even, n, rho, rc, kind, block, flow, seed = case
    print("case", case, flush=True)
    if variant == "flat":
        box = synth.square2d(n, rho, rc=rc, seed=seed)
    else:
        box = synth.fcc(n, rho, rc=rc, seed=seed)
    if k % 2:
        # a random particle order: a wave of the cell build then meets up to
        # 64 different cells (the lattice order gives it a few)
        box.pos = np.ascontiguousarray(box.pos[:, np.random.default_rng(seed).permutation(box.n)])
    skin = 0.4 if variant == "skin" else 0.0
    try:
        g = lc.Grid(box.L, box.rc, skin, even, half=variant == "half",
                    flat=variant == "flat")
    except lc.LCError:
        pytest.skip("box too small for this grid variant")
    try:
        s = lc.Schedule(g, kind, block=block)
    except lc.LCError as e:  # e.g. loop exchange on odd counts, block limits
        pytest.skip(f"schedule not defined here: {e}")
    ws = lc.Workspace(box.n, g.ncell)
    pos = torch.from_numpy(box.pos).to(DEV)
    cs, perm, coord = lc.build_cells(g, pos, ws)
    ws.clear_status()
    if flow is None:
        F, ew = lc.compute_forces(g, s, cs, coord, ws)
    else:
        F, ew = lc.compute_forces_dataflow(g, s, cs, coord, ws, flow)
    torch.cuda.synchronize()
    st = ws.status()
    Fh = F.cpu().numpy()
    Fu = np.empty_like(Fh)
    Fu[:, perm.cpu().numpy()] = Fh
    u = O.canonical(box.pos, box.L)
    Fo, Eo, Wo, npo = O.forces_brute_fx(u, box.L, box.rc)
    assert st == 0, case
    assert (Fu == Fo).all(), case
    assert [int(x) for x in ew.cpu()] == [Eo, Wo, npo], case
