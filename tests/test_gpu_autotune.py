"""The autotuner on small boxes: every configuration it picks is valid and
gives the oracle's forces bit for bit; its cache returns the stored pick."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import autotune, lc, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)


def _forces(g, kind, block, pos, n):
    ws = lc.Workspace(n, g.ncell)
    cs, perm, coord = lc.build_cells(g, pos, ws)
    s = lc.Schedule(g, kind, block=block)
    F, ew = lc.compute_forces(g, s, cs, coord, ws)
    torch.cuda.synchronize()
    Fh = F.cpu().numpy()
    out = np.empty_like(Fh)
    out[:, perm.cpu().numpy()] = Fh
    st = ws.status()
    s.close()
    ws.close()
    return out, [int(x) for x in ew.cpu().numpy()], st


def test_tune_box_pick_is_valid_and_exact(tmp_path, monkeypatch):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    box = synth.fcc(5003, 0.85, rc=2.5, seed=5)
    pos = torch.from_numpy(box.pos).to(DEV)
    _say("tune_box 5003")
    t = autotune.tune_box(pos, box.L, box.rc, reps=2,
                          kinds=("block8", "buffer", "atomic_tile", "fullshell"))
    assert t["trials"] and not t["fallback"]
    assert t["ms"] == min(x["ms"] for x in t["trials"] if not x["fallback"])
    assert {x["kind"] for x in t["trials"]} == {"block8", "buffer", "atomic_tile", "fullshell"}
    # the cells of side rc/2 are among the grids tried (no block colouring there)
    half = [x for x in t["trials"] if x["grid"].get("half")]
    assert half and {x["kind"] for x in half} == {"buffer", "atomic_tile", "fullshell"}
    u = O.canonical(box.pos, box.L)
    Fo, Eo, Wo, npo = O.forces_lc_fx(u, box.L, box.rc, O.grid_dims(box.L, box.rc))
    best_half = min(half, key=lambda x: x["ms"])
    for rec in [t, best_half] + sorted(t["trials"], key=lambda x: x["ms"])[:3]:
        g = autotune.make_grid(box.L, box.rc, rec["grid"])  # fallbacks are exact too
        F, ew, st = _forces(g, rec["kind"], tuple(rec["block"]), pos, box.n)
        assert st & lc.FLAG_OVERFLOW == 0 and (F == Fo).all() and ew == [Eo, Wo, npo], rec
        assert bool(st & lc.FLAG_FALLBACK) == rec["fallback"], rec
    # the cache returns the stored pick without timing again
    t2 = autotune.tune_box(pos, box.L, box.rc, reps=2,
                           kinds=("block8", "buffer", "atomic_tile", "fullshell"))
    assert (t2["kind"], t2["block"], t2["grid"]) == (t["kind"], t["block"], t["grid"])
    assert os.path.exists(tmp_path / "tune.json")


def test_tune_shape_on_a_skin_grid():
    box = synth.fcc(4000, 0.8, rc=2.5, seed=1001)
    pos = torch.from_numpy(box.pos).to(DEV)
    g = lc.Grid(box.L, box.rc, 0.6, True)
    _say("tune_shape skin grid", g.nc)
    t = autotune.tune_shape(g, pos, reps=2)
    assert t["kind"] in autotune.BOX_KINDS_CONFLICT_FREE
    assert not t["fallback"]
    assert t["ms"] == min(x["ms"] for x in t["trials"] if not x["fallback"])
    u = O.canonical(box.pos, box.L)
    Fo, Eo, Wo, npo = O.forces_lc_fx(u, box.L, box.rc, g.nc)
    F, ew, st = _forces(g, t["kind"], tuple(t["block"]), pos, box.n)
    assert st == 0 and (F == Fo).all() and ew == [Eo, Wo, npo]


def test_tune_shape_on_half_cells():
    box = synth.fcc(4000, 0.8, rc=2.5, seed=1002)
    pos = torch.from_numpy(box.pos).to(DEV)
    g = lc.Grid(box.L, box.rc, half=True)
    _say("tune_shape half cells", g.nc)
    t = autotune.tune_shape(g, pos, kinds=("buffer", "atomic_tile"), reps=2)
    assert t["kind"] in ("buffer", "atomic_tile") and not t["fallback"]
    assert {tuple(x["block"]) for x in t["trials"]} <= set(autotune.BLOCKS["uncoloured_half"])
    u = O.canonical(box.pos, box.L)
    Fo, Eo, Wo, npo = O.forces_lc_fx(u, box.L, box.rc, O.grid_dims(box.L, box.rc))
    F, ew, st = _forces(g, t["kind"], tuple(t["block"]), pos, box.n)
    assert st == 0 and (F == Fo).all() and ew == [Eo, Wo, npo]
