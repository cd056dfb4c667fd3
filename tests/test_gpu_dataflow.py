"""Dataflow executors (Sec. VI strategy 2, the mutual exclusion of Sec. VII)
against the oracle: one persistent launch of task runners that follow the
creation order's dependences (ordered), or keep the cells of concurrent tasks
apart (mutex, nested chains); forces and sums bit-identical to the oracle.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_4441_amd import dataflow_check as D
from paper_1401_4441_amd import lc, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)


class Box:
    def __init__(self, box, even=False):
        self.box = box
        self.g = lc.Grid(box.L, box.rc, 0.0, even)
        self.ws = lc.Workspace(box.n, self.g.ncell)
        self.pos = torch.from_numpy(box.pos).to(DEV)
        self.cs, self.perm, self.coord = lc.build_cells(self.g, self.pos, self.ws)
        self.perm_h = self.perm.cpu().numpy()
        self.u = O.canonical(box.pos, box.L)
        self.ref = O.forces_lc_fx(self.u, box.L, box.rc, self.g.nc)

    def run(self, kind, mode, limit_ms=5000.0, logged=False):
        s = lc.Schedule(self.g, kind)
        A, B = s.tasks()
        log = torch.full((2 * len(A),), -1, dtype=torch.int32, device=DEV) if logged else None
        self.ws.clear_status()
        F, ew = lc.compute_forces_dataflow(self.g, s, self.cs, self.coord, self.ws, mode,
                                           limit_ms=limit_ms, log=log)
        torch.cuda.synchronize()
        st = self.ws.status()
        s.close()
        Fh = F.cpu().numpy()
        out = np.empty_like(Fh)
        out[:, self.perm_h] = Fh
        self.last = (A, B, log.cpu().numpy() if logged else None)
        return out, [int(x) for x in ew.cpu().numpy()], st

    def check(self, kind, mode, logged=True):
        F, ew, st = self.run(kind, mode, logged=logged)
        Fo, Eo, Wo, npo = self.ref
        assert st == 0, (kind, mode, st)
        assert (F == Fo).all(), (kind, mode)
        assert ew == [Eo, Wo, npo], (kind, mode)
        if logged:
            self.check_log(kind, mode)

    def check_log(self, kind, mode):
        """The executor honoured its strategy: every task ran once, and
        ordered kept the creation order's dependences, mutex and nested kept
        tasks sharing a cell apart (nested: each chain in order)."""
        A, B, log = self.last
        T = len(A)
        assert D.check_complete(log, T) == 0, (kind, mode)
        if mode == "ordered":
            assert D.check_ordered(A, B, log) == 0, (kind, mode)
        else:
            assert D.check_exclusive(A, B, log) == 0, (kind, mode)
        if mode == "nested":
            assert D.check_chains(log, T, T // self.g.ncell) == 0, (kind, mode)
        # the mutual-exclusion executors do not keep the creation order:
        # report how often they ran a dependent task before its predecessor
        if mode != "ordered":
            _say("  out-of-order dependent pairs", D.check_ordered(A, B, log))


_c1 = None


def c1():
    global _c1
    if _c1 is None:
        _c1 = Box(synth.fcc(4000, 0.8, rc=2.5, seed=1001))
    return _c1


@pytest.mark.parametrize("mode", ["ordered", "mutex", "nested"])
@pytest.mark.parametrize("kind", ["lex", "opt", "bad"])
def test_dataflow_bit_exact_c1(kind, mode):
    _say("dataflow fcc4k", kind, mode)
    c1().check(kind, mode)


def test_schedule_tasks_are_the_oracle_creation_order():
    S = c1()
    for kind, order in (("lex", O.ORDER3_LEX), ("opt", O.ORDER3_OPT), ("bad", O.ORDER3_BAD)):
        s = lc.Schedule(S.g, kind)
        A, B = s.tasks()
        oa, ob = O.lc_tasks(S.g.nc, order)
        assert (A == oa).all() and (B == ob).all(), kind
        s.close()


@pytest.mark.parametrize("mode", ["ordered", "mutex"])
def test_dataflow_loopex(mode):
    _say("dataflow fcc4k loopex", mode)
    c1().check("loopex", mode)


def test_nested_needs_cell_chains_and_orders_need_a_creation_order():
    S = c1()
    for kind, mode in (("loopex", "nested"), ("buffer", "ordered"), ("block8", "mutex")):
        s = lc.Schedule(S.g, kind)
        with pytest.raises(lc.LCError):
            lc.compute_forces_dataflow(S.g, s, S.cs, S.coord, S.ws, mode)
        s.close()


def test_dataflow_ragged_and_small():
    for box in (synth.fcc(1234, 0.8, rc=2.5, seed=3), synth.fcc(108, 0.15, rc=2.5, seed=7)):
        S = Box(box)
        _say("dataflow ragged/small", box.n, S.g.nc)
        for mode in ("ordered", "mutex", "nested"):
            S.check("opt", mode)


def test_dataflow_full_size_256k():
    """256k particles: the optimal order's dependences, and both mutual
    exclusion executors, bit-exact at full size."""
    S = Box(synth.fcc(256000, 0.8, rc=2.5, seed=1002), even=True)
    for mode in ("ordered", "mutex", "nested"):
        _say("dataflow fcc256k opt", mode)
        S.check("opt", mode)


def test_expired_wait_abandons_the_evaluation():
    """A zero time limit: the first runner whose cells are not ready gives
    up, every runner stops, the call returns with FLAG_ABORT set (and the
    kernel has exited: the next evaluation on the workspace is exact)."""
    S = c1()
    _say("dataflow forced abort")
    _, _, st = S.run("lex", "ordered", limit_ms=0.0)
    assert st & lc.FLAG_ABORT
    with pytest.raises(lc.LCError) as e:  # the flag as a status code
        S.ws.check()
    assert e.value.code == -8
    S.check("lex", "ordered")
    S.ws.check()
