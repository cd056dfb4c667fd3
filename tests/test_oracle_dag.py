"""Pins for the oracle's task-DAG analysis (CPU only).

The oracle computes critical paths by the StarSs definition (every earlier
task sharing a written parameter is a predecessor).  These tests tie it to
what the paper prints (Fig. 2, Fig. 4, Fig. 5, the Delta ranges of Sec. V,
Eq. 2-4) and to an independent simulation, so that a plausible mistake (a
wrong task order, an ignored read-only parameter, a dropped wrap) fails.
"""
import itertools
import json
import os

import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_dag_values.json")))

MODES = {"in": O.IN, "out": O.OUT, "inout": O.INOUT}


def test_fig2_example_program():
    """Sec. III: the six-task example has three levels, CP 3, S = 2."""
    g = GOLD["fig2_example"]
    tasks = [[(ord(a), MODES[m]) for a, m in t["params"]] for t in g["tasks"]]
    depth, pred, cp = O.dag_generic(tasks)
    assert list(depth) == g["levels"]
    assert cp == g["critical_path"]
    assert len(tasks) / cp == 2.0
    # treating read-only parameters as written would chain tasks 4 and 5
    # through b and lengthen the path: the IN rule matters
    tasks_rw = [[(a, O.INOUT) for a, _ in t] for t in tasks]
    assert O.dag_generic(tasks_rw)[2] == 4


def test_fig4_naive_depths():
    """Fig. 4: chain 1-4, then tasks 5 and 6 both at depth 5 (off task 4)."""
    g = GOLD["fig4_naive_5x5"]
    A, B = O.lc_tasks((5, 5, 1), O.ORDER2_NAIVE)
    depth, _ = O.dag_lc(A, B)
    want = g["first_task_depths"]
    assert list(depth[:len(want)]) == want


@pytest.mark.parametrize("order", [O.ORDER2_NAIVE, O.ORDER2_BAD, O.ORDER2_OPT])
@pytest.mark.parametrize("dims", [(5, 5, 1), (6, 3, 1), (4, 4, 1), (3, 3, 3)])
def test_cp_matches_simulation(order, dims):
    """Longest path by definition == unbounded-worker simulation."""
    if dims[2] > 1:
        order = {id(O.ORDER2_NAIVE): O.ORDER3_LEX, id(O.ORDER2_BAD): O.ORDER3_BAD,
                 id(O.ORDER2_OPT): O.ORDER3_OPT}[id(order)]
    A, B = O.lc_tasks(dims, order)
    _, cp = O.dag_lc(A, B)
    assert cp == O.asap_steps(A, B)


def test_cp_matches_simulation_loopex():
    A, B = O.lc_tasks((6, 4, 1), O.ORDER2_NAIVE, loopex=True)
    assert O.dag_lc(A, B)[1] == O.asap_steps(A, B)


def test_generic_and_lc_dag_agree():
    """The generic address-based builder and the link-cell one agree."""
    A, B = O.lc_tasks((5, 4, 1), O.ORDER2_OPT)
    tasks = [[(int(a), O.INOUT)] + ([(int(b), O.INOUT)] if b != a else [])
             for a, b in zip(A, B)]
    d1, _, cp1 = O.dag_generic(tasks)
    d2, cp2 = O.dag_lc(A, B)
    assert cp1 == cp2 and (d1 == d2).all()


def _delta(order, dims_of, m=120):
    """Asymptotic growth of the critical path per stencil execution."""
    c1 = O.serialization_degree(dims_of(m), order)["cp"]
    c2 = O.serialization_degree(dims_of(2 * m), order)["cp"]
    d = dims_of(m)
    return (c2 - c1) / (m * d[1] * d[2])


def test_fig5_speedup_limits():
    """Fig. 5 / Eq. 3: S_max = 1.25 (naive), 1 (bad), 5 (optimal); the exact
    speedup on long domains approaches them."""
    g = GOLD["fig5_smax"]
    dims = lambda m: (m, 3, 1)
    for name, order in (("naive", O.ORDER2_NAIVE), ("bad", O.ORDER2_BAD),
                        ("opt", O.ORDER2_OPT)):
        delta = _delta(order, dims)
        assert O.smax_eq3(delta, 5) == pytest.approx(g[name])
        s = O.serialization_degree((2000, 3, 1), order)["S"]
        assert s == pytest.approx(g[name], rel=2e-3)


def test_basic_delta_range_2d():
    """Sec. V: over the 4! = 24 intra-first orders Delta spans [2, 5]; it is
    5 whenever the x neighbour comes last; best S_max(2,5) = 2.5."""
    g = GOLD["basic_delta_range"]
    inter = [(0, -1, 0), (1, -1, 0), (1, 0, 0), (1, 1, 0)]
    deltas = {}
    for p in itertools.permutations(inter):
        deltas[p] = _delta([O.INTRA] + list(p), lambda m: (m, 3, 1), m=60)
    assert len(deltas) == 24
    assert min(deltas.values()) == g["2d"][0]
    assert max(deltas.values()) == g["2d"][1]
    assert all(v == 5 for p, v in deltas.items() if p[-1] == (1, 0, 0))
    # x neighbour right after intra gives Delta = 2 for most orders; one order
    # (x, below, upper-right, lower-right) reaches 3 -- the exact DAG decides
    after = [v for p, v in deltas.items() if p[0] == (1, 0, 0)]
    assert after.count(2) == 5 and max(after) == 3
    assert O.smax_eq3(min(deltas.values()), 5) == g["best_basic_smax_2d"]


def test_3d_orders():
    """Sec. V: 3D basic orders have Delta in [2, 14]; best basic S_max = 7,
    worst 1; the x-neighbour-first order pipelines with Delta = 1 (S -> 14)."""
    g = GOLD["basic_delta_range"]
    dims = lambda m: (m, 3, 3)
    assert _delta(O.ORDER3_BEST, dims, m=40) == g["3d"][0]
    assert _delta(O.ORDER3_BAD, dims, m=40) == g["3d"][1]
    assert O.smax_eq3(2, 14) == g["best_basic_smax_3d"]
    assert O.smax_eq3(_delta(O.ORDER3_OPT, dims, m=40), 14) == \
        GOLD["opt_pipeline_bound"]["3d"]
    assert O.smax_eq3(_delta(O.ORDER3_BAD, dims, m=40), 14) == g["worst_smax"]
    # the lexicographic reading of the standard order sits in between
    assert _delta(O.ORDER3_LEX, dims, m=40) == 7


def test_eq2_eq4_closed_forms():
    """Eq. 2 at Delta = 1 is Eq. 4; Eq. 2 tends to Eq. 3; Delta = n gives 1."""
    for n in (5, 14):
        for k in (1, 7, 2500):
            assert O.speedup_eq2(1, k, n) == pytest.approx(O.pipeline_eq4(n, k))
            assert O.speedup_eq2(n, k, n) == pytest.approx(1.0)
    assert O.speedup_eq2(4, 10 ** 9, 5) == pytest.approx(1.25, rel=1e-8)
    assert O.pipeline_eq4(5, 10 ** 9) == pytest.approx(5.0, rel=1e-8)


def test_periodic_closed_forms_2d():
    """Exact critical paths on periodic Nx x Ny grids (derived from the
    row-by-row chain structure and confirmed here over a range of sizes):
    naive (4 Nx + 1) Ny, bad (5 Nx - 1) Ny + 1, optimal (Nx + 2) Ny + 2 for
    Nx >= 6.  At 50 x 50 these give S = 1.2438 / 1.0039 / 4.804."""
    for nx in range(6, 12):
        for ny in range(3, 7):
            k = nx * ny
            assert O.serialization_degree((nx, ny, 1), O.ORDER2_NAIVE)["cp"] == (4 * nx + 1) * ny
            assert O.serialization_degree((nx, ny, 1), O.ORDER2_BAD)["cp"] == (5 * nx - 1) * ny + 1
            assert O.serialization_degree((nx, ny, 1), O.ORDER2_OPT)["cp"] == (nx + 2) * ny + 2
            assert k * 5 == O.serialization_degree((nx, ny, 1), O.ORDER2_OPT)["T"]
    s = O.serialization_degree((50, 50, 1), O.ORDER2_OPT)["S"]
    assert s == pytest.approx(12500 / 2602)


def test_loop_exchange_colouring():
    """Sec. VI strategy 1: with loop exchange and two-strided colouring the
    critical path no longer grows with the domain (2n - 1 levels), so the
    speedup grows with the number of cells; colouring alone (without loop
    exchange) is not enough."""
    for dims in ((4, 4, 1), (8, 6, 1), (20, 20, 1)):
        sd = O.serialization_degree(dims, O.ORDER2_NAIVE, loopex=True)
        assert sd["cp"] == 2 * 5 - 1
    for dims in ((4, 4, 4), (6, 6, 6)):
        sd = O.serialization_degree(dims, O.ORDER3_LEX, loopex=True)
        assert sd["cp"] == 2 * 14 - 1
    # colour-major cell order with the whole stencil per cell (no exchange)
    import numpy as np
    nx = ny = 8
    order = O.ORDER2_OPT
    A, B = [], []
    for cy in range(2):
        for cx in range(2):
            for y in range(cy, ny, 2):
                for x in range(cx, nx, 2):
                    for d in order:
                        A.append(x + nx * y)
                        B.append(((x + d[0]) % nx) + nx * ((y + d[1]) % ny))
    _, cp_col = O.dag_lc(np.array(A, dtype=np.int32), np.array(B, dtype=np.int32))
    cp_lx = O.serialization_degree((nx, ny, 1), order, loopex=True)["cp"]
    assert cp_col > 2 * cp_lx


def test_loopex_rejects_odd_dims():
    with pytest.raises(O.OracleError):
        O.lc_tasks((5, 4, 1), O.ORDER2_OPT, loopex=True)


def test_weighted_dag_reduces_to_unit():
    """With unit durations the weighted critical path is the task count one;
    scaling all durations scales it."""
    import numpy as np
    A, B = O.lc_tasks((6, 4, 1), O.ORDER2_NAIVE)
    _, cp = O.dag_lc(A, B)
    _, cpw = O.dag_lc_weighted(A, B, np.ones(len(A)))
    assert cpw == cp
    _, cpw3 = O.dag_lc_weighted(A, B, 3.0 * np.ones(len(A)))
    assert cpw3 == 3 * cp
    # one heavy task on the critical chain adds its extra duration
    w = np.ones(len(A))
    w[0] = 10.0
    _, cpw10 = O.dag_lc_weighted(A, B, w)
    assert cpw10 == cp + 9
