"""The dataflow log checker on synthetic logs (no GPU): a serial run passes
every rule, and a log that breaks one rule is caught by that rule's check."""
import numpy as np

from paper_1401_4441_amd import dataflow_check as D

# four tasks on three cells: t0 (0,0), t1 (0,1), t2 (2,2), t3 (1,2)
A = np.array([0, 0, 2, 1])
B = np.array([0, 1, 2, 2])


def _log(intervals):
    s = np.array([a for a, _ in intervals])
    e = np.array([b for _, b in intervals])
    return np.concatenate([s, e])


def test_serial_run_passes_everything():
    log = _log([(0, 1), (2, 3), (4, 5), (6, 7)])
    assert D.check_complete(log, 4) == 0
    assert D.check_ordered(A, B, log) == 0
    assert D.check_exclusive(A, B, log) == 0
    assert D.check_chains(log, 4, 2) == 0


def test_independent_tasks_may_overlap_and_reorder():
    # t2 (cell 2) is independent of t0, t1 (cells 0, 1): it may run first
    # and overlap them; t3 needs t1 (cell 1) and t2 (cell 2) done
    log = _log([(1, 3), (4, 5), (0, 2), (6, 7)])
    assert D.check_complete(log, 4) == 0
    assert D.check_ordered(A, B, log) == 0
    assert D.check_exclusive(A, B, log) == 0


def test_ordered_catches_a_dependent_task_run_early():
    # t3 starts before t1 ended (they share cell 1), though they do not
    # overlap the other way round
    log = _log([(0, 1), (5, 6), (2, 3), (4, 7)])
    assert D.check_ordered(A, B, log) == 1
    # in a different order without overlap, mutual exclusion still holds
    assert D.check_exclusive(A, B, log) == 1  # t3 [4,7] overlaps t1 [5,6]
    log2 = _log([(0, 1), (6, 7), (2, 3), (4, 5)])  # t3 before t1, no overlap
    assert D.check_ordered(A, B, log2) == 1
    assert D.check_exclusive(A, B, log2) == 0


def test_exclusive_catches_overlap_on_a_shared_cell():
    log = _log([(0, 3), (1, 4), (5, 6), (2, 7)])  # t0, t1 share cell 0
    assert D.check_exclusive(A, B, log) >= 1
    # the intra task t2 and t3 share cell 2
    log = _log([(0, 1), (2, 3), (4, 6), (5, 7)])
    assert D.check_exclusive(A, B, log) == 1


def test_chains_and_completeness():
    # chains of two: (t0, t1) and (t2, t3); t3 starts before t2 ends
    log = _log([(0, 1), (2, 3), (4, 6), (5, 7)])
    assert D.check_chains(log, 4, 2) == 1
    assert D.check_complete(_log([(0, 1), (2, 3), (4, 5), (-1, -1)]), 4) >= 1
    assert D.check_complete(_log([(0, 1), (1, 3), (4, 5), (6, 7)]), 4) >= 1
    assert D.check_complete(_log([(1, 0), (2, 3), (4, 5), (6, 7)]), 4) >= 1
