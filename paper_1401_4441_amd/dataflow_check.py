"""Checks of a dataflow execution log (lc_compute_forces_dataflow_log)
against the constraint of its strategy.

The log holds, for every task t of a creation order, a start ticket log[t]
(taken once the task's cells were granted, before any of its work) and an
end ticket log[T + t] (taken after its force adds completed, before its cells
were released), all drawn from one device counter.  What each executor must
guarantee:

* ordered -- the inout dependences of the task DAG (Sec. III, Sec. V): a
  task starts only after every earlier task in creation order that touches
  one of its cells has ended;
* mutex / nested -- mutual exclusion on the cells a task writes (the clause
  Sec. VII asks for): two tasks sharing a cell never run at the same time;
  nested (Sec. VI strategy 2) also runs each cell's chain of tasks in order.

Pure numpy host logic; every function returns the number of violations.
"""
from __future__ import annotations

import numpy as np


def split_log(log, ntask: int):
    """(start, end) int64 arrays of a 2 x T log."""
    log = np.asarray(log, dtype=np.int64).reshape(-1)
    if log.shape[0] != 2 * ntask:
        raise ValueError(f"log has {log.shape[0]} entries, expected {2 * ntask}")
    return log[:ntask], log[ntask:]


def check_complete(log, ntask: int) -> int:
    """Every task ran once and its tickets are ordered: the 2T tickets are a
    permutation of 0 .. 2T-1 and start < end for every task.  Returns the
    number of tasks that break it."""
    start, end = split_log(log, ntask)
    bad = (start < 0) | (end < 0) | (start >= end)
    allv = np.concatenate([start, end])
    if not np.array_equal(np.sort(allv), np.arange(2 * ntask)):
        return int(bad.sum()) + 1
    return int(bad.sum())


def _cell_visits(A, B):
    """(cell, task) of every cell a task writes: A, and B when B != A."""
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    t = np.arange(A.shape[0], dtype=np.int64)
    other = B != A
    return np.concatenate([A, B[other]]), np.concatenate([t, t[other]])


def check_ordered(A, B, log) -> int:
    """Count pairs (t', t) of consecutive tasks on one cell in creation order
    where t started before t' ended.  Consecutive pairs suffice: the
    dependences along one cell form a chain."""
    start, end = split_log(log, len(A))
    cells, ts = _cell_visits(A, B)
    o = np.lexsort((ts, cells))
    c, t = cells[o], ts[o]
    same = c[1:] == c[:-1]
    return int(np.sum(same & (start[t[1:]] <= end[t[:-1]])))


def check_exclusive(A, B, log) -> int:
    """Count pairs of tasks sharing a cell whose [start, end] intervals
    overlap: per cell, sorted by start, each task must end before the next
    one starts."""
    start, end = split_log(log, len(A))
    cells, ts = _cell_visits(A, B)
    o = np.lexsort((start[ts], cells))
    c, t = cells[o], ts[o]
    same = c[1:] == c[:-1]
    return int(np.sum(same & (start[t[1:]] <= end[t[:-1]])))


def check_chains(log, ntask: int, chain: int) -> int:
    """Count consecutive tasks of one chain (tasks [c chain, (c + 1) chain))
    that did not run one after the other."""
    start, end = split_log(log, ntask)
    t = np.arange(ntask - 1)
    inner = (t + 1) % chain != 0
    return int(np.sum(inner & (start[t + 1] <= end[t])))
