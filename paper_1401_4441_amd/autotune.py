"""Autotuner for the link-cell force sweep.

It times candidate configurations on the device through the C-ABI and keeps
the fastest: the cell grid (cell side rc, optionally widened, cell counts
rounded to even or not), the conflict-free schedule (BLOCK8 colouring or
BUFFER buffer + reduce; ATOMIC_TILE when atomics are allowed) and the block
shape (for BLOCK8 the smallest block per axis, for the uncoloured kinds the
largest).  For a batch of boxes it picks the cell grids (side rc or widened),
the LDS tile the split boxes' block shapes are sized for, how boxes are split
(whole-box work-groups where they fit, or blocks) and whether the sweep runs
as a persistent launch.  Results are cached in a JSON file keyed
by the device name and a bucket of (N, density, rc).
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import lc

CACHE_ENV = "LC_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1401_4441_amd",
                             "tune.json")

BOX_KINDS_CONFLICT_FREE = ("block8", "buffer")
# Block sizes are upper bounds (BLOCK8: even block counts).  Tasks join the block of their lower corner cell, so a block's
# footprint is (bx + r)(by + r)(bz + r) cells at stencil reach r.  Shapes
# whose footprint outgrows the LDS tile lose on their own (fewer work-groups
# per compute unit), so they need no pruning here.
BLOCKS = {"block8": ((1, 1, 1), (1, 1, 2), (1, 2, 2), (1, 2, 3), (2, 2, 2), (1, 3, 3),
                     (2, 3, 3)),
          "uncoloured": ((1, 2, 2), (1, 2, 3), (1, 3, 3), (2, 2, 2), (2, 2, 3), (1, 3, 4),
                         (1, 4, 4), (2, 3, 3)),
          # cells of side rc/2 (reach 2): at most 8 cells per block (63
          # tasks per cell, 512 per work-group), footprints within 128 cells
          "uncoloured_half": ((1, 1, 1), (1, 1, 2), (1, 2, 2), (1, 2, 3), (2, 2, 2),
                              (1, 2, 4)),
          "block8_half": ((2, 2, 2),),
          # flat (2D) grids: one cell along z; a block's footprint is
          # (bx + 1) x (by + 1) cells
          "flat": ((2, 4, 1), (4, 4, 1), (4, 8, 1), (8, 8, 1), (6, 12, 1), (8, 12, 1),
                   (10, 10, 1))}


def shapes_for(kind: str, half: bool = False, flat: bool = False):
    if flat:
        return BLOCKS["flat"]
    if kind == "block8":
        return BLOCKS["block8_half"] if half else BLOCKS["block8"]
    return BLOCKS["uncoloured_half"] if half else BLOCKS["uncoloured"]
GRIDS = ({"extra": 0.0, "even": True}, {"extra": 0.0, "even": False},
         {"extra": 0.15, "even": True}, {"extra": 0.0, "even": False, "half": True})


def _first_schedule(grid, kinds):
    """A schedule of the first kind the grid supports (for clock warm-up)."""
    for kind in kinds:
        try:
            return lc.Schedule(grid, kind)
        except lc.LCError:
            continue
    raise lc.LCError(-1, "autotune: no schedule kind fits this grid")


def make_grid(L, rc: float, gopt: dict):
    """The grid a GRIDS entry (or a trial's "grid" record) describes."""
    return lc.Grid(L, rc, gopt["extra"], gopt["even"], half=gopt.get("half", False))


def _cache_path() -> str:
    return os.environ.get(CACHE_ENV, DEFAULT_CACHE)


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def box_key(n: int, L, rc: float) -> str:
    """Bucket: log2(N) in quarter steps, density to 0.05, rc to 0.01."""
    vol = float(L[0]) * float(L[1]) * float(L[2])
    rho = n / vol
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return f"{dev}|n{round(4 * math.log2(max(n, 1)))}|rho{round(rho / 0.05)}|rc{rc:.2f}"


def time_forces(grid, sched, cs, coord, ws, reps=5, warmup=2, rounds=3) -> float:
    """ms of one lc_compute_forces: the fastest of `rounds` averages over
    `reps` back-to-back calls (the minimum discards rounds slowed by other
    work or clock changes)."""
    for _ in range(warmup):
        lc.compute_forces(grid, sched, cs, coord, ws)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(rounds):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lc.compute_forces(grid, sched, cs, coord, ws)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def tune_box(pos: torch.Tensor, L, rc: float, allow_atomics: bool = False,
             reps: int = 5, use_cache: bool = True, kinds=None) -> dict:
    """Pick grid, schedule kind and block shape for one box.

    pos: (3, N) float64 cuda tensor.  kinds: the schedule kinds to try
    (default: the conflict-free ones, plus ATOMIC_TILE with allow_atomics).
    Returns {"grid": {...}, "kind": str, "block": [x, y, z], "ms": float,
    "trials": [...]} for the fastest of all trials."""
    n = pos.shape[1]
    if kinds is None:
        kinds = BOX_KINDS_CONFLICT_FREE + (("atomic_tile",) if allow_atomics else ())
    kinds = tuple(kinds)
    key = box_key(n, L, rc) + "|" + ",".join(kinds) + "|v6"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]
    trials = []
    best = None
    warmed = False
    for gopt in GRIDS:
        try:
            grid = make_grid(L, rc, gopt)
        except lc.LCError:
            continue
        ws = lc.Workspace(n, grid.ncell)
        cs, perm, coord = lc.build_cells(grid, pos, ws)
        # trials launch their groups heaviest first, as the final schedule
        # does, which also sizes each trial's LDS tile to its footprints
        cc = lc.cell_counts_of(cs)
        if not warmed:  # bring the clocks up before the first trial counts
            s0 = _first_schedule(grid, kinds)
            t_end = time.perf_counter() + 0.3
            while time.perf_counter() < t_end:
                time_forces(grid, s0, cs, coord, ws, reps=10, warmup=0, rounds=1)
            s0.close()
            warmed = True
        for kind in kinds:
            for block in shapes_for(kind, grid.reach == 2, grid.nc[2] == 1):
                try:
                    sched = lc.Schedule(grid, kind, block=block, cell_counts=cc)
                except lc.LCError:
                    continue
                ws.clear_status()
                ms = time_forces(grid, sched, cs, coord, ws, reps=reps)
                # a footprint beyond the LDS tile runs the (exact) global
                # fallback: that times the safety net, not the tiled sweep
                fell_back = bool(ws.status() & lc.FLAG_FALLBACK)
                ws.clear_status()
                rec = {"grid": dict(gopt), "kind": kind, "block": list(block), "ms": ms,
                       "nc": list(grid.nc), "fallback": fell_back}
                trials.append(rec)
                if not fell_back and (best is None or ms < best["ms"]):
                    best = rec
                sched.close()
        ws.close()
    if best is None:
        raise lc.LCError(-1, "autotune: no valid configuration")
    out = dict(best)
    out["trials"] = trials
    if use_cache:
        cache[key] = out
        _store_cache(cache)
    return out


def tune_shape(grid, pos: torch.Tensor, kinds=BOX_KINDS_CONFLICT_FREE, reps: int = 10) -> dict:
    """Schedule kind and block shape on a fixed grid (e.g. one with a
    Verlet skin).  Returns {"kind", "block", "ms", "trials"}."""
    n = pos.shape[1]
    ws = lc.Workspace(n, grid.ncell)
    cs, perm, coord = lc.build_cells(grid, pos, ws)
    cc = lc.cell_counts_of(cs)  # load-aware trials (see tune_box)
    s0 = _first_schedule(grid, kinds)
    t_end = time.perf_counter() + 0.3
    while time.perf_counter() < t_end:  # clocks up before the trials count
        time_forces(grid, s0, cs, coord, ws, reps=10, warmup=0, rounds=1)
    s0.close()
    trials, best = [], None
    for kind in kinds:
        for block in shapes_for(kind, grid.reach == 2, grid.nc[2] == 1):
            try:
                sched = lc.Schedule(grid, kind, block=block, cell_counts=cc)
            except lc.LCError:
                continue
            ws.clear_status()
            ms = time_forces(grid, sched, cs, coord, ws, reps=reps)
            fell_back = bool(ws.status() & lc.FLAG_FALLBACK)
            ws.clear_status()
            rec = {"kind": kind, "block": list(block), "ms": ms, "fallback": fell_back}
            trials.append(rec)
            if not fell_back and (best is None or ms < best["ms"]):
                best = rec
            sched.close()
    ws.close()
    if best is None:
        raise lc.LCError(-1, "autotune: no valid configuration")
    out = dict(best)
    out["trials"] = trials
    return out


BATCH_TILES = (512, 768, 1024, 2048)


def tune_batch(grids, ns, pos_all: torch.Tensor, reps: int = 5, grid_sets=None,
               tiles=BATCH_TILES) -> dict:
    """Pick, for a batch, the cell grids (``grid_sets``: name -> one grid per
    box, e.g. cells of side rc and cells widened by a skin; default: the
    given ``grids`` as "given"), the LDS tile the split boxes' block shapes
    are sized for (``tiles``), the box split (auto: whole-box work-groups
    where they fit, or blocks everywhere) and persistent vs
    one-group-per-work-group launch, all with buffer + reduce write-back.
    Returns {"grid", "tile", "modes", "persistent", "ms", "trials": [...]}."""
    if grid_sets is None:
        grid_sets = {"given": grids}
    trials = []
    best = None
    for gname, gset in grid_sets.items():
        for tile in tiles:
            for modes in ("auto", "blocks"):
                batch = lc.Batch(gset, ns, None if modes == "auto" else ["blocks"] * len(ns),
                                 tile=tile)
                info = batch.info()
                ws = lc.Workspace(info["ntot"], info["ncell"])
                cs, perm, coord = batch.build_cells(pos_all, ws)
                F = torch.empty((3, info["ntot"]), dtype=torch.int64, device=pos_all.device)
                ew = torch.empty((len(ns), 3), dtype=torch.int64, device=pos_all.device)
                for persistent in (True, False):
                    for _ in range(2):
                        batch.forces(cs, coord, ws, F, ew, persistent)
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        batch.forces(cs, coord, ws, F, ew, persistent)
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    rec = {"grid": gname, "tile": tile, "modes": modes,
                           "persistent": persistent, "ms": ms, "nwhole": info["nwhole"],
                           "ngroup": info["ngroup"], "lds_tile": info["lds_tile"],
                           "fallback": bool(ws.status() & lc.FLAG_FALLBACK)}
                    trials.append(rec)
                    if not rec["fallback"] and (best is None or ms < best["ms"]):
                        best = rec
                batch.close()
                ws.close()
    if best is None:  # every trial spilled out of its tile: take the fastest
        best = min(trials, key=lambda t: t["ms"])
    out = dict(best)
    out["trials"] = trials
    return out
