"""Python binding of ``liblc.so`` (include/lc.h): argument marshalling only.

Every step of the force sweep runs in the HIP library; this module turns
torch tensors (device memory) and the current torch stream into the raw
pointers the C-ABI takes, and raises :class:`LCError` on a negative status.
If the library has not been built the import fails loudly -- there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblc.so")

# schedule kinds (LC_SCHED_*)
LEX, OPT, BEST, BAD, LOOPEX, BLOCK8, ATOMIC_TILE, ATOMIC_PAIR, CUSTOM, BUFFER, FULLSHELL = \
    range(11)
KINDS = {"lex": LEX, "opt": OPT, "best": BEST, "bad": BAD, "loopex": LOOPEX,
         "block8": BLOCK8, "atomic_tile": ATOMIC_TILE, "atomic_pair": ATOMIC_PAIR,
         "custom": CUSTOM, "buffer": BUFFER, "fullshell": FULLSHELL}
PREC = {"fp32": 0, "fp64": 1}
FLAG_OVERFLOW, FLAG_DISP, FLAG_FALLBACK, FLAG_ABORT = 1, 2, 4, 8
# dataflow executors (LC_DF_*)
DATAFLOW = {"ordered": 0, "mutex": 1, "nested": 2}
SCALE = 2.0 ** 32


class LCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lc error {code}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("inv_box", ctypes.c_double * 3),
                ("rc", ctypes.c_double), ("skin", ctypes.c_double),
                ("nc", ctypes.c_int32 * 3), ("ncell", ctypes.c_int32),
                ("scale", ctypes.c_float * 3), ("rc2", ctypes.c_float),
                ("ecut", ctypes.c_float), ("reach", ctypes.c_int32)]


class _SchedInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nphase", ctypes.c_int32),
                ("ntask", ctypes.c_int64), ("ngroup", ctypes.c_int64),
                ("max_group_tasks", ctypes.c_int32),
                ("max_group_cells", ctypes.c_int32),
                ("write_mode", ctypes.c_int32), ("max_replicas", ctypes.c_int32)]


class _WSD(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_int64), ("work", ctypes.c_double),
                ("cp", ctypes.c_double), ("speedup", ctypes.c_double)]


class _SD(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_int64), ("cp", ctypes.c_int64),
                ("speedup", ctypes.c_double), ("degree", ctypes.c_double),
                ("n", ctypes.c_int32), ("delta", ctypes.c_int32),
                ("s_eq2", ctypes.c_double), ("s_max", ctypes.c_double)]


_lib = None
P = ctypes.c_void_p
I64 = ctypes.c_int64
INT = ctypes.c_int

SYMBOLS = {
    "lc_last_error": ([], ctypes.c_char_p),
    "lc_make_grid": ([P, ctypes.c_double, ctypes.c_double, INT, P], INT),
    "lc_workspace_create": ([I64, I64, P], INT),
    "lc_workspace_destroy": ([P], None),
    "lc_workspace_clear_status": ([P, P], INT),
    "lc_workspace_set_tile_hint": ([P, ctypes.c_int32], INT),
    "lc_workspace_status": ([P, P, P], INT),
    "lc_workspace_check": ([P, P], INT),
    "lc_build_cells": ([P, P, I64, P, P, P, P, P], INT),
    "lc_gather": ([P, I64, P, P, P, P, P], INT),
    "lc_make_schedule": ([P, INT, P, INT, P], INT),
    "lc_make_schedule_ex": ([P, INT, P, INT, P, P], INT),
    "lc_make_schedule_weighted": ([P, INT, P, INT, P, P, P], INT),
    "lc_schedule_group_work": ([P, P, P], INT),
    "lc_schedule_info_get": ([P, P], INT),
    "lc_schedule_free": ([P], None),
    "lc_schedule_plan": ([P, INT, P, INT, P], INT),
    "lc_schedule_plan_ex": ([P, INT, P, INT, P, P], INT),
    "lc_schedule_plan_tasks": ([P, INT, P, INT, P, P, P, P, P, I64, P], INT),
    "lc_validate_phases": ([I64, ctypes.c_int32, P, P, P], INT),
    "lc_serialization_degree": ([P, INT, P, INT, P, I64, P], INT),
    "lc_serialization_degree_weighted": ([P, INT, P, INT, P, P], INT),
    "lc_compute_forces": ([P, P, P, P, I64, P, P, INT, P, P], INT),
    "lc_compute_forces_dataflow": ([P, P, INT, P, P, I64, P, P, ctypes.c_double, P, P], INT),
    "lc_compute_forces_dataflow_log": ([P, P, INT, P, P, I64, P, P, ctypes.c_double, P, P, P],
                                       INT),
    "lc_schedule_tasks": ([P, P, P, I64, P], INT),
    "lc_schedule_cell_footprints": ([P, P, I64], INT),
    "lc_compute_forces_profiled": ([P, P, P, P, I64, P, P, INT, P, P, P, P], INT),
    "lc_compute_forces_noalloc": ([P, P, P, P, I64, P, P, INT, P, P], INT),
    "lc_verlet_step": ([P, P, P, P, P, I64, P, P, P, P, ctypes.c_double, INT,
                        INT, P, P, P], INT),
    "lc_kinetic_energy": ([P, I64, P, P, P], INT),
    "lc_selftest_recip": ([ctypes.c_uint32, ctypes.c_uint32, P], INT),
    "lc_batch_create": ([P, INT, P, P], INT),
    "lc_batch_create_ex": ([P, INT, P, P, P], INT),
    "lc_batch_info_get": ([P, P], INT),
    "lc_batch_offsets": ([P, P, P], INT),
    "lc_batch_free": ([P], None),
    "lc_batch_build_cells": ([P, P, P, P, P, P, P], INT),
    "lc_batch_forces": ([P, P, P, P, P, INT, P, P], INT),
    "lc_batch_graph_create": ([P, P, P, P, P, INT, P, P, P], INT),
    "lc_forces_graph_create": ([P, P, P, P, I64, P, P, INT, P, P, P], INT),
    "lc_graph_launch": ([P, P], INT),
    "lc_graph_free": ([P], None),
}


def lib():
    """Load the in-tree liblc.so; raise if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1401_4441_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _chk(rc: int):
    if rc < 0:
        raise LCError(rc, lib().lc_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _p(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------

GRID_EVEN, GRID_HALF, GRID_2D = 1, 2, 4


class Grid:
    """Periodic cell grid.  half: cells of side >= (rc + skin) / 2, so the
    stencil reaches two cells (fewer candidate pairs; schedules follow).
    flat: a 2D system (all particles at one z), one cell along z, the 2D
    stencil and orders."""

    def __init__(self, box, rc: float, skin: float = 0.0, even: bool = False,
                 half: bool = False, flat: bool = False):
        self._g = _Grid()
        b = (ctypes.c_double * 3)(*[float(x) for x in box])
        flags = (GRID_EVEN if even else 0) | (GRID_HALF if half else 0) | \
            (GRID_2D if flat else 0)
        _chk(lib().lc_make_grid(ctypes.cast(b, P), float(rc), float(skin),
                                flags, ctypes.byref(self._g)))

    @property
    def reach(self) -> int:
        return int(self._g.reach)

    @property
    def ptr(self):
        return ctypes.byref(self._g)

    @property
    def nc(self):
        return tuple(self._g.nc)

    @property
    def ncell(self) -> int:
        return int(self._g.ncell)

    @property
    def box(self):
        return tuple(self._g.box)

    @property
    def rc(self) -> float:
        return float(self._g.rc)

    @property
    def skin(self) -> float:
        return float(self._g.skin)


class Workspace:
    def __init__(self, max_n: int, max_cells: int):
        self._live_graphs = 0  # graphs captured with this workspace, alive
        self._h = ctypes.c_void_p()
        _chk(lib().lc_workspace_create(int(max_n), int(max_cells),
                                       ctypes.byref(self._h)))

    @property
    def ptr(self):
        return self._h

    def clear_status(self, stream=None):
        _chk(lib().lc_workspace_clear_status(self._h, _stream(stream)))

    def set_tile_hint(self, max_per_cell: int):
        _chk(lib().lc_workspace_set_tile_hint(self._h, int(max_per_cell)))

    def status(self, stream=None) -> int:
        v = ctypes.c_uint32(0)
        _chk(lib().lc_workspace_status(self._h, _stream(stream), ctypes.byref(v)))
        return int(v.value)

    def check(self, stream=None):
        """Synchronise and raise LCError (-5 overflow, -8 abandoned dataflow
        evaluation, -6 displacement beyond skin / 2) if a device flag is set."""
        _chk(lib().lc_workspace_check(self._h, _stream(stream)))

    def close(self):
        if self._live_graphs:
            raise LCError(-7, "the workspace is held by a live graph: close the graph first")
        if self._h:
            lib().lc_workspace_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _counts_array(cell_counts, ncell: int):
    import numpy as np
    if isinstance(cell_counts, torch.Tensor):
        cell_counts = cell_counts.detach().cpu().numpy()
    arr = np.ascontiguousarray(np.asarray(cell_counts, dtype=np.int32).reshape(-1))
    if arr.shape[0] != ncell:
        raise LCError(-1, f"cell_counts has {arr.shape[0]} entries, the grid {ncell} cells")
    return arr


def cell_counts_of(cell_start) -> "object":
    """Per-cell particle counts (host int32) from a cell_start array."""
    import numpy as np
    if isinstance(cell_start, torch.Tensor):
        cell_start = cell_start.detach().cpu().numpy()
    return np.diff(np.asarray(cell_start, dtype=np.int64)).astype(np.int32)


class Schedule:
    """A schedule of `kind` on `grid`.  cell_counts (per-cell particle
    counts, e.g. cell_counts_of(cell_start)): launch each phase's work-groups
    heaviest first (load-aware order)."""

    def __init__(self, grid: Grid, kind, offsets=None, block=None, cell_counts=None):
        if isinstance(kind, str):
            kind = KINDS[kind]
        self._h = ctypes.c_void_p()
        self.grid = grid
        if offsets is not None:
            import numpy as np
            arr = np.ascontiguousarray(np.asarray(offsets, dtype=np.int8).reshape(-1, 3))
            self._offs = arr
            op, n = ctypes.c_void_p(arr.ctypes.data), arr.shape[0]
        else:
            op, n = None, 0
        if block is not None:
            self._block = (ctypes.c_int32 * 3)(*[int(x) for x in block])
            bp = ctypes.cast(self._block, P)
        else:
            bp = None
        self.kind = int(kind)
        self.block = tuple(block) if block is not None else None
        self._live_graphs = 0  # graphs captured with this schedule, alive
        if cell_counts is None:
            _chk(lib().lc_make_schedule_ex(grid.ptr, int(kind), op, int(n), bp,
                                           ctypes.byref(self._h)))
        else:
            cc = _counts_array(cell_counts, grid.ncell)
            _chk(lib().lc_make_schedule_weighted(grid.ptr, int(kind), op, int(n), bp,
                                                 ctypes.c_void_p(cc.ctypes.data),
                                                 ctypes.byref(self._h)))

    def group_work(self, cell_counts):
        """Estimated work of every work-group, in launch order (numpy)."""
        import numpy as np
        cc = _counts_array(cell_counts, self.grid.ncell)
        out = np.zeros(self.info()["ngroup"], dtype=np.float64)
        _chk(lib().lc_schedule_group_work(self._h, ctypes.c_void_p(cc.ctypes.data),
                                          ctypes.c_void_p(out.ctypes.data)))
        return out

    @property
    def ptr(self):
        return self._h

    def info(self) -> dict:
        i = _SchedInfo()
        _chk(lib().lc_schedule_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _SchedInfo._fields_ if k != "pad"}

    def cell_footprints(self):
        """int32 numpy array, per cell: how many work-group footprints hold
        it (the replica slots of buffer + reduce)."""
        import numpy as np
        out = np.zeros(self.grid.ncell, dtype=np.int32)
        _chk(lib().lc_schedule_cell_footprints(self._h, ctypes.c_void_p(out.ctypes.data),
                                               self.grid.ncell))
        return out

    def tasks(self):
        """(A, B) int32 numpy arrays: a creation-order schedule's tasks in
        creation order."""
        import numpy as np
        nt = ctypes.c_int64(0)
        rc = lib().lc_schedule_tasks(self._h, None, None, 0, ctypes.byref(nt))
        if rc < 0 and nt.value == 0:
            _chk(rc)
        A = np.empty(nt.value, dtype=np.int32)
        B = np.empty(nt.value, dtype=np.int32)
        _chk(lib().lc_schedule_tasks(self._h, ctypes.c_void_p(A.ctypes.data),
                                     ctypes.c_void_p(B.ctypes.data), nt.value,
                                     ctypes.byref(nt)))
        return A, B

    def close(self):
        if self._live_graphs:
            raise LCError(-7, "the schedule is held by a live graph: close the graph first")
        if self._h:
            lib().lc_schedule_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def schedule_plan(grid: Grid, kind, offsets=None, block=None) -> dict:
    """Host-only: build and validate a schedule, return its shape.  block:
    the block shape of the block kinds (see Schedule)."""
    import numpy as np
    if isinstance(kind, str):
        kind = KINDS[kind]
    if offsets is not None:
        arr = np.ascontiguousarray(np.asarray(offsets, dtype=np.int8).reshape(-1, 3))
        op, n = ctypes.c_void_p(arr.ctypes.data), arr.shape[0]
    else:
        op, n = None, 0
    bp = None
    if block is not None:
        barr = np.ascontiguousarray(np.asarray(block, dtype=np.int32).reshape(3))
        bp = ctypes.c_void_p(barr.ctypes.data)
    i = _SchedInfo()
    _chk(lib().lc_schedule_plan_ex(grid.ptr, int(kind), op, int(n), bp, ctypes.byref(i)))
    return {k: getattr(i, k) for k, _ in _SchedInfo._fields_ if k != "pad"}


def schedule_plan_tasks(grid: Grid, kind, offsets=None, block=None):
    """Host-only: the tasks of the schedule schedule_plan describes, in
    launch order, as int32 numpy arrays (A, B, group, phase)."""
    import numpy as np
    if isinstance(kind, str):
        kind = KINDS[kind]
    if offsets is not None:
        arr = np.ascontiguousarray(np.asarray(offsets, dtype=np.int8).reshape(-1, 3))
        op, n = ctypes.c_void_p(arr.ctypes.data), arr.shape[0]
    else:
        op, n = None, 0
    bp = None
    if block is not None:
        barr = np.ascontiguousarray(np.asarray(block, dtype=np.int32).reshape(3))
        bp = ctypes.c_void_p(barr.ctypes.data)
    nt = ctypes.c_int64(0)
    rc = lib().lc_schedule_plan_tasks(grid.ptr, int(kind), op, int(n), bp, None, None, None,
                                      None, 0, ctypes.byref(nt))
    if rc not in (0, -7):  # LC_ECAPACITY: the count is set
        _chk(rc)
    out = [np.zeros(nt.value, dtype=np.int32) for _ in range(4)]
    _chk(lib().lc_schedule_plan_tasks(grid.ptr, int(kind), op, int(n), bp,
                                      *[ctypes.c_void_p(a.ctypes.data) for a in out],
                                      nt.value, ctypes.byref(nt)))
    return tuple(out)


def validate_phases(ncell: int, phase_grp, grp_foot, foot_cells) -> None:
    """Host-only schedule validator on explicit arrays; raises LCError
    (code LC_ESCHED = -4) when a phase has two groups writing one cell."""
    import numpy as np
    pg = np.ascontiguousarray(np.asarray(phase_grp, dtype=np.int32))
    gf = np.ascontiguousarray(np.asarray(grp_foot, dtype=np.int32))
    fc = np.ascontiguousarray(np.asarray(foot_cells, dtype=np.int32))
    _chk(lib().lc_validate_phases(int(ncell), len(pg) - 1, ctypes.c_void_p(pg.ctypes.data),
                                  ctypes.c_void_p(gf.ctypes.data),
                                  ctypes.c_void_p(fc.ctypes.data)))


def build_cells(grid: Grid, pos: torch.Tensor, ws: Workspace, cell_start=None,
                perm=None, coord=None, stream=None, tile_hint: bool = True):
    """Counting sort into cells.  pos: (3, N) float64 cuda.  Returns
    (cell_start int32 [ncell+1], perm int32 [N], coord uint32-as-int32 (3, N))."""
    n = pos.shape[1]
    dev = pos.device
    if cell_start is None:
        cell_start = torch.empty(grid.ncell + 1, dtype=torch.int32, device=dev)
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    if coord is None:
        coord = torch.empty((3, n), dtype=torch.int32, device=dev)
    _chk(lib().lc_build_cells(grid.ptr, _p(pos), n, _p(cell_start), _p(perm),
                              _p(coord), ws.ptr, _stream(stream)))
    if tile_hint:
        # the largest cell sizes the LDS tile of the sweep (one small sync)
        ws.set_tile_hint(int((cell_start[1:] - cell_start[:-1]).max().item()))
    return cell_start, perm, coord


def gather(perm: torch.Tensor, src3: torch.Tensor, ids: torch.Tensor | None = None,
           stream=None):
    n = perm.shape[0]
    out = torch.empty_like(src3)
    out_ids = torch.empty_like(ids) if ids is not None else None
    _chk(lib().lc_gather(_p(perm), n, _p(src3), _p(out), _p(ids), _p(out_ids),
                         _stream(stream)))
    return out, out_ids


def compute_forces(grid: Grid, sched: Schedule, cell_start, coord, ws: Workspace,
                   precision: str = "fp32", F=None, ew=None, stream=None):
    """One force evaluation.  Returns (F int64 (3, N) cell-sorted, ew int64
    [energy, virial, pairs])."""
    n = coord.shape[1]
    dev = coord.device
    if F is None:
        F = torch.empty((3, n), dtype=torch.int64, device=dev)
    if ew is None:
        ew = torch.empty(3, dtype=torch.int64, device=dev)
    _chk(lib().lc_compute_forces(grid.ptr, sched.ptr, _p(cell_start), _p(coord), n,
                                 _p(F), _p(ew), PREC[precision], ws.ptr,
                                 _stream(stream)))
    return F, ew


def forces_graph(grid: Grid, sched: Schedule, cell_start, coord, ws: Workspace, F, ew,
                 stream, precision: str = "fp32") -> "Graph":
    """Capture one compute_forces evaluation into a HIP graph on `stream`
    (not the null stream); Graph.launch replays it (same buffers, current
    contents)."""
    n = coord.shape[1]
    h = ctypes.c_void_p()
    _chk(lib().lc_forces_graph_create(grid.ptr, sched.ptr, _p(cell_start), _p(coord), n,
                                      _p(F), _p(ew), PREC[precision], ws.ptr,
                                      _stream(stream), ctypes.byref(h)))
    return Graph(h, sched, ws, (grid, cell_start, coord, F, ew))


def compute_forces_noalloc(grid: Grid, sched: Schedule, cell_start, coord, F, ew,
                           precision: str = "fp32", flags=None, stream=None):
    """lc_compute_forces_noalloc: the force evaluation of compute_forces with
    no workspace and no allocation; F (int64 (3, N)) and ew (int64 [3]) are
    caller-given outputs, flags an optional device uint32/int32 [1] that the
    status bits are OR-ed into."""
    n = coord.shape[1]
    _chk(lib().lc_compute_forces_noalloc(grid.ptr, sched.ptr, _p(cell_start), _p(coord), n,
                                         _p(F), _p(ew), PREC[precision],
                                         _p(flags),
                                         _stream(stream)))
    return F, ew


def compute_forces_dataflow(grid: Grid, sched: Schedule, cell_start, coord, ws: Workspace,
                            mode: str = "ordered", F=None, ew=None, limit_ms: float = 2000.0,
                            stream=None, log=None):
    """One force evaluation by a dataflow executor over a creation-order
    schedule (mode: "ordered" = the creation order's dependences, "mutex" =
    per-cell mutual exclusion, "nested" = per-cell chains under mutual
    exclusion).  Every wait is bounded by limit_ms; an expired wait abandons
    the evaluation and sets FLAG_ABORT.  Returns (F, ew) as compute_forces.
    log: an int32 device tensor of 2 x T entries receiving every task's
    start and end tickets (lc_compute_forces_dataflow_log), or None."""
    n = coord.shape[1]
    dev = coord.device
    if F is None:
        F = torch.empty((3, n), dtype=torch.int64, device=dev)
    if ew is None:
        ew = torch.empty(3, dtype=torch.int64, device=dev)
    _chk(lib().lc_compute_forces_dataflow_log(grid.ptr, sched.ptr, DATAFLOW[mode],
                                              _p(cell_start), _p(coord), n, _p(F), _p(ew),
                                              float(limit_ms), _p(log), ws.ptr, _stream(stream)))
    return F, ew


def compute_forces_profiled(grid: Grid, sched: Schedule, cell_start, coord,
                            ws: Workspace, precision: str = "fp32", F=None, ew=None,
                            stream=None):
    """compute_forces with HIP events around every sweep phase and the
    closing launch (synchronises).  Returns (F, ew, sweep_ms, per-phase ms
    list); the list's extra last entry is the closing launch (the gather of
    buffer + reduce, else the energy sums)."""
    import numpy as np
    n = coord.shape[1]
    dev = coord.device
    if F is None:
        F = torch.empty((3, n), dtype=torch.int64, device=dev)
    if ew is None:
        ew = torch.empty(3, dtype=torch.int64, device=dev)
    nphase = sched.info()["nphase"]
    ph = np.zeros(nphase + 1, dtype=np.float64)
    tot = ctypes.c_double(0.0)
    _chk(lib().lc_compute_forces_profiled(grid.ptr, sched.ptr, _p(cell_start), _p(coord), n,
                                          _p(F), _p(ew), PREC[precision], ws.ptr,
                                          _stream(stream), ctypes.byref(tot),
                                          ctypes.c_void_p(ph.ctypes.data)))
    return F, ew, float(tot.value), ph.tolist()


def verlet_step(grid: Grid, sched: Schedule, pos, vel, ids, ws: Workspace,
                dt: float, nsteps: int, rebuild_every: int, F=None,
                cell_start=None, perm=None, coord=None, trace=None, stream=None):
    """nsteps of velocity Verlet; pos/vel/ids are reordered in place into cell
    order.  Returns (trace int64 (nsteps+1, 2) [KE, PE], F)."""
    n = pos.shape[1]
    dev = pos.device
    if F is None:
        F = torch.empty((3, n), dtype=torch.int64, device=dev)
    if cell_start is None:
        cell_start = torch.empty(grid.ncell + 1, dtype=torch.int32, device=dev)
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    if coord is None:
        coord = torch.empty((3, n), dtype=torch.int32, device=dev)
    if trace is None:
        trace = torch.empty((nsteps + 1, 2), dtype=torch.int64, device=dev)
    _chk(lib().lc_verlet_step(grid.ptr, sched.ptr, _p(pos), _p(vel), _p(ids), n,
                              _p(F), _p(cell_start), _p(perm), _p(coord),
                              float(dt), int(nsteps), int(rebuild_every),
                              _p(trace), ws.ptr, _stream(stream)))
    return trace, F


def kinetic_energy(vel: torch.Tensor, ws: Workspace, out=None, stream=None):
    n = vel.shape[1]
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=vel.device)
    _chk(lib().lc_kinetic_energy(_p(vel), n, _p(out), ws.ptr, _stream(stream)))
    return out


RECIP_RANGE = (0x3E800000, 0x43000000)  # bit patterns of 0.25 and 128.0


def selftest_recip(lo_bits: int = RECIP_RANGE[0], hi_bits: int = RECIP_RANGE[1]) -> int:
    """Number of floats with bit patterns in [lo_bits, hi_bits) whose fast
    device reciprocal differs from IEEE division (0 over RECIP_RANGE, the
    range the FP32 sweep relies on)."""
    out = ctypes.c_uint64()
    _chk(lib().lc_selftest_recip(int(lo_bits), int(hi_bits), ctypes.byref(out)))
    return int(out.value)


def serialization_degree_weighted(dims, kind, cell_counts, offsets=None) -> dict:
    """Host-only: critical path with task durations n_A n_B (intra:
    n_A (n_A - 1) / 2) from per-cell particle counts (x fastest)."""
    import numpy as np
    if isinstance(kind, str):
        kind = KINDS[kind]
    d = (ctypes.c_int32 * 3)(*[int(x) for x in dims])
    cc = np.ascontiguousarray(np.asarray(cell_counts, dtype=np.int32))
    if offsets is not None:
        arr = np.ascontiguousarray(np.asarray(offsets, dtype=np.int8).reshape(-1, 3))
        op, n = ctypes.c_void_p(arr.ctypes.data), arr.shape[0]
    else:
        op, n = None, 0
    r = _WSD()
    _chk(lib().lc_serialization_degree_weighted(ctypes.cast(d, P), int(kind), op, int(n),
                                                ctypes.c_void_p(cc.ctypes.data),
                                                ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in _WSD._fields_}


def serialization_degree(dims, kind, offsets=None, hist_len: int = 0) -> dict:
    """Host-only: critical path of a creation order's task DAG (Eq. 1-4)."""
    import numpy as np
    if isinstance(kind, str):
        kind = KINDS[kind]
    d = (ctypes.c_int32 * 3)(*[int(x) for x in dims])
    if offsets is not None:
        arr = np.ascontiguousarray(np.asarray(offsets, dtype=np.int8).reshape(-1, 3))
        op, n = ctypes.c_void_p(arr.ctypes.data), arr.shape[0]
    else:
        op, n = None, 0
    hist = np.zeros(max(hist_len, 0), dtype=np.int64)
    hp = ctypes.c_void_p(hist.ctypes.data) if hist_len > 0 else None
    r = _SD()
    _chk(lib().lc_serialization_degree(ctypes.cast(d, P), int(kind), op, int(n), hp,
                                       int(hist_len), ctypes.byref(r)))
    out = {k: getattr(r, k) for k, _ in _SD._fields_}
    if hist_len > 0:
        out["level_hist"] = hist
    return out


# ---------------------------------------------------------------------------
# batched boxes
# ---------------------------------------------------------------------------

class _BoxDesc(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("n", ctypes.c_int64)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("nbox", ctypes.c_int32), ("nwhole", ctypes.c_int32),
                ("ntot", ctypes.c_int64), ("ncell", ctypes.c_int64),
                ("ngroup", ctypes.c_int64), ("ntask", ctypes.c_int64),
                ("max_replicas", ctypes.c_int32), ("lds_tile", ctypes.c_int32)]


BATCH_MODES = {"auto": 0, "whole": 1, "blocks": 2}
BATCH_WRITE = {"buffer": 0, "atomic": 1}


class _BatchOpts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("write_mode", ctypes.c_int32)]


class Graph:
    """A captured HIP graph of one force evaluation (batched, or of one box
    under a schedule).  It keeps the batch or schedule, the workspace and
    the buffers it was captured with alive (the graph holds their device
    addresses) until it is closed."""

    def __init__(self, handle, batch, ws, buffers):
        self._h = handle
        self._batch, self._ws, self._bufs = batch, ws, buffers
        batch._live_graphs += 1
        ws._live_graphs += 1

    def launch(self, stream=None):
        if not self._h:
            raise LCError(-1, "graph is closed")
        _chk(lib().lc_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().lc_graph_free(self._h)
            self._h = ctypes.c_void_p()
            self._batch._live_graphs -= 1
            self._ws._live_graphs -= 1
            self._batch = self._ws = self._bufs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent periodic boxes evaluated in one launch."""

    def __init__(self, grids, ns, modes=None, tile: int = 0, write: str = "buffer"):
        """tile: LDS tile (particles) the split boxes' blocks are sized for
        (768 = 0 default, 1024, 2048); write: "buffer" (replica slots and a
        gather, Sec. VI strategy 3) or "atomic" (the same groups with global
        atomic write-back, the tile-atomics baseline)."""
        import numpy as np
        self._live_graphs = 0
        nbox = len(grids)
        arr = (_BoxDesc * nbox)()
        for k, (g, n) in enumerate(zip(grids, ns)):
            arr[k].grid = g._g
            arr[k].n = int(n)
        self.grids = list(grids)
        self.ns = [int(n) for n in ns]
        if modes is not None:
            mv = np.ascontiguousarray(
                [BATCH_MODES[m] if isinstance(m, str) else int(m) for m in modes], dtype=np.int32)
            self._modes = mv
            mp = ctypes.c_void_p(mv.ctypes.data)
        else:
            mp = None
        self._h = ctypes.c_void_p()
        opts = _BatchOpts()
        opts.tile = int(tile)
        opts.write_mode = BATCH_WRITE[write]
        _chk(lib().lc_batch_create_ex(ctypes.cast(arr, P), nbox, mp, ctypes.byref(opts),
                                      ctypes.byref(self._h)))

    @property
    def ptr(self):
        return self._h

    def info(self) -> dict:
        i = _BatchInfo()
        _chk(lib().lc_batch_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _BatchInfo._fields_}

    def offsets(self):
        import numpy as np
        nb = len(self.grids)
        ps = np.zeros(nb + 1, dtype=np.int64)
        cs = np.zeros(nb + 1, dtype=np.int64)
        _chk(lib().lc_batch_offsets(self._h, ctypes.c_void_p(ps.ctypes.data),
                                    ctypes.c_void_p(cs.ctypes.data)))
        return ps, cs

    def build_cells(self, pos, ws: Workspace, stream=None):
        info = self.info()
        dev = pos.device
        cs = torch.empty(info["ncell"] + 1, dtype=torch.int32, device=dev)
        perm = torch.empty(info["ntot"], dtype=torch.int32, device=dev)
        coord = torch.empty((3, info["ntot"]), dtype=torch.int32, device=dev)
        _chk(lib().lc_batch_build_cells(self._h, _p(pos), _p(cs), _p(perm), _p(coord), ws.ptr,
                                        _stream(stream)))
        return cs, perm, coord

    def forces(self, cell_start, coord, ws: Workspace, F=None, ew=None, persistent=True,
               stream=None):
        ntot = coord.shape[1]
        dev = coord.device
        if F is None:
            F = torch.empty((3, ntot), dtype=torch.int64, device=dev)
        if ew is None:
            ew = torch.empty((len(self.grids), 3), dtype=torch.int64, device=dev)
        _chk(lib().lc_batch_forces(self._h, _p(cell_start), _p(coord), _p(F), _p(ew),
                                   1 if persistent else 0, ws.ptr, _stream(stream)))
        return F, ew

    def graph(self, cell_start, coord, F, ew, ws: Workspace, stream, persistent=True) -> Graph:
        """Capture forces() into a HIP graph on `stream` (not the null stream)."""
        h = ctypes.c_void_p()
        _chk(lib().lc_batch_graph_create(self._h, _p(cell_start), _p(coord), _p(F), _p(ew),
                                         1 if persistent else 0, ws.ptr, _stream(stream),
                                         ctypes.byref(h)))
        return Graph(h, self, ws, (cell_start, coord, F, ew))

    def close(self):
        if self._live_graphs:
            raise LCError(-7, "the batch is held by a live graph: close the graph first")
        if self._h:
            lib().lc_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
