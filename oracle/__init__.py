"""Link-cell oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, serial reference implementations of everything the link-cell
force sweep and its scheduling analysis compute.  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark use this package; the product
path (the HIP library and its binding) never imports it, and the two share no
code.  The C part lives in ``lc_oracle.c`` (built by ``build.py`` with gcc,
-ffp-contract=off); this module wraps it with ctypes and adds a few numpy
definitions for tiny inputs.

What each function follows (paper: Niethammer, Glass, Gracia, "Avoiding
Serialization Effects in Data / Dependency aware Task Parallel Algorithms for
Spatial Decomposition"):

* forces -- Sec. IV: link-cell method, cells of side >= rc, Newton's third law
  with the half stencils of Fig. 3; a cell-cell interaction updates both
  cells.  The plain definition it must reach is the minimum-image pair sum,
  given here by brute force.  Lennard-Jones details (epsilon = sigma = 1,
  truncated force, energy shifted at rc) are not in the paper; see the
  readings listed in the design notes.
* task orders -- Sec. V (basic order: per cell, intra then inter tasks; cells
  x, then y, then z), Fig. 5 (naive / bad / optimal 2D stencil orders),
  Sec. VI strategy 1 (loop exchange with two-strided colouring, Fig. 6).
* dependency DAG -- Sec. III (dependencies from parameter addresses, tasks in
  creation order) and Sec. V (unit task durations, Eq. 1 S = t_s / t_cp).
* closed forms -- Eq. 2 (stencil speedup), Eq. 3 (its limit), Eq. 4
  (pipeline).
"""
from __future__ import annotations

import ctypes
import math
import os
from collections import defaultdict

import numpy as np

from . import build as _build

_LIB = None

i64 = ctypes.c_int64
i32 = ctypes.c_int32
f64 = ctypes.c_double
P = ctypes.c_void_p


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def lib():
    """Load liblc_oracle.so, compiling it first only if it is absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_canonical.argtypes = [i64, P, P, P]
        L.orc_canonical.restype = None
        L.orc_cell_ids.argtypes = [i64, P, P, P]
        L.orc_cell_ids.restype = None
        L.orc_forces_brute_f64.argtypes = [i64, P, P, P, f64, P, P, P, P]
        L.orc_forces_brute_fx.argtypes = [i64, P, P, f64, P, P, P]
        L.orc_forces_lc_fx.argtypes = [i64, P, P, f64, P, P, ctypes.c_int, P, P, P]
        L.orc_forces_lc_f64.argtypes = [i64, P, P, P, f64, P, P, ctypes.c_int, P, P, P]
        L.orc_forces_loopex_omp.argtypes = [i64, P, P, f64, P, P, ctypes.c_int, ctypes.c_int,
                                            P, P, P, P]
        L.orc_lc_tasks.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_dag_generic.argtypes = [ctypes.c_int, P, P, P, P, P, P]
        L.orc_dag_lc.argtypes = [ctypes.c_int, P, P, P, P]
        L.orc_verlet_fx.argtypes = [i64, P, P, P, f64, P, P, ctypes.c_int, f64,
                                    ctypes.c_int, P, P]
        L.orc_forces_subset_fx.argtypes = [i64, P, P, f64, P, i64, P, P]
        L.orc_dag_lc_weighted.argtypes = [ctypes.c_int, P, P, P, P, P]
        for name in ("orc_forces_brute_f64", "orc_forces_brute_fx",
                     "orc_forces_lc_fx", "orc_forces_lc_f64", "orc_lc_tasks",
                     "orc_dag_generic", "orc_dag_lc", "orc_verlet_fx",
                     "orc_forces_subset_fx", "orc_dag_lc_weighted"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc < 0:
        raise OracleError(f"{what} failed with code {rc}")


# ---------------------------------------------------------------------------
# Stencils and creation orders
# ---------------------------------------------------------------------------

# Fig. 3(a): the 2D half stencil, x to the right, y up: the cell below the
# centre and the three cells of the column to its right.
H2 = [(0, -1, 0), (1, -1, 0), (1, 0, 0), (1, 1, 0)]

# Fig. 3(b), with the drawing's depth/right/up axes read as z/x/y: the whole
# +x layer (9 cells), the three +z cells of the centre layer, and the cell
# below the centre (13 cells).
H3 = ([(1, a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
      + [(0, a, 1) for a in (-1, 0, 1)] + [(0, -1, 0)])

INTRA = (0, 0, 0)

# Fig. 5, cells numbered in evaluation order: (a) naive, (b) bad, (c) optimal.
ORDER2_NAIVE = [INTRA, (0, -1, 0), (1, -1, 0), (1, 0, 0), (1, 1, 0)]
ORDER2_BAD = [INTRA, (0, -1, 0), (1, -1, 0), (1, 1, 0), (1, 0, 0)]
ORDER2_OPT = [(1, 0, 0), (1, -1, 0), (1, 1, 0), (0, -1, 0), INTRA]


def _lex_key(d):
    return (d[2], d[1], d[0])


# 3D orders over H3 (the paper does not print them; readings):
#   lex  -- intra first, then the offsets in ascending (dz, dy, dx) order;
#   opt  -- the x neighbour first, then the other dx = 1 offsets, then the
#           dx = 0 offsets, intra last (the x-neighbour-first rule of Sec. V);
#   best -- intra first, then the x neighbour, then as opt;
#   bad  -- intra first, the x neighbour last.
_H3_LEX = sorted(H3, key=_lex_key)
ORDER3_LEX = [INTRA] + _H3_LEX
_EX = (1, 0, 0)
_DX1 = [d for d in _H3_LEX if d[0] == 1 and d != _EX]
_DX0 = [d for d in _H3_LEX if d[0] == 0]
ORDER3_OPT = [_EX] + _DX1 + _DX0 + [INTRA]
ORDER3_BEST = [INTRA, _EX] + _DX1 + _DX0
ORDER3_BAD = [INTRA] + [d for d in _H3_LEX if d != _EX] + [_EX]


def offsets_array(order) -> np.ndarray:
    return np.ascontiguousarray(np.array(order, dtype=np.int8).reshape(-1, 3))


# ---------------------------------------------------------------------------
# Coordinates and cells
# ---------------------------------------------------------------------------

CELL_MARGIN = 1.0 + 1.0 / 4096.0


def canonical(pos: np.ndarray, L) -> np.ndarray:
    """uint32 box fractions u = floor(x / L * 2^32) mod 2^32, shape (3, N)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    u = np.empty((3, n), dtype=np.uint32)
    lib().orc_canonical(n, _ptr(pos), _ptr(Lv), _ptr(u))
    return u


def grid_dims(L, rc: float, skin: float = 0.0, even: bool = False):
    """Largest cell count per axis whose cell side is >= (rc + skin) with the
    FP32 safety margin; rounded down to even when ``even``."""
    out = []
    for Ld in np.asarray(L, dtype=np.float64).reshape(3):
        n = int(math.floor(Ld / (rc * CELL_MARGIN + skin)))
        if even and n % 2:
            n -= 1
        out.append(n)
    return np.array(out, dtype=np.int32)


def cell_ids(u: np.ndarray, nc) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.uint32)
    n = u.shape[1]
    ncv = np.ascontiguousarray(np.asarray(nc, dtype=np.int32).reshape(3))
    cid = np.empty(n, dtype=np.int32)
    lib().orc_cell_ids(n, _ptr(u), _ptr(ncv), _ptr(cid))
    return cid


def cell_start(u: np.ndarray, nc) -> np.ndarray:
    """Exclusive prefix sum of per-cell particle counts, length ncell + 1."""
    cid = cell_ids(u, nc)
    ncell = int(np.prod(np.asarray(nc, dtype=np.int64)))
    counts = np.bincount(cid, minlength=ncell).astype(np.int64)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)


# ---------------------------------------------------------------------------
# Forces
# ---------------------------------------------------------------------------

SCALE = 2.0 ** 32


def forces_brute_f64(pos, L, rc, u=None):
    """FP64 O(N^2) minimum-image Lennard-Jones sum.

    Returns (F (3,N), mag (N,) = sum_j |f_ij|, U, W, npairs).  With ``u``
    (canonical coordinates) the cutoff test is the canonical FP32 one."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    F = np.empty((3, n))
    mag = np.empty(n)
    ew = np.empty(2)
    np_ = ctypes.c_int64(0)
    uu = np.ascontiguousarray(u, dtype=np.uint32) if u is not None else None
    up = _ptr(uu) if uu is not None else None
    _check(lib().orc_forces_brute_f64(n, _ptr(pos), up, _ptr(Lv), rc, _ptr(F),
                                      _ptr(mag), _ptr(ew), ctypes.byref(np_)),
           "forces_brute_f64")
    return F, mag, float(ew[0]), float(ew[1]), int(np_.value)


def forces_brute_fx(u, L, rc):
    """Fixed-point O(N^2): canonical FP32 pair terms, int64 sums at 2^32.

    Returns (F int64 (3,N), E int64, W int64, npairs)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    n = u.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    F = np.empty((3, n), dtype=np.int64)
    ew = np.empty(2, dtype=np.int64)
    np_ = ctypes.c_int64(0)
    _check(lib().orc_forces_brute_fx(n, _ptr(u), _ptr(Lv), rc, _ptr(F),
                                     _ptr(ew), ctypes.byref(np_)),
           "forces_brute_fx")
    return F, int(ew[0]), int(ew[1]), int(np_.value)


def forces_lc_fx(u, L, rc, nc, stencil=H3):
    """Fixed-point serial link-cell sweep (half stencil, Newton's third law)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    n = u.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    ncv = np.ascontiguousarray(np.asarray(nc, dtype=np.int32).reshape(3))
    offs = offsets_array(stencil)
    F = np.empty((3, n), dtype=np.int64)
    ew = np.empty(2, dtype=np.int64)
    np_ = ctypes.c_int64(0)
    _check(lib().orc_forces_lc_fx(n, _ptr(u), _ptr(Lv), rc, _ptr(ncv),
                                  _ptr(offs), len(offs), _ptr(F), _ptr(ew),
                                  ctypes.byref(np_)), "forces_lc_fx")
    return F, int(ew[0]), int(ew[1]), int(np_.value)


def forces_loopex_omp(u, L, rc, nc, stencil=H3, threads=0):
    """The fixed-point link-cell sweep in the loop-exchange order with
    two-strided colouring (Sec. VI, strategy 1), parallel over the cells of
    each colour with OpenMP; needs even cell counts.  Same bits as
    forces_lc_fx.  threads <= 0: OpenMP's default.

    Returns (F, E, W, npairs, threads_used)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    n = u.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    ncv = np.ascontiguousarray(np.asarray(nc, dtype=np.int32).reshape(3))
    offs = offsets_array(stencil)
    F = np.empty((3, n), dtype=np.int64)
    ew = np.empty(2, dtype=np.int64)
    np_ = ctypes.c_int64(0)
    used = ctypes.c_int(0)
    _check(lib().orc_forces_loopex_omp(n, _ptr(u), _ptr(Lv), rc, _ptr(ncv), _ptr(offs),
                                       len(offs), int(threads), _ptr(F), _ptr(ew),
                                       ctypes.byref(np_), ctypes.byref(used)),
           "forces_loopex_omp")
    return F, int(ew[0]), int(ew[1]), int(np_.value), int(used.value)


def forces_lc_f64(pos, u, L, rc, nc, stencil=H3):
    """FP64 serial link-cell sweep; cells from the canonical coordinates."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.uint32)
    n = pos.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    ncv = np.ascontiguousarray(np.asarray(nc, dtype=np.int32).reshape(3))
    offs = offsets_array(stencil)
    F = np.empty((3, n))
    ew = np.empty(2)
    np_ = ctypes.c_int64(0)
    _check(lib().orc_forces_lc_f64(n, _ptr(pos), _ptr(u), _ptr(Lv), rc,
                                   _ptr(ncv), _ptr(offs), len(offs), _ptr(F),
                                   _ptr(ew), ctypes.byref(np_)), "forces_lc_f64")
    return F, float(ew[0]), float(ew[1]), int(np_.value)


def forces_subset_fx(u, L, rc, idx):
    """Fixed-point force on the particles ``idx`` by brute force over all
    others (O(N) each): returns (F int64 (3, m), neighbours per particle)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    n = u.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    m = len(idx)
    F = np.empty((3, m), dtype=np.int64)
    npair = np.empty(m, dtype=np.int64)
    _check(lib().orc_forces_subset_fx(n, _ptr(u), _ptr(Lv), rc, _ptr(idx), m, _ptr(F),
                                      _ptr(npair)), "forces_subset_fx")
    return F, npair


def brute_numpy_f64(pos, L, rc):
    """The plain definition in numpy (tiny N only): every ordered pair,
    minimum image, F_i = sum_j 24 (2 r^-12 - r^-6) / r^2 * (r_i - r_j),
    U = sum_{i<j} 4 (r^-12 - r^-6) - 4 (rc^-12 - rc^-6)."""
    x = np.asarray(pos, dtype=np.float64).T  # (N, 3)
    Lv = np.asarray(L, dtype=np.float64).reshape(1, 1, 3)
    d = x[:, None, :] - x[None, :, :]  # r_i - r_j
    d -= Lv * np.round(d / Lv)
    r2 = np.sum(d * d, axis=2)
    n = x.shape[0]
    mask = (r2 < rc * rc) & ~np.eye(n, dtype=bool)
    r2s = np.where(mask, r2, 1.0)
    sr6 = r2s ** -3
    fs = np.where(mask, 24.0 * (2.0 * sr6 * sr6 - sr6) / r2s, 0.0)
    F = np.sum(fs[:, :, None] * d, axis=1).T
    uc = 4.0 * (rc ** -12 - rc ** -6)
    U = 0.5 * np.sum(np.where(mask, 4.0 * (sr6 * sr6 - sr6) - uc, 0.0))
    return F, float(U), int(np.sum(mask) // 2)


def lj_pair_force_magnitude(r: float) -> float:
    """|F| of one Lennard-Jones pair at distance r: 24 (2 r^-13 - r^-7)."""
    return 24.0 * (2.0 * r ** -13 - r ** -7)


# ---------------------------------------------------------------------------
# Task orders, dependency DAG, critical path
# ---------------------------------------------------------------------------

def lc_tasks(dims, order, loopex: bool = False):
    """Cell-pair tasks (cellA, cellB) in creation order (see lc_oracle.c)."""
    dimsv = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(3))
    offs = offsets_array(order)
    T = int(np.prod(dimsv.astype(np.int64))) * len(offs)
    A = np.empty(T, dtype=np.int32)
    B = np.empty(T, dtype=np.int32)
    got = lib().orc_lc_tasks(_ptr(dimsv), _ptr(offs), len(offs), int(loopex),
                             _ptr(A), _ptr(B))
    _check(got, "lc_tasks")
    assert got == T
    return A, B


def dag_lc(A, B):
    """Depth of every task and the critical path, by the definition."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    depth = np.empty(len(A), dtype=np.int32)
    cp = ctypes.c_int32(0)
    _check(lib().orc_dag_lc(len(A), _ptr(A), _ptr(B), _ptr(depth),
                            ctypes.byref(cp)), "dag_lc")
    return depth, int(cp.value)


def dag_lc_weighted(A, B, w):
    """Weighted critical path by the definition (every earlier task that
    shares a cell must finish first).  Returns (finish times, cp)."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    fin = np.empty(len(A))
    cp = ctypes.c_double(0.0)
    _check(lib().orc_dag_lc_weighted(len(A), _ptr(A), _ptr(B), _ptr(w), _ptr(fin),
                                     ctypes.byref(cp)), "dag_lc_weighted")
    return fin, float(cp.value)


IN, OUT, INOUT = 0, 1, 2


def dag_generic(tasks):
    """``tasks``: list of parameter lists [(address, mode), ...] in creation
    order, mode in {IN, OUT, INOUT}.  Returns (depth, pred, cp)."""
    pstart = np.zeros(len(tasks) + 1, dtype=np.int32)
    addr, mode = [], []
    for t, params in enumerate(tasks):
        for a, m in params:
            addr.append(a)
            mode.append(m)
        pstart[t + 1] = len(addr)
    addr = np.ascontiguousarray(np.array(addr, dtype=np.int64))
    mode = np.ascontiguousarray(np.array(mode, dtype=np.int32))
    depth = np.empty(len(tasks), dtype=np.int32)
    pred = np.empty(len(tasks), dtype=np.int32)
    cp = ctypes.c_int32(0)
    _check(lib().orc_dag_generic(len(tasks), _ptr(pstart), _ptr(addr),
                                 _ptr(mode), _ptr(depth), _ptr(pred),
                                 ctypes.byref(cp)), "dag_generic")
    return depth, pred, int(cp.value)


def asap_steps(A, B):
    """Critical path by simulation: unbounded workers, unit-time tasks; at
    every step run each not-yet-run task all of whose earlier tasks on each
    of its cells have finished.  A second, independent algorithm for the
    same number (tiny grids only: O(T * CP))."""
    T = len(A)
    touching = defaultdict(list)  # cell -> tasks touching it, creation order
    cells_of = []
    for t in range(T):
        cs = sorted({int(A[t]), int(B[t])})
        cells_of.append(cs)
        for c in cs:
            touching[c].append(t)
    first = {c: 0 for c in touching}  # first unfinished task on each cell
    done = np.zeros(T, dtype=bool)
    steps, remaining = 0, T
    while remaining:
        ready = [t for t in range(T) if not done[t]
                 and all(touching[c][first[c]] == t for c in cells_of[t])]
        assert ready, "no task ready: the order is not a DAG"
        for t in ready:
            done[t] = True
        remaining -= len(ready)
        for c, lst in touching.items():
            while first[c] < len(lst) and done[lst[first[c]]]:
                first[c] += 1
        steps += 1
    return steps


def serialization_degree(dims, order, loopex: bool = False):
    """T, critical path, S = T / CP (Eq. 1 with unit tasks), CP / T."""
    A, B = lc_tasks(dims, order, loopex)
    _, cp = dag_lc(A, B)
    T = len(A)
    return {"T": T, "cp": cp, "S": T / cp, "degree": cp / T}


def speedup_eq2(delta: float, k: int, n: int) -> float:
    """Eq. 2: S(Delta, k, n) = n k / (n + Delta (k - 1))."""
    return n * k / (n + delta * (k - 1))


def smax_eq3(delta: float, n: int) -> float:
    """Eq. 3: the k -> infinity limit n / Delta."""
    return n / delta


def pipeline_eq4(n: int, k: int) -> float:
    """Eq. 4: pipeline speedup n k / (n + k - 1)."""
    return n * k / (n + k - 1)


# ---------------------------------------------------------------------------
# Velocity Verlet
# ---------------------------------------------------------------------------

def verlet_fx(pos, vel, L, rc, dt, nsteps, nc=None, stencil=H3):
    """Kick-drift-kick Verlet, FP64 state, fixed-point forces (see C).

    Returns (pos, vel, F, trace) with trace (nsteps+1, 2) int64 [KE, PE] in
    units of 2^-32."""
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    vel = np.array(vel, dtype=np.float64, order="C", copy=True)
    n = pos.shape[1]
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(3))
    if nc is None:
        nc = grid_dims(Lv, rc)
    ncv = np.ascontiguousarray(np.asarray(nc, dtype=np.int32).reshape(3))
    offs = offsets_array(stencil)
    F = np.empty((3, n), dtype=np.int64)
    trace = np.empty((nsteps + 1, 2), dtype=np.int64)
    _check(lib().orc_verlet_fx(n, _ptr(pos), _ptr(vel), _ptr(Lv), rc,
                               _ptr(ncv), _ptr(offs), len(offs), dt, nsteps,
                               _ptr(F), _ptr(trace)), "verlet_fx")
    return pos, vel, F, trace
