"""Benchmark of the link-cell force sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload fcc256k]

A step is one whole force evaluation (lc_compute_forces under the fastest
conflict-free configuration -- BLOCK8 colouring or BUFFER buffer+reduce, with
the cell grid and block shape the autotuner picks, all named in the output)
over a 256,000-particle Lennard-Jones FCC crystal at density 0.8 with
rc = 2.5 in a periodic cube (26^3 or 27^3 cells), cells prebuilt and all
inputs resident in HBM.
Prints ONE JSON line: pair interactions per second (pairs inside the cutoff
evaluated per second), the roofline of the dominant kernel (the tile sweep,
bound by vector ALU work), the same evaluation under the atomics baselines
and the paper's creation orders, and the serial CPU oracle timed on the
host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Vector-ALU peak of MI355X without packed FP32: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz lane-operations per second.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU work of the sweep: per candidate pair (separation from box
# fractions, r^2, cutoff test) and per pair inside the cutoff (division, LJ
# terms, five quantisations, six int64 accumulations, energy/virial).
OPS_PER_CANDIDATE = 10
OPS_PER_PAIR = 50

WORKLOADS = {
    "fcc256k": dict(n=256000, rho=0.8, rc=2.5, seed=1002,
                    desc="LJ FCC+jitter N=256000 rho=0.8 rc=2.5 periodic cube"),
    "fcc4k": dict(n=4000, rho=0.8, rc=2.5, seed=1001,
                  desc="LJ FCC+jitter N=4000 rho=0.8 rc=2.5 periodic cube"),
    "fcc4m": dict(n=4_000_000, rho=0.8, rc=2.5, seed=1003,
                  desc="LJ FCC+jitter N=4000000 rho=0.8 rc=2.5 periodic cube"),
}
EXTRA_WORKLOADS = ("fcc4m_md", "slab2m", "boxes512", "lj2d_1m")

H3 = ([(1, a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
      + [(0, a, 1) for a in (-1, 0, 1)] + [(0, -1, 0)])


def source_hash() -> str:
    """sha256 over the HIP library sources: identifies the kernel build."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1401_4441_amd", "csrc")
    for name in ("lc.hip", "lc_sched.cpp", "lc_sched.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_prefix: str, workload: str, config: dict):
    """HBM bytes per launch of the kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when
    the kernel sources or the configuration (schedule, cells, block shape)
    differ from the ones the counters were taken on."""
    path = os.path.join(ROOT, "profiles", f"k_sweep_{workload}_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != source_hash():
        return None
    for entry in d.get("configs", []):
        if entry.get("config") == config:
            k = entry.get("kernels", {}).get(kernel_prefix)
            return None if k is None else k["bytes_per_launch"]
    return None


def half_shell(reach: int):
    """Half shell of a stencil reaching `reach` cells: the offsets with
    dx > 0, or dx = 0 and dz > 0, or dx = dz = 0 and dy < 0 (13 at reach 1,
    62 at reach 2)."""
    if reach == 1:
        return H3
    r = range(-reach, reach + 1)
    return [(x, y, z) for z in r for y in r for x in r
            if x > 0 or (x == 0 and z > 0) or (x == 0 and z == 0 and y < 0)]


def candidate_pairs(cell_start: np.ndarray, nc, reach: int = 1) -> int:
    """Candidate pairs the half-stencil sweep visits: n_c(n_c-1)/2 per cell
    plus n_c * n_{c+d} per cell and half-stencil offset d."""
    cnt = np.diff(cell_start.astype(np.int64)).reshape(nc[2], nc[1], nc[0])
    total = int(np.sum(cnt * (cnt - 1) // 2))
    for dx, dy, dz in half_shell(reach):
        nb = np.roll(cnt, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        total += int(np.sum(cnt * nb))
    return total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fcc256k",
                    choices=sorted(WORKLOADS) + list(EXTRA_WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the baseline schedules (atomics, paper orders)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other evaluated configurations (4M MD, 512 boxes, 2M "
                         "slab) that the default run adds under 'workloads'")
    ap.add_argument("--schedule", choices=("block8", "buffer"),
                    help="fix the headline schedule instead of autotuning (with --block and "
                         "--grid; used to profile one configuration)")
    ap.add_argument("--block", default=None, help="block shape X,Y,Z for --schedule")
    ap.add_argument("--load-aware", action="store_true",
                    help="with --schedule: launch the groups heaviest first by the input's "
                         "cell counts")
    ap.add_argument("--grid", default="natural", choices=("even", "natural", "wide", "half"),
                    help="cell grid for --schedule: even counts, natural (side >= rc), "
                         "or widened 15%% with even counts")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 64 MiB device copy three times (the reference "
                         "that scales rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(64 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; "
                          "--gpus must be 1 (multi-GPU sharding is design-only)"}))
        sys.exit(2)

    import torch
    from paper_1401_4441_amd import autotune, lc, synth

    if args.workload == "fcc4m_md":
        return bench_md(args)
    if args.workload == "slab2m":
        return bench_slab(args)
    if args.workload == "boxes512":
        return bench_boxes(args)
    if args.workload == "lj2d_1m":
        return bench_2d(args)
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    box = synth.fcc(w["n"], w["rho"], rc=w["rc"], seed=w["seed"])
    pos = torch.from_numpy(box.pos).to(dev)

    # ---- pick the configuration: the autotuner times every cell grid x
    # schedule kind x block shape (conflict-free kinds, and ATOMIC_TILE for
    # the baseline table); the fastest conflict-free one is the headline
    if args.schedule:
        gopt = {"even": {"extra": 0.0, "even": True}, "natural": {"extra": 0.0, "even": False},
                "wide": {"extra": 0.15, "even": True},
                "half": {"extra": 0.0, "even": False, "half": True}}[args.grid]
        blk0 = [int(x) for x in args.block.split(",")] if args.block else [1, 2, 2]
        pick = {"kind": args.schedule, "block": blk0, "grid": gopt}
        tune = {"trials": [dict(pick, nc=[0, 0, 0], ms=0.0, fallback=False)]}
        load_aware = args.load_aware
    else:
        tune = autotune.tune_box(pos, box.L, box.rc, reps=10, use_cache=False,
                                 kinds=("block8", "buffer", "atomic_tile", "fullshell"))
        cf = [t for t in tune["trials"]
              if t["kind"] in autotune.BOX_KINDS_CONFLICT_FREE and not t["fallback"]]
        pick = min(cf, key=lambda t: t["ms"])
        load_aware = None  # decided below by timing both launch orders
    g = autotune.make_grid(box.L, box.rc, pick["grid"])
    ws = lc.Workspace(box.n, g.ncell)
    cs, perm, coord = lc.build_cells(g, pos, ws)
    counts = lc.cell_counts_of(cs)

    def best_block(kind):
        on_grid = [t for t in tune["trials"]
                   if t["kind"] == kind and t["grid"] == pick["grid"] and not t.get("fallback")]
        return tuple(min(on_grid, key=lambda t: t["ms"])["block"]) if on_grid else None
    torch.cuda.synchronize()
    ncand = candidate_pairs(cs.cpu().numpy(), g.nc, g.reach)
    F = torch.empty((3, box.n), dtype=torch.int64, device=dev)
    ew = torch.empty(3, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def time_sched(kind, steps, warmup, block=None, weighted=False):
        s = lc.Schedule(g, kind, block=block, cell_counts=counts if weighted else None)
        for _ in range(warmup):
            lc.compute_forces(g, s, cs, coord, ws, "fp32", F, ew)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        t0 = time.perf_counter()
        for _ in range(steps):
            lc.compute_forces(g, s, cs, coord, ws, "fp32", F, ew)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / steps
        return s, ms, wall

    best, blk = pick["kind"], tuple(pick["block"])
    order_trials = None
    if load_aware is None:
        # the autotuner's three fastest conflict-free shapes on the picked
        # grid, each with its groups launched in the fixed order or heaviest
        # first by this input's cell counts (the schedule is built before the
        # timed region, like the autotuner's pick); the fastest combination
        # is the headline
        cands = sorted((t for t in cf if t["grid"] == pick["grid"]), key=lambda t: t["ms"])[:3]
        order_trials = []
        for t in cands:
            for w_ in (False, True):
                ms_ = []
                for _ in range(3):
                    s_, m_, _ = time_sched(t["kind"], 20, 3, tuple(t["block"]), weighted=w_)
                    s_.close()
                    ms_.append(m_)
                order_trials.append({"kind": t["kind"], "block": list(t["block"]),
                                     "load_aware": w_, "ms": statistics.median(ms_)})
        top = min(order_trials, key=lambda r: r["ms"])
        best, blk, load_aware = top["kind"], tuple(top["block"]), top["load_aware"]

    # ---- the timed region: K evaluations under that schedule
    ws.clear_status()
    sched, ms, wall = time_sched(best, args.steps, args.warmup, blk, weighted=load_aware)
    pairs = int(ew[2].item())
    status = ws.status()
    value = pairs / (ms * 1e-3)

    # ---- the 1e-5 gate: FP32 pair math (int64 sums) against FP64 pair
    # arithmetic on the same box fractions and pair set
    F64, ew64 = lc.compute_forces(g, sched, cs, coord, ws, "fp64")
    F32, ew32 = lc.compute_forces(g, sched, cs, coord, ws, "fp32")
    d = (F32 - F64).double()
    err_norm = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(F64.double()))
    err_energy = abs(int(ew32[0]) - int(ew64[0])) / abs(int(ew64[0]))

    # ---- dominant kernel: the sweep phases, HIP events around each launch
    sweep_ms, close_ms = [], []
    for _ in range(5):
        _, _, tot, per_phase = lc.compute_forces_profiled(g, sched, cs, coord, ws, "fp32", F, ew)
        sweep_ms.append(tot)
        close_ms.append(per_phase[-1])
    sweep_ms = statistics.median(sweep_ms)
    close_ms = statistics.median(close_ms)
    nphase = sched.info()["nphase"]
    ops = OPS_PER_CANDIDATE * ncand + OPS_PER_PAIR * pairs
    achieved_tops = ops / (sweep_ms * 1e-3) / 1e12
    # algorithmic HBM bytes of one evaluation: coords (12 B) + force write
    # (24 B) per particle, cell table
    alg_bytes = box.n * (12 + 24) + (g.ncell + 1) * 4
    hbm_gbs = alg_bytes / (sweep_ms * 1e-3) / 1e9

    out = {
        "metric": "pair interactions/sec (LJ cell-pair force sweep, Newton-3, conflict-free schedule)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair math, int64 fixed-point accumulation",
        "data": "synthetic (seeded FCC lattice + uniform jitter)",
        "config": {"workload": w["desc"], "n": box.n, "cells": list(g.nc),
                   "schedule": best, "block": list(blk), "grid_choice": pick["grid"],
                   "load_aware": load_aware, "launch_order_trials": order_trials,
                   "autotune_trials": [[t["kind"], t["nc"][0], t["block"], round(t["ms"], 4)]
                                       for t in tune["trials"]],
                   "pairs_in_cutoff": pairs,
                   "candidate_pairs": ncand, "status_flags": status},
        "accuracy": {"force_normwise_rel_err_vs_fp64": err_norm,
                     "energy_rel_err_vs_fp64": err_energy, "gate": 1e-5,
                     "pass": err_norm <= 1e-5 and err_energy <= 1e-5},
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tops,
            "peak": VALU_PEAK_TOPS,
            "unit": "Tops/s (VALU lane-ops)",
            "frac": achieved_tops / VALU_PEAK_TOPS,
            "traffic": measured_traffic(f"k_sweep_wmode{sched.info()['write_mode']}", args.workload,
                                        {"kind": best, "nc": list(g.nc), "block": list(blk),
                                         "load_aware": load_aware}),
            "traffic_source": f"profiles/k_sweep_{args.workload}_traffic.json (rocprofv3 --pmc "
                              "FETCH_SIZE / WRITE_SIZE, scaled by a 64 MiB copy); null if the "
                              "kernel changed since",
            "source_sha256": source_hash(),
            "kernel": "k_sweep",
            "kernel_ms_per_step": sweep_ms,
            "launches_per_step": nphase,
            "work_per_step": {"candidates": ncand, "pairs": pairs, "lane_ops": ops},
            "hbm_algorithmic_GBps": hbm_gbs,
            "hbm_frac": hbm_gbs / HBM_PEAK_GBS,
        },
        "wall_s_timed": wall,
    }

    # ---- buffer + reduce: the gather that closes the evaluation is HBM-bound;
    # per particle it reads its cell's R_c replica slots (24 B each) and the
    # replica count (4 B) and writes the force (24 B)
    if sched.info()["write_mode"] == 3:
        nc_cells = np.diff(cs.cpu().numpy().astype(np.int64))
        reps = sched.cell_footprints().astype(np.int64)
        gbytes = int(np.sum(nc_cells * (24 * reps + 28)))
        out["gather"] = {"kernel": "k_gather_partials", "ms": close_ms,
                         "algorithmic_bytes": gbytes,
                         "mean_replicas": float(np.sum(nc_cells * reps) / box.n),
                         "GBps": gbytes / (close_ms * 1e-3) / 1e9,
                         "hbm_frac": gbytes / (close_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # ---- the cell build (a1) alone and the evaluation with it, candidate rate
    copy_gbs = copy_bandwidth_gbs()
    out["cell_build"] = cell_build_stats(lc, g, pos, ws, copy_gbs)
    cs_b = torch.empty_like(cs)
    perm_b = torch.empty_like(perm)
    coord_b = torch.empty_like(coord)

    def build_and_eval():
        lc.build_cells(g, pos, ws, cs_b, perm_b, coord_b, tile_hint=False)
        lc.compute_forces(g, sched, cs_b, coord_b, ws, "fp32", F, ew)
    ms_wb = statistics.median(_time_evals(build_and_eval, 20, 3) for _ in range(3))
    out["with_cell_build"] = {"ms_per_step": ms_wb, "pairs_per_s": pairs / (ms_wb * 1e-3)}
    out["candidate_pairs_per_s"] = ncand / (ms * 1e-3)

    # ---- baselines: same evaluation under the other schedules
    if not args.no_extra:
        extra = {}
        for kind, st, wu in (("block8", 20, 3), ("buffer", 20, 3), ("atomic_tile", 20, 3),
                             ("fullshell", 20, 3), ("atomic_pair", 20, 3), ("loopex", 10, 2),
                             ("opt", 2, 1), ("lex", 1, 1)):
            kb = best_block(kind)
            if g.reach == 2 and kind in ("loopex", "opt", "lex"):
                extra[kind] = {"skipped": "creation orders are timed on the rc-cell grid "
                                          "(paper_strategies)"}
                continue
            try:
                # the tile kinds launch their groups in the headline's order
                # (fixed or heaviest first), so that only the write-back and
                # the phase count differ
                tiled = kind in ("block8", "buffer", "atomic_tile", "fullshell", "atomic_pair")
                s, kms, _ = time_sched(kind, st, wu, kb, weighted=bool(load_aware) and tiled)
            except lc.LCError as e:  # loop exchange needs even cell counts
                extra[kind] = {"skipped": str(e)}
                continue
            extra[kind] = {"ms_per_step": kms, "pairs_per_s": pairs / (kms * 1e-3),
                           "phases": s.info()["nphase"], "block": list(kb) if kb else None,
                           "load_aware": bool(load_aware) and tiled,
                           "time_vs_headline": kms / ms,
                           # every schedule must give the headline's bits
                           # (forces, energy, virial, pair count)
                           "same_bits_as_headline": bool(torch.equal(F, F32)
                                                         and torch.equal(ew, ew32))}
            s.close()
        out["schedules"] = extra
        out["conflict_free_vs_atomics"] = {
            "speedup_over_atomic_pair": extra["atomic_pair"]["ms_per_step"] / ms,
            "speedup_over_atomic_tile": extra["atomic_tile"]["ms_per_step"] / ms,
            # the same conflict-free sweep without Newton's third law: every
            # pair evaluated twice, no write sharing at all
            "speedup_over_full_shell": extra["fullshell"]["ms_per_step"] / ms,
            # the plain atomics against the 8-colour block sweep (both pass
            # the accuracy gate: they give the same bits)
            "atomic_pair_over_block8": extra["atomic_pair"]["ms_per_step"]
            / extra["block8"]["ms_per_step"],
            # the fair baseline is the same tile code with atomic write-back
            # in one phase (atomic_tile); the per-pair atomics are reported
            # beside it
            "target": ">= 3x faster than the tile-atomics baseline (atomic_tile: same tile "
                      "code, one phase, global atomic write-back)",
            "target_met": extra["atomic_tile"]["ms_per_step"] / ms >= 3.0,
            "block8_over_atomic_tile_time": extra["block8"]["ms_per_step"]
            / extra["atomic_tile"]["ms_per_step"]}
        # the paper's serialisation degree on this grid (host computation)
        sdo = {}
        for k in ("lex", "opt", "best", "bad", "loopex"):
            try:
                v = lc.serialization_degree(g.nc, k)
            except lc.LCError as e:  # loop exchange needs even cell counts
                sdo[k] = {"skipped": str(e)}
                continue
            sdo[k] = {"cp": v["cp"], "S": v["speedup"], "delta": v["delta"], "S_eq2": v["s_eq2"]}
        out["serialization_degree"] = sdo
        out["paper_strategies"] = paper_strategies(box, pos)
        # What the paper itself reports (it prints no throughput, only the
        # speedup limits of its stencil orders, Sec. V, Eq. 3-4 and Fig. 5,
        # and qualitative agreement of its measurements, Sec. VII, whose
        # plots are not in the text), with the hardware it names.
        out["paper_reported"] = {
            "S_max": {"2d_naive": 1.25, "2d_bad": 1.0, "2d_opt": 5.0,
                      "3d_best_basic": 7.0, "3d_opt": 14.0},
            "measurements": "basic order vs Eq. 2 'excellent agreement' on one Laki node "
                            "(NEC, dual-socket Xeon X5560, 8 cores, SMPSs 2.4); bad/opt orders "
                            "'perfect agreement', loop exchange 'perfect scaling up to 32 "
                            "threads', nested tasks 'nearly perfect' to 23 threads on one "
                            "Hermit node (Cray XE6, dual-socket Opteron 6276, 32 cores, OmpSs); "
                            "2D 50x50 and 3D 30x10x10 cell domains, 5-10 ms synthetic tasks",
            "this_device": {k: v.get("S") for k, v in sdo.items() if "S" in v}}

    # ---- CPU baseline: the serial oracle on the host (rank 0, N=1 only)
    if not args.no_cpu:
        import oracle as O
        u = O.canonical(box.pos, box.L)
        times = []
        t_begin = time.perf_counter()
        while len(times) < 5 and (time.perf_counter() - t_begin) < 20.0:
            t0 = time.perf_counter()
            _, _, _, npo = O.forces_lc_fx(u, box.L, box.rc, O.grid_dims(box.L, box.rc))
            times.append(time.perf_counter() - t0)
        t = statistics.median(times)
        out["cpu_baseline"] = {
            "value": npo / t, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} full serial fixed-point link-cell evaluations of the "
                      f"same {box.n}-particle box (median {t:.3f} s each)"}
        # the headline's FP32 forces against the FP64 serial link-cell oracle
        # (FP64 arithmetic and the FP64 cutoff test, cells from the same box
        # fractions); pairs within an FP32 ulp of the cutoff may be in one
        # pair set and not the other
        F64o, U64o, W64o, np64o = O.forces_lc_f64(box.pos, u, box.L, box.rc,
                                                  O.grid_dims(box.L, box.rc))
        Fin = np.empty((3, box.n))
        Fin[:, perm.cpu().numpy()] = F32.double().cpu().numpy() / 2.0 ** 32
        out["cpu_baseline"]["fp64_oracle_check"] = {
            "force_normwise_rel_err": float(np.linalg.norm(Fin - F64o) / np.linalg.norm(F64o)),
            "energy_rel_err": abs(int(ew32[0]) / 2.0 ** 32 - U64o) / abs(U64o),
            "virial_rel_err": abs(int(ew32[1]) / 2.0 ** 32 - W64o) / abs(W64o),
            "pairs_fp32_cutoff": int(ew32[2]), "pairs_fp64_cutoff": np64o,
            "gate": 1e-5}
        # the paper's own CPU scheme beside it: the same sweep in the
        # loop-exchange order with two-strided colouring, parallel over each
        # colour's cells with OpenMP on the host's threads (even cell counts)
        nce = O.grid_dims(box.L, box.rc, even=True)
        ptimes, used = [], 0
        t_begin = time.perf_counter()
        while len(ptimes) < 5 and (time.perf_counter() - t_begin) < 10.0:
            t0 = time.perf_counter()
            _, _, _, npp, used = O.forces_loopex_omp(u, box.L, box.rc, nce)
            ptimes.append(time.perf_counter() - t0)
        tp = statistics.median(ptimes)
        out["cpu_parallel_reference"] = {
            "value": npp / tp, "unit": "pairs/s", "cores": used,
            "kind": "oracle, loop exchange + 2x2x2 colouring (Sec. VI), OpenMP",
            "sample": f"{len(ptimes)} full evaluations of the same box on "
                      f"{'x'.join(map(str, nce))} cells (median {tp:.3f} s each)",
            "cpu_model": cpu_model()}

    # ---- the other evaluated configurations, each measured in this run
    if not args.no_workloads and args.workload == "fcc256k" and not args.schedule:
        out["workloads"] = {}
        for name, fn in (("fcc4m_md", bench_md), ("boxes512", bench_boxes),
                         ("slab2m", bench_slab)):
            torch.cuda.empty_cache()
            t0 = time.perf_counter()
            print(f"workload {name}", file=sys.stderr, flush=True)
            r = fn(args, emit=False)
            r["wall_s"] = time.perf_counter() - t0
            out["workloads"][name] = r
    print(json.dumps(out), flush=True)


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def paper_strategies(box, pos):
    """The paper's comparison on the device, on the even grid (loop exchange
    needs even cell counts): every creation order (bad, lex = the standard
    order, opt, loop exchange) with its exact critical path, run (a) as one
    launch per DAG level and (b) as one dataflow launch that follows the
    order's dependences; strategy 2 (nested chains) and plain mutual
    exclusion over the opt order; strategy 3 (buffer + reduce), the
    colouring and the full shell as the conflict-free references."""
    import torch
    from paper_1401_4441_amd import lc
    g = lc.Grid(box.L, box.rc, 0.0, True)
    ws = lc.Workspace(box.n, g.ncell)
    cs, perm, coord = lc.build_cells(g, pos, ws)

    def one(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = {}
    ws.clear_status()
    for kind in ("bad", "lex", "opt", "loopex"):
        s = lc.Schedule(g, kind)
        sd = lc.serialization_degree(g.nc, kind)
        reps = 1 if sd["cp"] > 50000 else 3
        rows[kind] = {
            "cp": sd["cp"], "S": sd["speedup"],
            "levels_ms": one(lambda: lc.compute_forces(g, s, cs, coord, ws), reps),
            "dataflow_ordered_ms": one(lambda: lc.compute_forces_dataflow(
                g, s, cs, coord, ws, "ordered", limit_ms=20000.0), reps)}
        if kind == "opt":
            for mode in ("nested", "mutex"):
                rows[kind][f"dataflow_{mode}_ms"] = one(lambda: lc.compute_forces_dataflow(
                    g, s, cs, coord, ws, mode, limit_ms=20000.0), 3)
        s.close()
    for kind in ("buffer", "block8", "fullshell"):
        s = lc.Schedule(g, kind)
        rows[kind] = {"ms": one(lambda: lc.compute_forces(g, s, cs, coord, ws), 10)}
        s.close()
    return {"cells": list(g.nc), "status_flags": ws.status(), "rows": rows}


def _time_evals(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# algorithmic bytes of the cell build: read the positions (3 x f64), write
# the permutation (int32) and the box fractions (3 x u32) of every particle,
# and cell_start (int32) of every cell.  The counting sort as built moves
# 64 B per particle: the count pass reads the positions (24 B) and stores
# nothing per particle; the scatter pass reads them again and writes the
# permutation and box fractions (40 B).  The per-cell counters and starts
# stay in the L2 caches.
BUILD_BYTES_PER_PARTICLE = 24 + 4 + 12
BUILD_BYTES_PER_CELL = 4
BUILD_BYTES_MOVED_PER_PARTICLE = 64


def copy_bandwidth_gbs(nbytes=256 * 2 ** 20):
    """Device-to-device copy bandwidth, bytes read + written per second
    (GB/s), median of 5 timings of 10 copies."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ms = statistics.median(_time_evals(lambda: y.copy_(x), 10, 2) for _ in range(5))
    del x, y
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cell_build_stats(lc, g, pos, ws, copy_gbs, reps=20):
    """The cell build (counting sort of `pos` into the cells of `g`) into
    outputs of its own: time and HBM rate against 8 TB/s and against the
    measured copy bandwidth."""
    import torch
    n = pos.shape[1]
    cs = torch.empty(g.ncell + 1, dtype=torch.int32, device=pos.device)
    perm = torch.empty(n, dtype=torch.int32, device=pos.device)
    coord = torch.empty((3, n), dtype=torch.int32, device=pos.device)
    ms = statistics.median(
        _time_evals(lambda: lc.build_cells(g, pos, ws, cs, perm, coord, tile_hint=False), reps, 3)
        for _ in range(3))
    alg = n * BUILD_BYTES_PER_PARTICLE + (g.ncell + 1) * BUILD_BYTES_PER_CELL
    gbs = alg / (ms * 1e-3) / 1e9
    return {"ms": ms, "n": n, "cells": g.ncell, "algorithmic_bytes": alg, "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "copy_GBps": copy_gbs, "frac_of_copy": gbs / copy_gbs,
            "bytes_moved_per_particle": BUILD_BYTES_MOVED_PER_PARTICLE,
            "moved_GBps": (n * BUILD_BYTES_MOVED_PER_PARTICLE) / (ms * 1e-3) / 1e9}


def _line(metric, value, unit, ms, args, config, dtype="f32 pair math, int64 fixed-point accumulation",
          emit=True, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded)", "config": config}
    out.update(extra)
    if emit:
        print(json.dumps(out), flush=True)
    return out


def _best_trial(trials, kinds):
    ok = [t for t in trials if t["kind"] in kinds and not t["fallback"]]
    return min(ok, key=lambda t: t["ms"]) if ok else None


def bench_md(args, emit=True):
    """4M-particle crystal, thermal velocities at T = 1: velocity Verlet with
    dt = 0.005 and a cell rebuild every 10 steps (cells of rc + 0.6 skin).
    The conflict-free pick runs the 100 timed steps; the tile-atomics
    schedule runs 20 steps on a copy of the state for the ratio."""
    import torch
    from paper_1401_4441_amd import lc, synth
    from paper_1401_4441_amd import autotune
    box = synth.workload("fcc4m")
    dev = torch.device("cuda:0")
    g = lc.Grid(box.L, box.rc, 0.6, True)
    pos = torch.from_numpy(box.pos).to(dev)
    # the skin fixes the grid; the schedule and block shape are tuned on the
    # starting configuration (ATOMIC_TILE shapes too, for the baseline)
    tune_all = autotune.tune_shape(g, pos, kinds=("block8", "buffer", "atomic_tile"))
    tune = _best_trial(tune_all["trials"], autotune.BOX_KINDS_CONFLICT_FREE)
    tune_at = _best_trial(tune_all["trials"], ("atomic_tile",))
    ws = lc.Workspace(box.n, g.ncell)
    sched = lc.Schedule(g, tune["kind"], block=tune["block"])
    vel = torch.from_numpy(box.vel).to(dev)
    ids = torch.arange(box.n, dtype=torch.int32, device=dev)
    cs, perm, coord = lc.build_cells(g, pos, ws)  # sets the tile hint
    # launch order: fixed, or heaviest groups first by the starting cell
    # counts (any order gives the same bits; a crystal's counts barely move);
    # 20 steps of each on copies of the state decide
    sched_la = lc.Schedule(g, tune["kind"], block=tune["block"],
                           cell_counts=lc.cell_counts_of(cs))
    order_ms = {}
    sched_at = lc.Schedule(g, "atomic_tile", block=tune_at["block"])
    sched_at_la = lc.Schedule(g, "atomic_tile", block=tune_at["block"],
                              cell_counts=lc.cell_counts_of(cs))
    for name, sc in (("fixed", sched), ("load_aware", sched_la), ("atomic_tile", sched_at),
                     ("atomic_tile_load_aware", sched_at_la)):
        p_, v_, i_ = pos.clone(), vel.clone(), ids.clone()
        lc.verlet_step(g, sc, p_, v_, i_, ws, 0.005, 2, 10)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        lc.verlet_step(g, sc, p_, v_, i_, ws, 0.005, 20, 10)
        t1.record()
        torch.cuda.synchronize()
        order_ms[name] = t0.elapsed_time(t1) / 20
        del p_, v_, i_
    load_aware = order_ms["load_aware"] < order_ms["fixed"]
    if load_aware:
        sched = sched_la
    # the tile-atomics baseline in the same launch order as the headline
    at_fixed, at_la = order_ms.pop("atomic_tile"), order_ms.pop("atomic_tile_load_aware")
    at_ms = at_la if load_aware else at_fixed
    nsteps = 100 if args.steps >= 10 else args.steps
    ws.clear_status()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    trace, F = lc.verlet_step(g, sched, pos, vel, ids, ws, 0.005, nsteps, 10)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nsteps
    st = ws.status()
    tr = trace.cpu().numpy().astype(np.float64) / 2.0 ** 32
    etot = tr[:, 0] + tr[:, 1]
    # pairs per evaluation, for the throughput figure
    cs2, _, co2 = lc.build_cells(g, pos, ws)
    _, ew = lc.compute_forces(g, sched, cs2, co2, ws)
    pairs = int(ew[2].item())
    # the cell build at 4M: on the final positions (stored in cell order by
    # the rebuilds) and on the starting ones (lattice order)
    copy_gbs = copy_bandwidth_gbs()
    build = {"cell_order": cell_build_stats(lc, g, pos, ws, copy_gbs),
             "lattice_order": cell_build_stats(
                 lc, g, torch.from_numpy(box.pos).to(dev), ws, copy_gbs)}
    return _line(
          "pair interactions/sec during velocity-Verlet MD (step incl. kick/drift, rebuilds, energies)",
          pairs / (ms * 1e-3), "pairs/s", ms, args,
          {"workload": "LJ FCC+jitter N=4000000 rho=0.8 rc=2.5, MB T=1, dt=0.005, "
                       "rebuild every 10, skin 0.6, 54^3 cells", "nsteps": nsteps,
           "schedule": tune["kind"], "block": tune["block"], "load_aware": load_aware,
           "launch_order_trials_ms_per_step": order_ms, "status_flags": st,
           "autotune_trials": [[t["kind"], t["block"], round(t["ms"], 4)]
                               for t in tune_all["trials"]]},
          dtype="f32 pairs, int64 forces, f64 positions/velocities/energies",
          emit=emit,
          atomic_tile={"ms_per_step": at_ms, "block": tune_at["block"], "steps": 20,
                       "load_aware": load_aware, "fixed_order_ms_per_step": at_fixed,
                       "load_aware_ms_per_step": at_la, "time_vs_headline": at_ms / ms},
          cell_build=build,
          energy={"E0_per_particle": etot[0] / box.n,
                  "drift_per_particle": (etot[-1] - etot[0]) / box.n,
                  "fluct_per_particle": float(etot.max() - etot.min()) / box.n,
                  "KE0": tr[0, 0] / box.n, "PE0": tr[0, 1] / box.n})


def bench_slab(args, emit=True):
    """2M-particle slab (dense middle third, dilute gas), rc = 3.0, on the
    autotuned grid, with the cell-side variants rc and rc/2."""
    import torch
    from paper_1401_4441_amd import lc, synth
    from paper_1401_4441_amd import autotune
    box = synth.workload("slab2m")
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(box.pos).to(dev)
    tune = autotune.tune_box(pos, box.L, box.rc, reps=5, use_cache=False,
                             kinds=("block8", "buffer", "atomic_tile", "fullshell"))
    cf = [t for t in tune["trials"]
          if t["kind"] in autotune.BOX_KINDS_CONFLICT_FREE and not t["fallback"]]
    pick = min(cf, key=lambda t: t["ms"])
    g = autotune.make_grid(box.L, box.rc, pick["grid"])
    ws = lc.Workspace(box.n, g.ncell)
    cs, perm, coord = lc.build_cells(g, pos, ws)
    F = torch.empty((3, box.n), dtype=torch.int64, device=dev)
    ew = torch.empty(3, dtype=torch.int64, device=dev)
    res = {}
    for kind in ("buffer", "block8", "atomic_tile", "fullshell", "atomic_pair"):
        on_grid = [t for t in tune["trials"]
                   if t["kind"] == kind and t["grid"] == pick["grid"] and not t.get("fallback")]
        blk = tuple(min(on_grid, key=lambda t: t["ms"])["block"]) if on_grid else None
        try:
            s = lc.Schedule(g, kind, block=blk)
        except lc.LCError as e:  # e.g. no block colouring on cells of side rc/2
            res[kind] = {"skipped": str(e)}
            continue
        ws.clear_status()
        ms = _time_evals(lambda: lc.compute_forces(g, s, cs, coord, ws, "fp32", F, ew),
                         max(args.steps // 5, 3), 2)
        res[kind] = {"ms": ms, "block": list(blk) if blk else None, "status_flags": ws.status()}
        s.close()
    pairs = int(ew[2].item())
    counts = (cs[1:] - cs[:-1]).cpu().numpy()
    # load-aware launch order (groups heaviest first by n_A n_B) for the
    # conflict-free kinds: the dense slab's groups start first
    cc = lc.cell_counts_of(cs)
    for kind in ("buffer", "block8", "atomic_tile"):
        if "ms" not in res[kind]:
            continue
        blk = tuple(res[kind]["block"]) if res[kind]["block"] else None
        s = lc.Schedule(g, kind, block=blk, cell_counts=cc)
        ms = _time_evals(lambda: lc.compute_forces(g, s, cs, coord, ws, "fp32", F, ew),
                         max(args.steps // 5, 3), 2)
        res[kind + "_load_aware"] = {"ms": ms, "block": res[kind]["block"],
                                     "status_flags": ws.status()}
        s.close()
    best = min((k for k in ("buffer", "block8", "buffer_load_aware", "block8_load_aware")
                if k in res and "ms" in res[k]), key=lambda k: res[k]["ms"])
    # the tile-atomics baseline in the headline's launch order
    at_key = "atomic_tile_load_aware" if best.endswith("_load_aware") else "atomic_tile"
    # cell side rc against rc/2 (the reach-2 stencil: fewer candidate pairs,
    # smaller and more numerous tasks), fastest trial of each kind per grid
    variants = {}
    for name, gopt in (("rc", {"extra": 0.0, "even": False}),
                       ("rc/2", {"extra": 0.0, "even": False, "half": True})):
        gv = autotune.make_grid(box.L, box.rc, gopt)
        wsv = lc.Workspace(box.n, gv.ncell)
        csv_, _, _ = lc.build_cells(gv, pos, wsv)
        entry = {"cells": list(gv.nc), "candidate_pairs": candidate_pairs(csv_.cpu().numpy(), gv.nc,
                                                                           gv.reach)}
        for kind in ("buffer", "atomic_tile"):
            tr = [t for t in tune["trials"] if t["kind"] == kind and t["grid"] == gopt
                  and not t["fallback"]]
            if tr:
                t = min(tr, key=lambda t: t["ms"])
                entry[kind] = {"ms": t["ms"], "block": t["block"]}
        if "buffer" in entry and "atomic_tile" in entry:
            entry["buffer_speedup_over_atomic_tile"] = (entry["atomic_tile"]["ms"]
                                                        / entry["buffer"]["ms"])
        variants[name] = entry
        wsv.close()
    if "buffer" in variants["rc"] and "buffer" in variants["rc/2"]:
        variants["rc/2_over_rc_time"] = variants["rc/2"]["buffer"]["ms"] / variants["rc"]["buffer"]["ms"]
    return _line("pair interactions/sec (LJ cell-pair force sweep, inhomogeneous slab)",
          pairs / (res[best]["ms"] * 1e-3), "pairs/s", res[best]["ms"], args,
          {"workload": "LJ slab N=2000000, rho 0.75 middle third / 0.02 gas, rc=3.0",
           "cells": list(g.nc), "schedule": best, "block": res[best]["block"],
           "pairs_in_cutoff": pairs, "grid_choice": pick["grid"], "cell_size_variants": variants,
           "autotune_trials": [[t["kind"], t["nc"][0], t["block"], round(t["ms"], 4),
                                t["fallback"]] for t in tune["trials"]],
           "cell_occupancy": {"max": int(counts.max()), "mean": float(counts.mean()),
                              "empty_frac": float((counts == 0).mean())}},
          emit=emit,
          speedup_over_atomic_tile=res[at_key]["ms"] / res[best]["ms"]
          if "ms" in res.get(at_key, {}) else None,
          status_flags=int(np.bitwise_or.reduce([v.get("status_flags", 0) for v in res.values()])),
          schedules={k: (dict(v, pairs_per_s=pairs / (v["ms"] * 1e-3)) if "ms" in v else v)
                     for k, v in res.items()})


def bench_2d(args):
    """A flat (2D) LJ system, 1M particles at areal density 0.7, rc = 2.5, on
    the 2D stencil (Fig. 3a): the autotuned conflict-free sweep against the
    atomics and full-shell baselines, and the paper's 2D creation orders
    (Fig. 5: naive, bad, optimal; loop exchange) run level by level on a
    64k-particle flat box, beside their exact critical paths."""
    import torch
    from paper_1401_4441_amd import autotune, lc, synth
    box = synth.workload("lj2d_1m")
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(box.pos).to(dev)
    g = lc.Grid(box.L, box.rc, flat=True)
    tune = autotune.tune_shape(g, pos, kinds=("block8", "buffer", "atomic_tile", "fullshell"),
                               reps=5)
    ws = lc.Workspace(box.n, g.ncell)
    cs, perm, coord = lc.build_cells(g, pos, ws)
    F = torch.empty((3, box.n), dtype=torch.int64, device=dev)
    ew = torch.empty(3, dtype=torch.int64, device=dev)
    res = {}
    for kind in ("buffer", "block8", "atomic_tile", "fullshell", "atomic_pair"):
        tr = [t for t in tune["trials"] if t["kind"] == kind and not t["fallback"]]
        blk = tuple(min(tr, key=lambda t: t["ms"])["block"]) if tr else None
        s = lc.Schedule(g, kind, block=blk)
        ws.clear_status()
        ms = _time_evals(lambda: lc.compute_forces(g, s, cs, coord, ws, "fp32", F, ew),
                         max(args.steps // 5, 3), 2)
        res[kind] = {"ms": ms, "block": list(blk) if blk else None, "phases": s.info()["nphase"],
                     "status_flags": ws.status()}
        s.close()
    pairs = int(ew[2].item())
    # the conflict-free kinds with their groups launched heaviest first
    cc = lc.cell_counts_of(cs)
    for kind in ("buffer", "block8", "atomic_tile"):
        blk = tuple(res[kind]["block"]) if res[kind]["block"] else None
        s = lc.Schedule(g, kind, block=blk, cell_counts=cc)
        ws.clear_status()
        ms = _time_evals(lambda: lc.compute_forces(g, s, cs, coord, ws, "fp32", F, ew),
                         max(args.steps // 5, 3), 2)
        res[kind + "_load_aware"] = {"ms": ms, "block": res[kind]["block"],
                                     "phases": s.info()["nphase"], "status_flags": ws.status()}
        s.close()
    best = min(("buffer", "block8", "buffer_load_aware", "block8_load_aware"),
               key=lambda k: res[k]["ms"])
    # the paper's 2D orders on a smaller flat box (one launch per DAG level)
    small = synth.square2d(65536, 0.7, rc=2.5, seed=1007)
    gs = lc.Grid(small.L, small.rc, even=True, flat=True)
    wss = lc.Workspace(small.n, gs.ncell)
    ps = torch.from_numpy(small.pos).to(dev)
    css, _, cos = lc.build_cells(gs, ps, wss)
    orders = {}
    for kind in ("lex", "bad", "opt", "loopex"):
        s = lc.Schedule(gs, kind)
        ms = _time_evals(lambda: lc.compute_forces(gs, s, css, cos, wss), 2, 1)
        sd = lc.serialization_degree(gs.nc, kind)
        orders[kind] = {"levels": s.info()["nphase"], "cp": sd["cp"], "S": sd["speedup"],
                        "delta": sd["delta"], "ms": ms}
        s.close()
    _line("pair interactions/sec (LJ cell-pair force sweep, flat 2D system)",
          pairs / (res[best]["ms"] * 1e-3), "pairs/s", res[best]["ms"], args,
          {"workload": "flat LJ N=1000000, square lattice + jitter, areal density 0.7, rc=2.5",
           "cells": list(g.nc), "schedule": best, "block": res[best]["block"],
           "pairs_in_cutoff": pairs},
          schedules={k: dict(v, pairs_per_s=pairs / (v["ms"] * 1e-3)) for k, v in res.items()},
          conflict_free_vs_atomics={
              "speedup_over_atomic_pair": res["atomic_pair"]["ms"] / res[best]["ms"],
              # tile atomics in the headline's launch order
              "speedup_over_atomic_tile": res["atomic_tile_load_aware" if best.endswith(
                  "_load_aware") else "atomic_tile"]["ms"] / res[best]["ms"],
              "speedup_over_full_shell": res["fullshell"]["ms"] / res[best]["ms"]},
          paper_orders_2d={"n": small.n, "cells": list(gs.nc), "orders": orders})


def bench_boxes(args, emit=True):
    """512 independent boxes, N ~ U{500..20000}, density ~ U[0.5, 0.9]: one
    persistent launch (HIP graph replay) against a per-box launch loop.  The
    autotuner picks the cell grids (side rc, or widened by 0.15), the LDS tile
    the split boxes' blocks are sized for, the split and the launch mode; the
    same batch with atomic write-back is the tile-atomics baseline.  Every
    variant's forces are compared with the graph's, per box in input order."""
    import torch
    from paper_1401_4441_amd import autotune, lc, synth
    boxes = synth.boxes(512, 500, 20000, 0.5, 0.9, rc=2.5, seed=777)
    dev = torch.device("cuda:0")
    grid_sets = {"rc": [lc.Grid(b.L, b.rc) for b in boxes],
                 "rc+0.15": [lc.Grid(b.L, b.rc, 0.15) for b in boxes]}
    ns = [b.n for b in boxes]
    pos_all = torch.from_numpy(np.ascontiguousarray(np.concatenate([b.pos for b in boxes], 1))).to(dev)
    tune = autotune.tune_batch(None, ns, pos_all, reps=3, grid_sets=grid_sets)
    grids = grid_sets[tune["grid"]]
    modes = None if tune["modes"] == "auto" else ["blocks"] * len(ns)

    def run_graph(write):
        batch = lc.Batch(grids, ns, modes, tile=tune["tile"], write=write)
        info = batch.info()
        ws = lc.Workspace(info["ntot"], info["ncell"])
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            cs, perm, coord = batch.build_cells(pos_all, ws, stream=side)
            F = torch.empty((3, info["ntot"]), dtype=torch.int64, device=dev)
            ew = torch.empty((len(ns), 3), dtype=torch.int64, device=dev)
            batch.forces(cs, coord, ws, F, ew, tune["persistent"], stream=side)
        side.synchronize()
        graph = batch.graph(cs, coord, F, ew, ws, side, tune["persistent"])
        with torch.cuda.stream(side):
            ms = _time_evals(lambda: graph.launch(side), args.steps, args.warmup)
        side.synchronize()
        st = ws.status()
        Fu = torch.empty_like(F)
        Fu[:, perm.long()] = F  # input order
        graph.close()
        return {"ms": ms, "info": info, "status_flags": st, "F": Fu, "ew": ew.clone()}

    g_buf = run_graph("buffer")
    g_at = run_graph("atomic")
    info = g_buf["info"]
    pairs = int(g_buf["ew"][:, 2].sum().item())
    same_at = bool(torch.equal(g_at["F"], g_buf["F"]) and torch.equal(g_at["ew"], g_buf["ew"]))
    # per-box launch loop: every box its own arrays, schedule and launches
    ps = np.concatenate([[0], np.cumsum(ns)])
    per = []
    for k, (b, g) in enumerate(zip(boxes, grids)):
        wsb = lc.Workspace(b.n, g.ncell)
        c, pm, co = lc.build_cells(g, pos_all[:, ps[k]:ps[k + 1]].contiguous(), wsb)
        per.append((g, lc.Schedule(g, "buffer"), c, pm, co, wsb))

    def loop():
        for g, s, c, pm, co, wsb in per:
            lc.compute_forces(g, s, c, co, wsb)
    ms_loop = _time_evals(loop, max(args.steps // 10, 2), 1)
    # the loop's forces against the graph's, box by box in input order
    same_loop = True
    loop_flags = 0
    for k, (g, s, c, pm, co, wsb) in enumerate(per):
        F, ew = lc.compute_forces(g, s, c, co, wsb)
        Fu = torch.empty_like(F)
        Fu[:, pm.long()] = F
        same_loop &= bool(torch.equal(Fu, g_buf["F"][:, ps[k]:ps[k + 1]])
                          and torch.equal(ew, g_buf["ew"][k]))
        loop_flags |= wsb.status()
    return _line("pair interactions/sec over 512 independent boxes (one persistent graph launch)",
                 pairs / (g_buf["ms"] * 1e-3), "pairs/s", g_buf["ms"], args,
                 {"workload": "512 LJ FCC boxes, N~U{500..20000}, rho~U[0.5,0.9], rc=2.5",
                  "ntot": info["ntot"], "groups": info["ngroup"],
                  "whole_box_groups": info["nwhole"], "max_replicas": info["max_replicas"],
                  "lds_tile": info["lds_tile"], "pairs_in_cutoff": pairs,
                  "autotune": {k: v for k, v in tune.items() if k != "trials"},
                  "autotune_trials": [[t["grid"], t["tile"], t["modes"], t["persistent"],
                                       round(t["ms"], 4), t["fallback"]] for t in tune["trials"]],
                  "status_flags": g_buf["status_flags"]},
                 emit=emit,
                 atomic_tile={"ms": g_at["ms"], "status_flags": g_at["status_flags"],
                              "same_bits_as_headline": same_at,
                              "time_vs_headline": g_at["ms"] / g_buf["ms"]},
                 per_box_loop={"ms": ms_loop, "pairs_per_s": pairs / (ms_loop * 1e-3),
                               "graph_speedup": ms_loop / g_buf["ms"],
                               "same_bits_as_graph": same_loop, "status_flags": loop_flags})

if __name__ == "__main__":
    main()
