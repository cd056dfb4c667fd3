"""Host-side logic of bench.py (no GPU): the one-GPU guard, the candidate
pair count it reports, the half shells it counts over, and the source hash
that keys the committed profiles."""
import itertools
import json
import os
import subprocess
import sys

import numpy as np

import oracle as O
from paper_1401_4441_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_half_shells():
    for reach, size in ((1, 13), (2, 62)):
        hs = bench.half_shell(reach)
        assert len(hs) == size == ((2 * reach + 1) ** 3 - 1) // 2
        full = set(hs) | {tuple(-c for c in d) for d in hs}
        assert len(full) == 2 * size and (0, 0, 0) not in full
        assert all(max(abs(c) for c in d) <= reach for d in hs)


def _brute_candidates(u, nc, reach):
    """Unordered pairs whose cells differ by at most `reach` per axis
    (periodic), counted pair by pair."""
    cid = O.cell_ids(u, nc)
    cz, rem = np.divmod(cid, nc[0] * nc[1])
    cy, cx = np.divmod(rem, nc[0])
    total = 0
    n = u.shape[1]
    for i in range(n):
        d = []
        for c, m in ((cx, nc[0]), (cy, nc[1]), (cz, nc[2])):
            x = (c[i + 1:] - c[i]) % m
            d.append(np.minimum(x, m - x))
        total += int(np.sum((d[0] <= reach) & (d[1] <= reach) & (d[2] <= reach)))
    return total


def test_candidate_pairs_match_brute_force():
    for n, rho, reach in ((700, 0.8, 1), (900, 0.8, 2)):
        b = synth.fcc(n, rho, rc=2.5 if reach == 1 else 1.25, seed=31)
        nc = O.grid_dims(b.L, b.rc)
        assert (nc >= 2 * reach + 1).all()
        u = O.canonical(b.pos, b.L)
        cs = O.cell_start(u, nc)
        assert bench.candidate_pairs(cs, nc, reach) == _brute_candidates(u, nc, reach)


def test_load_aware_flag_and_source_hash():
    h = bench.source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert bench.source_hash() == h
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "--load-aware" in r.stdout
