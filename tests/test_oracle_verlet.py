"""Pins for the oracle's velocity Verlet (CPU only): time reversibility,
second-order energy fluctuation, and agreement of the first step with the
update written out by hand."""
import numpy as np
import pytest

import oracle as O
from paper_1401_4441_amd import synth

S = O.SCALE


def _system(n=500, seed=21):
    b = synth.fcc(n, 0.8, rc=2.5, seed=seed)
    v = synth.maxwell_boltzmann(b.n, 1.0, seed=seed + 1)
    return b, v


def test_first_step_by_hand():
    b, v = _system()
    dt = 0.005
    u = O.canonical(b.pos, b.L)
    F0, *_ = O.forces_lc_fx(u, b.L, b.rc, O.grid_dims(b.L, b.rc))
    v1 = v + (0.5 * dt) * (F0.astype(np.float64) / S)
    x1 = b.pos + dt * v1
    F1, E1, *_ = O.forces_lc_fx(O.canonical(x1, b.L), b.L, b.rc,
                                O.grid_dims(b.L, b.rc))
    v2 = v1 + (0.5 * dt) * (F1.astype(np.float64) / S)
    pos, vel, F, trace = O.verlet_fx(b.pos, v, b.L, b.rc, dt, 1)
    assert (pos == x1).all() and (vel == v2).all() and (F == F1).all()
    assert trace[1, 1] == E1
    ke = np.sum(np.rint(0.5 * np.sum(v2 * v2, axis=0) * S).astype(np.int64))
    assert abs(int(trace[1, 0]) - int(ke)) <= b.n  # summation order of v^2 terms


def test_time_reversibility():
    """Integrate forward, flip velocities, integrate back: the start state
    returns up to FP64 rounding."""
    b, v = _system(seed=31)
    pos, vel, _, _ = O.verlet_fx(b.pos, v, b.L, b.rc, 0.005, 40)
    pos2, vel2, _, _ = O.verlet_fx(pos, -vel, b.L, b.rc, 0.005, 40)
    assert np.abs(pos2 - b.pos).max() < 1e-7
    assert np.abs(-vel2 - v).max() < 1e-7


def test_energy_fluctuation_second_order():
    """Halving dt quarters the total-energy fluctuation (Verlet is second
    order); no systematic drift over the run."""
    b, v = _system(seed=41)
    amp = []
    for dt, steps in ((0.004, 100), (0.002, 200)):
        _, _, _, tr = O.verlet_fx(b.pos, v, b.L, b.rc, dt, steps)
        e = (tr[:, 0] + tr[:, 1]).astype(np.float64) / S
        amp.append(e.max() - e.min())
    ratio = amp[0] / amp[1]
    assert 3.0 < ratio < 5.0
    assert amp[1] / b.n < 5e-4
