"""Seeded synthetic inputs for the link-cell force sweep.

This module draws particle configurations only: lattice sites, jitter,
vacancies and thermal velocities.  It holds none of the method's arithmetic
(no cells, no pair forces, no fixed-point encoding); both the GPU path and the
CPU oracle consume the arrays it returns, so the two sides see identical bits.

The paper (Sec. IV) describes the link-cell method for short-range particle
interactions but prints no particle data, so the workloads are synthetic
Lennard-Jones systems in reduced units (epsilon = sigma = mass = k_B = 1):

* ``fcc``      -- face-centred cubic crystal with uniform jitter, periodic cube;
* ``slab``     -- dense FCC slab (middle third along z) in a dilute FCC gas;
* ``boxes``    -- many independent periodic boxes of uneven size and density;
* ``square2d`` -- a flat (2D) square lattice with jitter, all particles at z = 0;
* ``maxwell_boltzmann`` -- seeded thermal velocities at a target temperature.

All positions are returned as float64 arrays of shape ``(3, N)`` (SoA, one
contiguous row per axis), wrapped into ``[0, L)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Conventional FCC basis in units of the lattice constant.
_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]
)


@dataclass
class Box:
    """One periodic box: SoA positions (3, N), edge lengths, cutoff."""

    pos: np.ndarray
    L: np.ndarray
    rc: float
    seed: int
    vel: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


def _fcc_sites(m: int, a: float) -> np.ndarray:
    """All 4*m^3 FCC sites of an m x m x m block of unit cells, shape (N, 3)."""
    g = np.arange(m, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    corners = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    sites = (corners[:, None, :] + _FCC_BASIS[None, :, :]).reshape(-1, 3)
    return sites * a


def _wrap(pos: np.ndarray, L: np.ndarray) -> np.ndarray:
    out = np.mod(pos, L[:, None])
    # np.mod can return exactly L for tiny negative inputs; fold those to 0.
    out[out >= L[:, None]] = 0.0
    return out


def fcc(n: int, density: float, rc: float = 2.5, jitter: float = 0.05,
        seed: int = 1234) -> Box:
    """FCC crystal of ``n`` particles at ``density`` in a periodic cube.

    When ``n`` is not 4*m^3 the lattice is built with m = ceil((n/4)^(1/3))
    unit cells per side and a seeded random subset of ``n`` sites is kept
    (uniform vacancies).  Each coordinate then gets independent uniform jitter
    in ``[-jitter, +jitter]``.
    """
    rng = np.random.default_rng(seed)
    L = (n / density) ** (1.0 / 3.0)
    m = round((n / 4) ** (1.0 / 3.0))
    if 4 * m ** 3 != n:
        m = math.ceil((n / 4) ** (1.0 / 3.0))
    a = L / m
    sites = _fcc_sites(m, a)
    if sites.shape[0] != n:
        keep = np.sort(rng.choice(sites.shape[0], size=n, replace=False))
        sites = sites[keep]
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    Lv = np.array([L, L, L])
    pos = _wrap(np.ascontiguousarray(sites.T), Lv)
    return Box(pos=np.ascontiguousarray(pos), L=Lv, rc=rc, seed=seed,
               meta={"kind": "fcc", "density": density, "a": a, "m": m,
                     "jitter": jitter})


def square2d(n: int, density: float, rc: float = 2.5, jitter: float = 0.05,
             seed: int = 1234) -> Box:
    """A flat (2D) system: ``n`` particles on a square lattice at areal
    ``density`` with uniform jitter in x and y, all at z = 0.

    When ``n`` is not m^2 a seeded random subset of the m = ceil(sqrt(n))
    lattice is kept.  The box is L x L in the plane; its z edge (4 rc) only
    has to be positive, since every z difference is zero.
    """
    rng = np.random.default_rng(seed)
    L = math.sqrt(n / density)
    m = math.isqrt(n)
    if m * m != n:
        m = math.ceil(math.sqrt(n))
    a = L / m
    g = np.arange(m, dtype=np.float64)
    cy, cx = np.meshgrid(g, g, indexing="ij")
    sites = np.stack([cx.ravel(), cy.ravel()], axis=1) * a
    if sites.shape[0] != n:
        keep = np.sort(rng.choice(sites.shape[0], size=n, replace=False))
        sites = sites[keep]
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    Lv = np.array([L, L, 4.0 * rc])
    pos = np.zeros((3, n))
    pos[:2] = sites.T
    pos = _wrap(pos, Lv)
    return Box(pos=np.ascontiguousarray(pos), L=Lv, rc=rc, seed=seed,
               meta={"kind": "square2d", "density": density, "a": a, "m": m,
                     "jitter": jitter})


def maxwell_boltzmann(n: int, temperature: float = 1.0, seed: int = 99) -> np.ndarray:
    """Seeded thermal velocities, shape (3, N), unit mass.

    Components are standard normal draws; the centre-of-mass velocity is
    removed and the result is rescaled so that sum(v^2) = (3N - 3) * T.
    """
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(size=(3, n))
    v -= v.mean(axis=1, keepdims=True)
    ke2 = float(np.sum(v * v))
    v *= math.sqrt((3 * n - 3) * temperature / ke2)
    return np.ascontiguousarray(v)


def slab(n: int, rho_dense: float = 0.75, rho_gas: float = 0.02,
         rc: float = 3.0, jitter: float = 0.05, gap: float = 1.0,
         seed: int = 4321) -> Box:
    """Inhomogeneous slab: dense FCC in the middle third along z, dilute FCC
    gas elsewhere, in a periodic cube of side L = (n / (rho_d/3 + 2 rho_g/3))^(1/3).

    The dense region gets round(rho_d * L^3 / 3) particles and the gas the
    rest; each phase is a seeded random subset of an FCC lattice fitted to the
    box that is at least as dense as required (so no two particles overlap),
    with the gas kept ``gap`` away from the interfaces."""
    rng = np.random.default_rng(seed)
    L = (n / (rho_dense / 3.0 + 2.0 * rho_gas / 3.0)) ** (1.0 / 3.0)
    z0, z1 = L / 3.0, 2.0 * L / 3.0
    n_dense = min(n, int(round(rho_dense * L ** 3 / 3.0)))
    n_gas = n - n_dense

    def lattice(rho, inside, want):
        m = max(1, int(math.ceil(L * (rho / 4.0) ** (1.0 / 3.0))))
        while True:
            sites = _fcc_sites(m, L / m)
            sites = sites[inside(sites[:, 2])]
            if sites.shape[0] >= want:
                keep = np.sort(rng.choice(sites.shape[0], size=want, replace=False))
                return sites[keep]
            m += 1

    dense = lattice(rho_dense, lambda z: (z >= z0) & (z < z1), n_dense)
    gas = lattice(rho_gas, lambda z: (z < z0 - gap) | (z >= z1 + gap), n_gas)
    sites = np.concatenate([dense, gas], axis=0)
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    Lv = np.array([L, L, L])
    pos = _wrap(np.ascontiguousarray(sites.T), Lv)
    return Box(pos=np.ascontiguousarray(pos), L=Lv, rc=rc, seed=seed,
               meta={"kind": "slab", "rho_dense": rho_dense,
                     "rho_gas": rho_gas, "n_dense": int(n_dense)})


def boxes(count: int = 512, n_lo: int = 500, n_hi: int = 20000,
          rho_lo: float = 0.5, rho_hi: float = 0.9, rc: float = 2.5,
          seed: int = 777) -> list[Box]:
    """``count`` independent periodic FCC boxes, N ~ U{n_lo..n_hi},
    density ~ U[rho_lo, rho_hi], each with its own seed."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    rhos = rng.uniform(rho_lo, rho_hi, size=count)
    seeds = rng.integers(1, 2 ** 31 - 1, size=count)
    return [fcc(int(ns[b]), float(rhos[b]), rc=rc, seed=int(seeds[b]))
            for b in range(count)]


# Named workloads.  Sizes follow the configurations the force sweep is
# evaluated on; everything is derived from a fixed seed.
def workload(name: str) -> Box:
    if name == "fcc4k":
        return fcc(4000, 0.8, rc=2.5, seed=1001)
    if name == "fcc256k":
        return fcc(256000, 0.8, rc=2.5, seed=1002)
    if name == "fcc4m":
        b = fcc(4_000_000, 0.8, rc=2.5, seed=1003)
        b.vel = maxwell_boltzmann(b.n, 1.0, seed=2003)
        return b
    if name == "slab2m":
        return slab(2_000_000, seed=1005)
    if name == "lj2d_1m":
        return square2d(1_000_000, 0.7, rc=2.5, seed=1006)
    raise KeyError(name)
