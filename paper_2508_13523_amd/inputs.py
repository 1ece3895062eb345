"""Seeded synthetic inputs for the Lennard-Jones hot path.

This module only builds geometry, types, velocities and parameter tables; it
holds none of the method's arithmetic (no pair energy, force or integrator)
and imports nothing else from this package.  Both the HIP path and the CPU
oracle are fed from it, so they see identical bits.

The paper benchmarks LJ on LAMMPS' own input decks, which are not reproduced
here; these recipes stand in for them at the same scale (an FCC liquid at
reduced density 0.8442, T = 1.44, cutoff 2.5 sigma, skin 0.3, and a binary
80:20 liquid at density 1.2 with type-pair parameters).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

RHO_FCC = 0.8442
T_FCC = 1.44
RHO_BINARY = 1.2
T_BINARY = 0.8

# Binary A/B liquid parameters: eps_AA=1, sig_AA=1; eps_AB=1.5, sig_AB=0.8;
# eps_BB=0.5, sig_BB=0.88; cutoff 2.5 sig_ij.
BINARY_EPS = np.array([[1.0, 1.5], [1.5, 0.5]])
BINARY_SIGMA = np.array([[1.0, 0.8], [0.8, 0.88]])


@dataclasses.dataclass
class System:
    """One periodic LJ system, host arrays (float64 / int32)."""

    x: np.ndarray          # [n, 3] positions in [0, L)
    v: np.ndarray          # [n, 3] velocities
    types: np.ndarray      # [n] int32
    box: np.ndarray        # [3] box lengths
    eps: np.ndarray        # [T, T]
    sigma: np.ndarray      # [T, T]
    rc: np.ndarray         # [T, T]
    skin: float
    mass: np.ndarray       # [T]
    dt: float = 0.005
    rebuild_every: int = 20
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def ntypes(self) -> int:
        return int(self.eps.shape[0])


def fcc_lattice(ncell: int, rho: float = RHO_FCC):
    """Perfect FCC crystal of ncell^3 cubic unit cells at number density rho.

    Atom order: unit cell z (slowest), y, x, then the 4-atom basis
    (0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2).
    """
    a = (4.0 / rho) ** (1.0 / 3.0)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    r = np.arange(ncell, dtype=np.float64)
    cz, cy, cx = np.meshgrid(r, r, r, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    x = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    box = np.full(3, ncell * a)
    return np.ascontiguousarray(x), box


def into_box(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Map coordinates into [0, L) (input preparation only)."""
    y = np.mod(x, box)
    y[y >= box] = 0.0
    return np.ascontiguousarray(y)


def jitter(x: np.ndarray, box: np.ndarray, std: float, seed: int) -> np.ndarray:
    """Add N(0, std^2) to every coordinate (numpy PCG64), then map into the box."""
    rng = np.random.default_rng(seed)
    return into_box(x + rng.normal(0.0, std, size=x.shape), box)


def maxwell(n: int, temperature: float, masses: np.ndarray, seed: int) -> np.ndarray:
    """Maxwell velocities: N(0, T/m) per component, zero total momentum, and
    rescaled so that the kinetic temperature with 3n-3 degrees of freedom is
    exactly `temperature`."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64).reshape(n, 1)
    v = rng.normal(0.0, 1.0, size=(n, 3)) * np.sqrt(temperature / m)
    v -= (m * v).sum(axis=0) / m.sum()
    ke = 0.5 * float((m * v * v).sum())
    target = 0.5 * (3 * n - 3) * temperature
    if ke > 0:
        v *= math.sqrt(target / ke)
    return np.ascontiguousarray(v)


def binary_types(n: int, frac_a: float, seed: int) -> np.ndarray:
    """Exactly round((1-frac_a) n) atoms of type 1 (B), placed by a seeded
    permutation; the rest are type 0 (A)."""
    rng = np.random.default_rng(seed)
    nb = int(round((1.0 - frac_a) * n))
    t = np.zeros(n, dtype=np.int32)
    t[rng.permutation(n)[:nb]] = 1
    return t


def random_sites(n: int, rho: float, seed: int, std: float = 0.02):
    """n atoms on a random subset of an m^3 simple-cubic grid (m^3 >= n) in a
    cubic box at density rho, each jittered by N(0, std^2).  No two atoms
    start closer than about the grid spacing (~0.9 at rho = 1.2)."""
    rng = np.random.default_rng(seed)
    L = (n / rho) ** (1.0 / 3.0)
    m = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    while m ** 3 < n:
        m += 1
    sites = rng.permutation(m ** 3)[:n]
    iz, rem = np.divmod(sites, m * m)
    iy, ix = np.divmod(rem, m)
    h = L / m
    x = (np.stack([ix, iy, iz], axis=1).astype(np.float64) + 0.5) * h
    box = np.full(3, L)
    x = into_box(x + rng.normal(0.0, std, size=x.shape), box)
    return x, box


def single_type_tables(eps=1.0, sigma=1.0, rc=2.5):
    return (np.array([[eps]], dtype=np.float64), np.array([[sigma]], dtype=np.float64),
            np.array([[rc]], dtype=np.float64))


def binary_tables(rc_over_sigma: float = 2.5):
    eps = BINARY_EPS.copy()
    sig = BINARY_SIGMA.copy()
    return eps, sig, rc_over_sigma * sig


def fcc_liquid(ncell: int, seed_pos: int = 1, seed_vel: int = 2, rho: float = RHO_FCC,
               temperature: float = T_FCC, jitter_std: float = 0.01) -> System:
    """FCC start jittered by N(0, 0.01^2), Maxwell velocities at T = 1.44,
    eps = sigma = 1, rc = 2.5, skin 0.3 (the single-type LJ workloads)."""
    x, box = fcc_lattice(ncell, rho)
    x = jitter(x, box, jitter_std, seed_pos)
    n = x.shape[0]
    v = maxwell(n, temperature, np.ones(n), seed_vel)
    eps, sig, rc = single_type_tables()
    return System(x=x, v=v, types=np.zeros(n, dtype=np.int32), box=box, eps=eps, sigma=sig,
                  rc=rc, skin=0.3, mass=np.ones(1), name=f"fcc{ncell}")


def binary_liquid(n: int, seed: int, rho: float = RHO_BINARY,
                  temperature: float = T_BINARY) -> System:
    """80:20 binary LJ liquid start: random grid sites at density 1.2, exact
    composition, Maxwell velocities at T = 0.8, rc_ij = 2.5 sigma_ij."""
    x, box = random_sites(n, rho, seed)
    t = binary_types(n, 0.8, seed + 7919)
    v = maxwell(n, temperature, np.ones(n), seed + 104729)
    eps, sig, rc = binary_tables()
    return System(x=x, v=v, types=t, box=box, eps=eps, sigma=sig, rc=rc, skin=0.3,
                  mass=np.ones(2), name=f"binary{n}")


def perturbed_params(eps: np.ndarray, sigma: np.ndarray, seed: int, frac: float = 0.05):
    """theta' = theta (1 + u), u ~ U(-frac, frac), independently for each of the
    unique (upper-triangle) entries; the tables stay symmetric."""
    rng = np.random.default_rng(seed)
    T = eps.shape[0]
    e2, s2 = eps.copy(), sigma.copy()
    for a in range(T):
        for b in range(a, T):
            ue, us = rng.uniform(-frac, frac, size=2)
            e2[a, b] = e2[b, a] = eps[a, b] * (1 + ue)
            s2[a, b] = s2[b, a] = sigma[a, b] * (1 + us)
    return e2, s2


def replica_sizes(count: int = 512, lo: int = 500, hi: int = 8000, seed: int = 6) -> np.ndarray:
    """Replica atom counts, integers uniform on [lo, hi] inclusive."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count).astype(np.int64)


def replica_batch(sizes, seed_base: int = 1000) -> dict:
    """Independent binary-liquid systems, system r prepared as
    binary_liquid(sizes[r], seed_base + r), concatenated: x, v, types
    (batch-wide arrays), offsets [R+1], boxes [R, 3] and the shared tables."""
    systems = [binary_liquid(int(nr), seed_base + r) for r, nr in enumerate(sizes)]
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    np.cumsum([s.n for s in systems], out=off[1:])
    s0 = systems[0]
    return dict(x=np.concatenate([s.x for s in systems]),
                v=np.concatenate([s.v for s in systems]),
                types=np.concatenate([s.types for s in systems]),
                offsets=off, boxes=np.stack([s.box for s in systems]),
                eps=s0.eps, sigma=s0.sigma, rc=s0.rc, skin=s0.skin, mass=s0.mass,
                systems=systems)
