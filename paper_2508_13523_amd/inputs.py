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


def fcc_lattice(ncell, rho: float = RHO_FCC):
    """Perfect FCC crystal of ncell^3 cubic unit cells (or nx x ny x nz of
    them when ncell is a triple: an orthorhombic box) at number density rho.

    Atom order: unit cell z (slowest), y, x, then the 4-atom basis
    (0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2).
    """
    nc = np.broadcast_to(np.asarray(ncell, dtype=np.int64), (3,))
    a = (4.0 / rho) ** (1.0 / 3.0)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cz, cy, cx = np.meshgrid(np.arange(nc[2], dtype=np.float64),
                             np.arange(nc[1], dtype=np.float64),
                             np.arange(nc[0], dtype=np.float64), indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    x = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    box = nc.astype(np.float64) * a
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


def rsa_positions(types: np.ndarray, L: float, dmin: np.ndarray, seed: int,
                  batch: int = 4096, slots: int = 16):
    """Random sequential addition in a periodic cubic box of side L: every atom
    is inserted at a uniformly random point, and an insertion is kept only if
    the point lies at least dmin[t_i][t_j] (minimum image) from every atom
    already placed; a rejected atom tries again at a new random point.

    Insertions are processed in rounds: each round draws several trial points
    for each waiting atom (in atom order), keeps each atom's first trial point
    that clears the atoms placed in earlier rounds, then accepts those points
    in atom order, dropping any that comes within dmin of a point accepted
    before it in the same round.  A uniform grid of cells at least max(dmin)
    wide holds the placed atoms (at most `slots` per cell)."""
    rng = np.random.default_rng(seed)
    types = np.asarray(types, dtype=np.int64)
    n = types.shape[0]
    dmin2 = np.asarray(dmin, dtype=np.float64) ** 2
    ng = max(1, int(math.floor(L / float(np.max(dmin)))))
    if ng < 3:
        raise ValueError("box too small for the cell grid of the insertion")
    cw = L / ng
    occ = np.full((ng ** 3, slots), -1, dtype=np.int64)
    cnt = np.zeros(ng ** 3, dtype=np.int64)
    x = np.zeros((n, 3))
    placed = np.zeros(n, dtype=bool)
    off = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])

    def cell_of(p):
        c = np.minimum((p / cw).astype(np.int64), ng - 1)
        return c

    def min_image(d):
        return d - L * np.round(d / L)

    waiting = np.arange(n)
    while waiting.size:
        atoms = waiting[:batch]
        m = max(1, batch // atoms.size)  # trial points per waiting atom
        trial = rng.uniform(0.0, L, size=(atoms.size, m, 3)).reshape(-1, 3)
        tt = np.repeat(types[atoms], m)
        c3 = cell_of(trial)
        nb = (c3[:, None, :] + off[None, :, :]) % ng
        nb_id = (nb[..., 2] * ng + nb[..., 1]) * ng + nb[..., 0]
        kmax = max(1, int(cnt.max()))  # filled slots of the fullest cell
        others = occ[nb_id][..., :kmax].reshape(trial.shape[0], -1)  # [trials, 27 * kmax]
        valid = others >= 0
        oj = np.where(valid, others, 0)
        d = min_image(trial[:, None, :] - x[oj])
        r2 = (d * d).sum(axis=2)
        clear = np.all(~valid | (r2 >= dmin2[tt[:, None], types[oj]]), axis=1)
        clear = clear.reshape(atoms.size, m)
        has = clear.any(axis=1)
        pick = np.argmax(clear, axis=1)
        cand_atoms = atoms[has]
        cand = trial.reshape(atoms.size, m, 3)[np.nonzero(has)[0], pick[has]]
        # accept in atom order against the points accepted before in this round
        acc = np.ones(cand_atoms.size, dtype=bool)
        if cand_atoms.size > 1:
            ct = types[cand_atoms]
            for k0 in range(0, cand_atoms.size, 512):
                blk = slice(k0, min(cand_atoms.size, k0 + 512))
                dd = min_image(cand[blk][:, None, :] - cand[None, :blk.stop, :])
                rr = (dd * dd).sum(axis=2)
                clash = rr < dmin2[ct[blk][:, None], ct[None, :blk.stop]]
                rows_k = np.arange(blk.start, blk.stop)
                clash &= np.arange(blk.stop)[None, :] < rows_k[:, None]  # earlier points only
                for r_ in np.nonzero(clash.any(axis=1))[0]:
                    k = blk.start + r_
                    if np.any(acc[np.nonzero(clash[r_])[0]]):
                        acc[k] = False
        new = cand_atoms[acc]
        x[new] = cand[acc]
        placed[new] = True
        cc = cell_of(x[new])
        cid = (cc[:, 2] * ng + cc[:, 1]) * ng + cc[:, 0]
        for a_, c_ in zip(new, cid):
            if cnt[c_] >= slots:
                raise RuntimeError("insertion grid cell overflow")
            occ[c_, cnt[c_]] = a_
            cnt[c_] += 1
        waiting = waiting[~placed[waiting]]
    return x


def binary_liquid_random(n: int, seed: int, rho: float = RHO_BINARY,
                         temperature: float = T_BINARY, dmin_frac: float = 0.8) -> System:
    """80:20 binary LJ liquid start with random positions at density rho:
    exact composition by a seeded permutation, then random sequential
    addition with minimum distances dmin_frac * sigma_ij (a plain uniform
    placement would put atoms on top of each other), Maxwell velocities at
    T = 0.8; rc_ij = 2.5 sigma_ij.  The caller equilibrates it."""
    L = (n / rho) ** (1.0 / 3.0)
    t = binary_types(n, 0.8, seed + 7919)
    eps, sig, rc = binary_tables()
    x = rsa_positions(t, L, dmin_frac * sig, seed)
    x = into_box(x, np.full(3, L))
    v = maxwell(n, temperature, np.ones(n), seed + 104729)
    return System(x=x, v=v, types=t, box=np.full(3, L), eps=eps, sigma=sig, rc=rc, skin=0.3,
                  mass=np.ones(2), name=f"binary_rsa{n}")


def single_type_tables(eps=1.0, sigma=1.0, rc=2.5):
    return (np.array([[eps]], dtype=np.float64), np.array([[sigma]], dtype=np.float64),
            np.array([[rc]], dtype=np.float64))


def binary_tables(rc_over_sigma: float = 2.5):
    eps = BINARY_EPS.copy()
    sig = BINARY_SIGMA.copy()
    return eps, sig, rc_over_sigma * sig


def fcc_liquid(ncell, seed_pos: int = 1, seed_vel: int = 2, rho: float = RHO_FCC,
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


def grid_system(shape, rho: float, seed: int, binary: bool = False,
                jitter_std: float = 0.08, temperature: float = 1.0) -> System:
    """Atoms on an nx x ny x nz simple-cubic grid at number density rho (an
    orthorhombic box of nx a x ny a x nz a, a = rho^(-1/3)), each jittered by
    N(0, jitter_std^2); single-type LJ, or the 80:20 binary mixture."""
    nc = np.asarray(shape, dtype=np.int64)
    a = (1.0 / rho) ** (1.0 / 3.0)
    iz, iy, ix = np.meshgrid(np.arange(nc[2]), np.arange(nc[1]), np.arange(nc[0]),
                             indexing="ij")
    x = (np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64) + 0.5) * a
    box = nc.astype(np.float64) * a
    x = jitter(x, box, jitter_std, seed)
    n = x.shape[0]
    if binary:
        t = binary_types(n, 0.8, seed + 11)
        eps, sig, rc = binary_tables()
        mass = np.ones(2)
    else:
        t = np.zeros(n, dtype=np.int32)
        eps, sig, rc = single_type_tables()
        mass = np.ones(1)
    v = maxwell(n, temperature, np.ones(n), seed + 23)
    return System(x=x, v=v, types=t, box=box, eps=eps, sigma=sig, rc=rc, skin=0.3, mass=mass,
                  name=f"grid{tuple(int(k) for k in nc)}")


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
