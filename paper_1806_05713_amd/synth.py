"""Seeded synthetic inputs for the Lennard-Jones path.

This module only draws inputs: lattice sites, uniform jitter, a random atom
order, Maxwell velocities and the parameters of a batch of systems.  It holds
none of the force, list or cell arithmetic, so the CPU oracle and the GPU
library can both be fed from it without sharing any of the method.

Workloads follow the paper's benchmark (Sec. II): atoms on a face-centred
cubic lattice in a cubic periodic box at number density rho, cutoff 3 sigma,
sigma = epsilon = 1.  The lattice of n^3 unit cells holds N = 4 n^3 atoms, so
the box length is L = (N / rho)^(1/3) and the lattice constant is L / n.

All randomness comes from numpy's PCG64 seeded with an integer (or a
SeedSequence child for the batched systems), so every input is reproducible.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Basis of the conventional FCC unit cell, in units of the lattice constant.
_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]],
    dtype=np.float64,
)


@dataclasses.dataclass
class System:
    """One periodic LJ system: positions in [0, L)^3 plus its parameters."""

    pos: np.ndarray          # (N, 3) float64, row-major
    box: np.ndarray          # (3,) float64, cubic here
    rc: float
    skin: float
    eps: float = 1.0
    sigma: float = 1.0
    vel: Optional[np.ndarray] = None   # (N, 3) float64 or None
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def rho(self) -> float:
        return self.n / float(np.prod(self.box))


def wrap(x: np.ndarray, L: float) -> np.ndarray:
    """Map coordinates into [0, L): x - L*floor(x/L), with a result equal to L set to 0."""
    y = x - L * np.floor(x / L)
    y[y >= L] = 0.0
    return y


def fcc_sites(n: int, L: float) -> np.ndarray:
    """All 4 n^3 FCC sites of an n x n x n lattice in a box of side L.

    Site = a * (cell + basis + 1/4) with a = L / n; the quarter offset keeps
    every site off the box faces.  Order: x fastest, then y, then z, with the
    four basis atoms innermost (the lattice order, spatially coherent).
    """
    a = L / n
    idx = np.arange(n, dtype=np.float64)
    cz, cy, cx = np.meshgrid(idx, idx, idx, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)  # x fastest
    sites = (cells[:, None, :] + _FCC_BASIS[None, :, :] + 0.25) * a
    return sites.reshape(-1, 3)


def fcc_box(n: int, rho: float) -> float:
    return (4.0 * n ** 3 / rho) ** (1.0 / 3.0)


def jitter(pos: np.ndarray, L: float, delta: float, rng: np.random.Generator) -> np.ndarray:
    """Add U(-delta, delta) independently to each coordinate, then wrap into [0, L)."""
    if delta == 0.0:
        return pos.copy()
    out = pos + rng.uniform(-delta, delta, size=pos.shape)
    return wrap(out, L)


def maxwell(n: int, T: float, rng: np.random.Generator) -> np.ndarray:
    """Maxwell velocities for unit mass: N(0, T) per component, zero total
    momentum, rescaled so that the kinetic temperature with 3N-3 degrees of
    freedom equals T exactly."""
    v = rng.normal(0.0, math.sqrt(T), size=(n, 3))
    v -= v.mean(axis=0, keepdims=True)
    ke2 = float(np.sum(v * v))           # = 2 * kinetic energy
    dof = 3 * n - 3
    if ke2 > 0.0 and dof > 0:
        v *= math.sqrt(T * dof / ke2)
    return v


def permuted(sys: System, seed: int) -> System:
    """The same system with its atoms in a seeded random order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(sys.n)
    vel = None if sys.vel is None else sys.vel[perm].copy()
    return dataclasses.replace(sys, pos=sys.pos[perm].copy(), vel=vel,
                               name=sys.name + "-perm")


def cell_sorted(sys: System) -> System:
    """The same system with its atoms sorted by cell: cubic cells of side at
    least rs = rc + skin (the linked-list cells of the cell method), cells in
    z-major order (x fastest), atoms of a cell in their previous order."""
    rs = sys.rc + sys.skin
    nc = np.maximum(np.floor(sys.box / rs).astype(np.int64), 1)
    c = np.minimum((sys.pos / (sys.box / nc)).astype(np.int64), nc - 1)
    cid = (c[:, 2] * nc[1] + c[:, 1]) * nc[0] + c[:, 0]
    perm = np.lexsort((np.arange(sys.n), cid))
    vel = None if sys.vel is None else sys.vel[perm].copy()
    return dataclasses.replace(sys, pos=sys.pos[perm].copy(), vel=vel,
                               name=sys.name + "-cellsorted")


def fcc_system(n: int, rho: float, delta: float, seed: int, rc: float, skin: float,
               T: Optional[float] = None, name: str = "") -> System:
    L = fcc_box(n, rho)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(fcc_sites(n, L), L, delta, rng)
    vel = maxwell(pos.shape[0], T, rng) if T is not None else None
    return System(pos=pos, box=np.array([L, L, L]), rc=rc, skin=skin, vel=vel, name=name)


def vacancy_system(N: int, rho: float, delta: float, rng: np.random.Generator,
                   rc: float, skin: float, T: Optional[float]) -> System:
    """N atoms on a seeded choice of N of the 4 n^3 FCC sites, n = ceil((N/4)^(1/3)),
    in a box of side (N/rho)^(1/3) so that the density is exactly rho."""
    n = int(math.ceil((N / 4.0) ** (1.0 / 3.0) - 1e-12))
    while 4 * n ** 3 < N:
        n += 1
    L = (N / rho) ** (1.0 / 3.0)
    sites = fcc_sites(n, L)
    keep = np.sort(rng.choice(sites.shape[0], size=N, replace=False))
    pos = jitter(sites[keep], L, delta, rng)
    vel = maxwell(N, T, rng) if T is not None else None
    return System(pos=pos, box=np.array([L, L, L]), rc=rc, skin=skin, vel=vel)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes, densities, cutoffs and jitter are those of the five
# benchmark configurations; seeds are fixed here.
# ---------------------------------------------------------------------------

SEEDS = {"lj4k": 1806, "lj131k": 5713, "lj4m": 2018, "lj500k": 4096, "batch512": 512,
         "perm": 77, "lj4m_jit": 2019}


def lj4k() -> System:
    """4,000 atoms (10^3 FCC cells), rho = 1.0, jitter +-0.05, rc = 3.0, skin 0.3."""
    return fcc_system(10, 1.0, 0.05, SEEDS["lj4k"], 3.0, 0.3, name="lj4k")


def lj131k() -> System:
    """131,072 atoms (32^3 FCC cells), rho = 1.0, jitter +-0.1, rc = 3.0, skin 0.3."""
    return fcc_system(32, 1.0, 0.1, SEEDS["lj131k"], 3.0, 0.3, name="lj131k")


def lj4m() -> System:
    """4,000,000 atoms (100^3 FCC cells), rho = 0.85, Maxwell T = 1.0, rc = 2.5, skin 0.3."""
    return fcc_system(100, 0.85, 0.0, SEEDS["lj4m"], 2.5, 0.3, T=1.0, name="lj4m")


def lj4m_jittered() -> System:
    """The 4M-atom fluid's geometry (100^3 FCC cells, rho = 0.85, rc = 2.5,
    skin 0.3) with every coordinate jittered by U(-0.1, 0.1): forces of the
    size of a fluid's instead of a perfect lattice's roundoff (parity checks)."""
    return fcc_system(100, 0.85, 0.1, SEEDS["lj4m_jit"], 2.5, 0.3, name="lj4m-jit")


def lj500k() -> System:
    """500,000 atoms (50^3 FCC cells), rho = 1.0, Maxwell T = 0.7, rc = 3.0, skin 0.3."""
    return fcc_system(50, 1.0, 0.0, SEEDS["lj500k"], 3.0, 0.3, T=0.7, name="lj500k")


def small_fcc(n: int, rho: float, delta: float, seed: int, rc: float = 3.0,
              skin: float = 0.3, T: Optional[float] = None) -> System:
    return fcc_system(n, rho, delta, seed, rc, skin, T=T, name=f"fcc{n}")


def batch512(count: int = 512, nmin: int = 256, nmax: int = 16384, seed: Optional[int] = None,
             delta: float = 0.05, T: float = 1.0, skin: float = 0.3) -> List[System]:
    """Independent systems of uneven size: N ~ U{nmin..nmax}, rho ~ U[0.7, 1.1],
    rc ~ U[2.5, 3.0], each a jittered FCC (with random vacancies) with its own
    SeedSequence child.  A draw whose box is shorter than 2 (rc + skin) is drawn
    again from the same child stream."""
    ss = np.random.SeedSequence(SEEDS["batch512"] if seed is None else seed)
    out = []
    for k, child in enumerate(ss.spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        while True:
            N = int(rng.integers(nmin, nmax + 1))
            rho = float(rng.uniform(0.7, 1.1))
            rc = float(rng.uniform(2.5, 3.0))
            L = (N / rho) ** (1.0 / 3.0)
            if L >= 2.0 * (rc + skin):
                break
        s = vacancy_system(N, rho, delta, rng, rc, skin, T)
        s.name = f"batch{k}"
        out.append(s)
    return out


def aos4(pos: np.ndarray) -> np.ndarray:
    """(N,3) -> (N,4) with a zero pad column: the padded array-of-structures layout."""
    out = np.zeros((pos.shape[0], 4), dtype=np.float64)
    out[:, :3] = pos
    return out


def soa(pos: np.ndarray) -> np.ndarray:
    """(N,3) -> (3,N) contiguous: x block, y block, z block."""
    return np.ascontiguousarray(pos.T)
