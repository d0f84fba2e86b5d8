"""Seeded synthetic inputs for the LJ hot path: lattices, velocities, workloads.

This module serves both the HIP library's callers (tests, bench) and the CPU
oracle's tests.  It holds none of the method's arithmetic (no potential, no
neighbour search, no integration): only the initial states the paper's
benchmarks and cavitation runs start from.

Workload shapes follow the paper's benchmark conditions (Sec. III.B: FCC
lattice, number density 0.5, periodic cube, cutoff 2.5, Eq. 1 truncation) and
its cavitation protocol (Sec. IV.A: liquid at density 0.7, T = 0.9, cutoff 3.0,
uniform expansion of all lengths).  Velocities are Maxwell-Boltzmann at the
stated temperature instead of the paper's fixed speed 0.9 in random directions.

Every array is float64, C-contiguous, shape (n, 3), in caller order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Basis of the conventional FCC cell, in units of the lattice constant.
_FCC_BASIS = np.array([[0.0, 0.0, 0.0],
                       [0.5, 0.5, 0.0],
                       [0.5, 0.0, 0.5],
                       [0.0, 0.5, 0.5]])


def fcc_positions(ncell: int, a: float) -> np.ndarray:
    """FCC sites of an ncell^3 block of conventional cells with constant a.

    Order: z-major over cells (iz, iy, ix), then the four basis sites.
    With a = 2 (density 0.5) every coordinate is an exact integer.
    """
    idx = np.indices((ncell, ncell, ncell)).reshape(3, -1).T[:, ::-1]  # (ix,iy,iz), x fastest
    sites = idx[:, None, :].astype(np.float64) + _FCC_BASIS[None, :, :]
    return np.ascontiguousarray((sites.reshape(-1, 3) * a).astype(np.float64))


def sc_positions(n: int, a: float) -> np.ndarray:
    """Simple-cubic sites of an n^3 block with spacing a (x fastest)."""
    idx = np.indices((n, n, n)).reshape(3, -1).T[:, ::-1]
    return np.ascontiguousarray(idx.astype(np.float64) * a)


def maxwell_boltzmann(n: int, T: float, mass: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian velocities at temperature T with zero total momentum.

    After removing the mean, the set is rescaled so that
    sum(m v^2) / (3n - 3) equals T exactly (3n - 3 degrees of freedom).
    """
    v = rng.standard_normal((n, 3)) * math.sqrt(T / mass)
    v -= v.mean(axis=0)
    t_now = mass * float(np.einsum("ij,ij->", v, v)) / (3 * n - 3)
    v *= math.sqrt(T / t_now)
    return np.ascontiguousarray(v)


def diluted_fcc(n: int, rho: float, rng: np.random.Generator):
    """n sites at density rho in a cube: an FCC block scaled to the box with
    randomly chosen sites removed.  Returns (positions, L)."""
    L = (n / rho) ** (1.0 / 3.0)
    nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-12))
    while 4 * nc ** 3 < n:
        nc += 1
    pos = fcc_positions(nc, L / nc)
    drop = 4 * nc ** 3 - n
    if drop:
        keep = np.sort(rng.permutation(pos.shape[0])[: pos.shape[0] - drop])
        pos = pos[keep]
    return np.ascontiguousarray(pos), L


def jittered(pos: np.ndarray, amp: float, L: float, rng: np.random.Generator) -> np.ndarray:
    """Lattice plus uniform noise in [-amp, amp) per coordinate, wrapped into [0, L)."""
    q = pos + rng.uniform(-amp, amp, size=pos.shape)
    return np.ascontiguousarray(np.mod(q, L))


@dataclass
class Workload:
    """One periodic cubic box and its run parameters (reduced LJ units)."""
    name: str
    pos: np.ndarray
    vel: np.ndarray
    box: tuple
    rc: float = 2.5
    skin: float = 0.3
    dt: float = 0.005
    mass: float = 1.0
    nsteps: int = 100
    T: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def fcc_workload(name: str, ncell: int, seed: int, nsteps: int, rho: float = 0.5,
                 T: float = 1.0, rc: float = 2.5, skin: float = 0.3, dt: float = 0.005) -> Workload:
    """The benchmark shape: perfect FCC at density rho, MB velocities at T."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    if rho == 0.5:
        a = 2.0  # (4/0.5)^(1/3) is exactly 2; avoid the cube-root rounding
    pos = fcc_positions(ncell, a)
    L = ncell * a
    rng = np.random.Generator(np.random.PCG64(seed))
    vel = maxwell_boltzmann(pos.shape[0], T, 1.0, rng)
    return Workload(name, pos, vel, (L, L, L), rc=rc, skin=skin, dt=dt, nsteps=nsteps, T=T,
                    meta={"lattice": "fcc", "ncell": ncell, "rho": rho, "seed": seed})


def small_nve() -> Workload:
    """4000 particles, 10^3 FCC cells, L = 20, T = 1, 100 steps, FP64."""
    return fcc_workload("fcc4000_rho0.5", 10, seed=1, nsteps=100)


def medium_1m() -> Workload:
    """1,048,576 particles, 64^3 FCC cells, L = 128, 1000 steps."""
    return fcc_workload("fcc1M_rho0.5", 64, seed=2, nsteps=1000)


def large_32m() -> Workload:
    """32,000,000 particles, 200^3 FCC cells, L = 400, 500 steps."""
    return fcc_workload("fcc32M_rho0.5", 200, seed=3, nsteps=500)


def cavitation_liquid(n_side: int = 128, seed: int = 4, rho: float = 0.7, T: float = 0.9) -> Workload:
    """Simple-cubic start for the cavitation box (n_side^3 sites at density rho,
    cutoff 3.0).  The liquid is prepared from this by equilibration; the
    expansion by 1.1 per axis follows (see ``expand``)."""
    a = (1.0 / rho) ** (1.0 / 3.0)
    pos = sc_positions(n_side, a)
    L = n_side * a
    rng = np.random.Generator(np.random.PCG64(seed))
    vel = maxwell_boltzmann(pos.shape[0], T, 1.0, rng)
    return Workload(f"sc{n_side}^3_rho{rho}", pos, vel, (L, L, L), rc=3.0, skin=0.3,
                    dt=0.005, nsteps=5000, T=T,
                    meta={"lattice": "sc", "n_side": n_side, "rho": rho, "seed": seed})


@dataclass
class BatchSpec:
    """Per-box sizes of an ensemble of independent boxes."""
    n: np.ndarray      # int64 particle counts
    rho: np.ndarray    # densities
    T: np.ndarray      # temperatures


def batch_spec(nbox: int = 256, seed: int = 5, nmin: int = 2000, nmax: int = 65536,
               rho_lo: float = 0.3, rho_hi: float = 0.8, t_lo: float = 0.7, t_hi: float = 1.2) -> BatchSpec:
    """Uneven ensemble: N_b ~ U{nmin..nmax}, rho_b ~ U[rho_lo, rho_hi], T_b ~ U[t_lo, t_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.integers(nmin, nmax + 1, size=nbox).astype(np.int64)
    rho = rng.uniform(rho_lo, rho_hi, size=nbox)
    T = rng.uniform(t_lo, t_hi, size=nbox)
    return BatchSpec(n, rho, T)


def batch_box(spec: BatchSpec, b: int):
    """State of box b: diluted FCC at rho_b, MB velocities at T_b (seed 1000 + b).
    Returns (positions, velocities, L)."""
    rng = np.random.Generator(np.random.PCG64(1000 + b))
    pos, L = diluted_fcc(int(spec.n[b]), float(spec.rho[b]), rng)
    vel = maxwell_boltzmann(pos.shape[0], float(spec.T[b]), 1.0, rng)
    return pos, vel, L


def free_gas(vmax: float, seed: int = 3):
    """8 particles 10 apart in a box of side 20, so that no pair comes within a
    list radius for hundreds of steps: the first moves at exactly vmax along x,
    the others more slowly in random directions.  Returns (positions,
    velocities, L)."""
    g = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=np.float64)
    q = 5.0 + 10.0 * g
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=(8, 3))
    v *= (0.9 * vmax * rng.uniform(0.1, 1.0, 8) / np.linalg.norm(v, axis=1))[:, None]
    v[0] = (vmax, 0.0, 0.0)
    return q, v, 20.0


def random_box(n: int, L, seed: int, min_sep: float = 0.0) -> np.ndarray:
    """Uniform random positions in [0, L) (no overlap control unless min_sep > 0,
    in which case a jittered cubic lattice with spacing >= min_sep is used)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    if min_sep <= 0.0:
        return np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(n, 3)) * Lv)
    # jittered lattice: spacing s per axis, jitter keeps pairs >= min_sep apart
    m = int(math.ceil(n ** (1.0 / 3.0)))
    s = Lv / m
    amp = max(0.0, (float(s.min()) - min_sep) / 2.0)
    idx = np.indices((m, m, m)).reshape(3, -1).T[:, ::-1][:n].astype(np.float64)
    q = (idx + 0.5) * s + rng.uniform(-amp, amp, size=(n, 3))
    return np.ascontiguousarray(np.mod(q, Lv))


def subcell_field_positions(counts: np.ndarray, L, seed: int, margin: float = 0.01) -> np.ndarray:
    """Positions that realise a given count field: counts[z, y, x] particles drawn
    uniformly inside subcell (x, y, z) of a regular nx*ny*nz grid over the box,
    keeping a relative margin from the subcell faces so that no particle sits
    on a boundary.  Returned in subcell order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.asarray(counts, dtype=np.int64)
    nz, ny, nx = counts.shape
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    e = Lv / np.array([nx, ny, nz])
    z, y, x = np.nonzero(counts)
    k = counts[z, y, x]
    lo = np.repeat(np.stack([x, y, z], axis=1) * e, k, axis=0)
    t = rng.uniform(margin, 1.0 - margin, size=(int(k.sum()), 3))
    return lo + t * e


def bubble_field(shape, p_gas: float, seed: int, liquid: int = 8, gas_max: int = 5, border: bool = False):
    """A random gas/liquid pattern on a subcell grid (shape = (nz, ny, nx)) and a
    count field for it: liquid subcells hold `liquid` particles, gas subcells
    0..gas_max.  With border=True the outermost layer is liquid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gas = rng.uniform(size=shape) < p_gas
    if border:
        gas[0, :, :] = gas[-1, :, :] = False
        gas[:, 0, :] = gas[:, -1, :] = False
        gas[:, :, 0] = gas[:, :, -1] = False
    counts = np.where(gas, rng.integers(0, gas_max + 1, size=shape), liquid)
    return gas, counts
