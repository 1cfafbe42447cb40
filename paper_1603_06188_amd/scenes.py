"""Seeded synthetic inputs shaped like the paper's workloads.

This module is the one piece the GPU path and the CPU oracle both use: it
draws particle sets and scene parameters and nothing else.  It holds none of
the method's arithmetic (no weights, transfers, stresses or updates).

The paper (Sec. 6) runs procedural scenes only -- disks/cylinders seeded at
4 particles per cell in 2D, spheres at 8 particles per cell in 3D, many small
bodies, neo-Hookean solids -- and uses no external dataset.  The generators
below stand in for those workloads:

* ``disk2d``     -- rotating elastic disk of Sec. 6.1, resized to a 64x64 grid
* ``cube3d``     -- elastic cube under gravity, 128^3 grid, ~2.1M particles
* ``spheres3d``  -- two colliding spinning spheres, the 3D scene of Sec. 6.5
* ``random_particles`` / ``single_particle`` -- tiny cases for exact checks

Positions are stored as an integer cell index plus an offset inside the cell
in cell units.  For an ``fp32`` scene every floating input (offset, velocity,
B, F, mass) is rounded to a binary32 value first and kept in float64 arrays,
so both sides of a parity test see exactly the same numbers; the absolute
position ``x = (cell + off) * dx`` is exact whenever ``dx`` is a power of two.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Scene:
    name: str
    dim: int
    degree: int                 # 1 multilinear (lagged C in B), 2 quadratic, 3 cubic B-spline
    cells: tuple                # cells per axis (nodes = cells + 1)
    dx: float
    precision: str              # "fp32" or "fp64"
    cell: np.ndarray            # int32 [n, dim]
    off: np.ndarray             # float64 [n, dim], offset in cell units, [0, 1)
    v: np.ndarray               # float64 [n, dim]
    B: np.ndarray               # float64 [n, dim, dim]
    F: np.ndarray               # float64 [n, dim, dim]
    m: np.ndarray               # float64 [n]
    rho0: float                 # rest density; particle volume V = m / rho0
    model: int = 0              # 0 transfer only, 1 neo-Hookean
    mu: float = 0.0
    lam: float = 0.0
    dt: float = 0.0
    gravity: tuple = (0.0, 0.0, 0.0)
    band: tuple = (0, 0, 0, 0, 0, 0)   # sticky band width in nodes: -x,+x,-y,+y,-z,+z
    transfer: int = 0           # affine part carried: 0 APIC, 1 RPIC (skew), 2 PIC (none)
    cfl: float = 0.0            # CFL number for adaptive steps (dt is then their cap)
    steps: int = 1

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    @property
    def x(self) -> np.ndarray:
        """Absolute particle positions in float64."""
        return (self.cell.astype(np.float64) + self.off) * self.dx

    @property
    def V(self) -> np.ndarray:
        return self.m / self.rho0

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, cell=self.cell[idx].copy(), off=self.off[idx].copy(), v=self.v[idx].copy(),
            B=self.B[idx].copy(), F=self.F[idx].copy(), m=self.m[idx].copy())

    def with_state(self, x=None, v=None, B=None, F=None) -> "Scene":
        """Copy with replaced particle state (absolute positions re-split)."""
        s = dataclasses.replace(self)
        if x is not None:
            s.cell, s.off = split_positions(np.asarray(x, dtype=np.float64), self.dx, self.precision)
        if v is not None:
            s.v = _round(np.asarray(v, dtype=np.float64), self.precision)
        if B is not None:
            s.B = _round(np.asarray(B, dtype=np.float64), self.precision)
        if F is not None:
            s.F = _round(np.asarray(F, dtype=np.float64), self.precision)
        return s


def lame(E: float, nu: float):
    """Lame parameters (mu, lambda) from Young's modulus and Poisson ratio."""
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def _round(a: np.ndarray, precision: str) -> np.ndarray:
    if precision == "fp32":
        return a.astype(np.float32).astype(np.float64)
    return a.astype(np.float64)


def split_positions(x: np.ndarray, dx: float, precision: str):
    """Absolute positions -> (int32 cell, offset in [0,1) in cell units)."""
    s = x / dx
    cell = np.floor(s)
    off = _round(s - cell, precision)
    carry = off >= 1.0
    cell = cell + carry
    off = np.where(carry, 0.0, off)
    return cell.astype(np.int32), off


def _stratified(rng, cell_lo: Sequence[int], cell_hi: Sequence[int], per_axis: int, dx: float):
    """One uniform point in each of per_axis^d sub-cells of every cell in the
    box [cell_lo, cell_hi) (cell indices); returns absolute positions."""
    d = len(cell_lo)
    axes = [np.arange(cell_lo[a] * per_axis, cell_hi[a] * per_axis, dtype=np.float64) for a in range(d)]
    mesh = np.meshgrid(*axes, indexing="ij")
    base = np.stack([m.reshape(-1) for m in mesh], axis=1)
    jitter = rng.random(base.shape)
    return (base + jitter) * (dx / per_axis)


def _finish(name, dim, degree, cells, dx, precision, x, v, B, F, m, rho0, **kw) -> Scene:
    cell, off = split_positions(x, dx, precision)
    return Scene(name=name, dim=dim, degree=degree, cells=tuple(int(c) for c in cells), dx=float(dx),
                 precision=precision, cell=cell, off=off, v=_round(v, precision), B=_round(B, precision),
                 F=_round(F, precision), m=_round(m, precision), rho0=float(rho0), **kw)


def disk2d(seed: int = 1, cells: int = 64, radius: float = 0.3, center=(0.5, 0.5), omega: float = 1.0,
           shear: float = 0.2, noise: float = 0.01, precision: str = "fp64", degree: int = 2,
           steps: int = 10) -> Scene:
    """2D disk, 2x2 stratified jitter per cell (4 per cell), mass 1/N,
    velocity = rigid rotation + affine shear (shear * (y - 0.5), 0) + N(0, noise^2);
    B = 0, F = I, transfer only (dt = 0)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / cells
    x = _stratified(rng, (0, 0), (cells, cells), 2, dx)
    c = np.asarray(center, dtype=np.float64)
    keep = np.sum((x - c) ** 2, axis=1) < radius ** 2
    x = x[keep]
    n = x.shape[0]
    r = x - c
    v = np.stack([-omega * r[:, 1], omega * r[:, 0]], axis=1)
    v[:, 0] += shear * (x[:, 1] - 0.5)
    v += rng.normal(0.0, noise, size=v.shape)
    B = np.zeros((n, 2, 2))
    F = np.tile(np.eye(2), (n, 1, 1))
    m = np.full(n, 1.0 / n)
    return _finish("disk2d", 2, degree, (cells, cells), dx, precision, x, v, B, F, m, rho0=1.0,
                   model=0, dt=0.0, steps=steps)


def cube3d(seed: int = 2, cells: int = 128, lo: float = 0.25, hi: float = 0.75, E: float = 1e4,
           nu: float = 0.3, rho: float = 1000.0, vel_sigma: float = 0.1, gravity: float = -9.8,
           floor_band: int = 3, dt: float = 1e-4, precision: str = "fp32", degree: int = 2,
           steps: int = 100) -> Scene:
    """Elastic cube [lo, hi]^3 on the unit cube, 2x2x2 stratified jitter per
    cell (8 per cell), V0 = dx^3/8, m = rho V0, neo-Hookean (E, nu),
    v ~ N(0, vel_sigma^2) per component, B = 0, F = I, gravity along -z,
    sticky floor band of floor_band nodes."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / cells
    clo = int(round(lo * cells))
    chi = int(round(hi * cells))
    x = _stratified(rng, (clo,) * 3, (chi,) * 3, 2, dx)
    n = x.shape[0]
    v = rng.normal(0.0, vel_sigma, size=(n, 3))
    B = np.zeros((n, 3, 3))
    F = np.tile(np.eye(3), (n, 1, 1))
    m = np.full(n, rho * dx ** 3 / 8.0)
    mu, lam = lame(E, nu)
    return _finish("cube3d", 3, degree, (cells,) * 3, dx, precision, x, v, B, F, m, rho0=rho, model=1,
                   mu=mu, lam=lam, dt=dt, gravity=(0.0, 0.0, gravity), band=(0, 0, 0, 0, floor_band, 0),
                   steps=steps)


def spheres3d(seed: int = 3, cells: int = 256, radius: float = 0.2,
              centers=((0.28, 0.5, 0.5), (0.72, 0.5, 0.5)), speed: float = 1.0, omega: float = 5.0,
              E: float = 1e4, nu: float = 0.3, rho: float = 1000.0, dt: float = 1e-4,
              precision: str = "fp32", degree: int = 3, steps: int = 300) -> Scene:
    """Two spheres at 8 particles per cell moving at +-speed along x and
    spinning at omega about z, no gravity (the 3D colliding spheres of Sec. 6.5
    moved to the unit cube)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / cells
    xs, vs = [], []
    for k, c in enumerate(centers):
        c = np.asarray(c, dtype=np.float64)
        lo = np.floor((c - radius) / dx).astype(int)
        hi = np.ceil((c + radius) / dx).astype(int)
        x = _stratified(rng, lo, hi, 2, dx)
        x = x[np.sum((x - c) ** 2, axis=1) < radius ** 2]
        r = x - c
        w = np.array([0.0, 0.0, omega])
        v = np.cross(np.broadcast_to(w, r.shape), r)
        v[:, 0] += speed if k == 0 else -speed
        xs.append(x)
        vs.append(v)
    x = np.concatenate(xs)
    v = np.concatenate(vs)
    n = x.shape[0]
    B = np.zeros((n, 3, 3))
    F = np.tile(np.eye(3), (n, 1, 1))
    m = np.full(n, rho * dx ** 3 / 8.0)
    mu, lam = lame(E, nu)
    return _finish("spheres3d", 3, degree, (cells,) * 3, dx, precision, x, v, B, F, m, rho0=rho, model=1,
                   mu=mu, lam=lam, dt=dt, steps=steps)


def body3d(seed: int, n_target: Optional[int] = None, n_lo: float = 1e3, n_hi: float = 2e5,
           precision: str = "fp32", degree: int = 2, dt: float = 1e-4, gravity: float = -9.8,
           floor_band: int = 3) -> Scene:
    """One small body of a batched workload: a box or a sphere at 8
    particles per cell holding about n_target particles (default: drawn
    log-uniformly in [n_lo, n_hi]), centred in the unit cube on a grid of
    n = clamp(roundup_8(3 x body extent in cells), 32, 128) cells; neo-Hookean
    with E log-uniform in [1e3, 1e5], nu = 0.3, rho = 1000; rigid velocity
    v ~ N(0, 0.5^2) per component plus rotation omega ~ N(0, 2^2); gravity
    along -z, sticky floor."""
    rng = np.random.default_rng(seed)
    if n_target is None:
        n_target = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
    sphere = bool(rng.random() < 0.5)
    body_cells = n_target / 8.0
    if sphere:
        extent = 2.0 * (3.0 * body_cells / (4.0 * np.pi)) ** (1.0 / 3.0)
    else:
        extent = body_cells ** (1.0 / 3.0)
    cells = int(min(max(8 * int(np.ceil(3.0 * extent / 8.0)), 32), 128))
    dx = 1.0 / cells
    c = np.full(3, 0.5)
    half = 0.5 * extent * dx
    lo = np.floor((c - half) / dx).astype(int)
    hi = np.ceil((c + half) / dx).astype(int)
    x = _stratified(rng, lo, hi, 2, dx)
    if sphere:
        x = x[np.sum((x - c) ** 2, axis=1) < half ** 2]
    else:
        x = x[np.all(np.abs(x - c) < half, axis=1)]
    n = x.shape[0]
    w = rng.normal(0.0, 2.0, size=3)
    v = rng.normal(0.0, 0.5, size=3)[None, :] + np.cross(np.broadcast_to(w, x.shape), x - c)
    B = np.zeros((n, 3, 3))
    F = np.tile(np.eye(3), (n, 1, 1))
    m = np.full(n, 1000.0 * dx ** 3 / 8.0)
    E = float(np.exp(rng.uniform(np.log(1e3), np.log(1e5))))
    mu, lam = lame(E, 0.3)
    return _finish("body3d", 3, degree, (cells,) * 3, dx, precision, x, v, B, F, m, rho0=1000.0, model=1,
                   mu=mu, lam=lam, dt=dt, gravity=(0.0, 0.0, gravity), band=(0, 0, 0, 0, floor_band, 0),
                   steps=50)


def many_bodies(n_scenes: int = 512, seed: int = 4, **kw):
    """The batched workload: body3d(seed + scene index) for every scene."""
    return [body3d(seed + k, **kw) for k in range(n_scenes)]


def random_particles(n: int, dim: int = 3, cells: int = 8, degree: int = 2, seed: int = 0,
                     precision: str = "fp64", margin: Optional[float] = None, model: int = 1,
                     E: float = 1e3, nu: float = 0.3, rho: float = 10.0, dt: float = 1e-3,
                     vel_sigma: float = 0.5, b_sigma: float = 0.01, f_sigma: float = 0.1) -> Scene:
    """n particles uniformly inside the grid, away from the faces by
    `margin` cells (default: the kernel support), random v, B and F near I."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / cells
    if margin is None:
        margin = {1: 1.0, 2: 1.5}.get(degree, 2.0)
    x = margin * dx + rng.random((n, dim)) * (cells - 2 * margin) * dx
    v = rng.normal(0.0, vel_sigma, size=(n, dim))
    B = rng.normal(0.0, b_sigma, size=(n, dim, dim))
    F = np.eye(dim)[None] + rng.normal(0.0, f_sigma, size=(n, dim, dim))
    m = 0.5 + rng.random(n)
    mu, lam = lame(E, nu)
    return _finish("random", dim, degree, (cells,) * dim, dx, precision, x, v, B, F, m, rho0=rho,
                   model=model, mu=mu, lam=lam, dt=dt, steps=1)


def single_particle(x, v, B=None, dim: int = 3, cells: int = 8, degree: int = 2, mass: float = 1.0,
                    precision: str = "fp64", dt: float = 0.0) -> Scene:
    """One force-free particle (used for the lone-particle property of Sec. 5.4)."""
    x = np.asarray(x, dtype=np.float64).reshape(1, dim)
    v = np.asarray(v, dtype=np.float64).reshape(1, dim)
    B = np.zeros((1, dim, dim)) if B is None else np.asarray(B, dtype=np.float64).reshape(1, dim, dim)
    F = np.eye(dim)[None].copy()
    m = np.array([mass])
    return _finish("single", dim, degree, (cells,) * dim, 1.0 / cells, precision, x, v, B, F, m, rho0=1.0,
                   model=0, dt=dt, steps=1)


def expected_count_disk(cells: int = 64, radius: float = 0.3) -> float:
    """Expected particle count of disk2d: disk area times 4 per cell."""
    return math.pi * radius ** 2 * cells * cells * 4
