"""Seeded synthetic initial conditions for the five benchmark workloads.

This module only builds inputs: grid sizes, extents, boundary kinds, solid masks, initial
states and run settings.  It holds none of the scheme's arithmetic, so both the GPU path and the
oracle-based tests can draw their inputs from it.

State arrays are float64 ``[4, ny, nx]`` = (rho, rho*u, rho*v, p), x fastest.  Densities are set
by testing cell centres (no volume fractions).  Unless stated, u = v = p = 0 at the start, as in
the paper's dam-break and hydrostatic tests (Sec. 3.2, 3.3).  The paper measures no public
dataset; these setups scale its tests up and stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

WALL = 0
PERIODIC = 1


@dataclass
class Tank:
    nx: int
    ny: int
    lx: float
    ly: float
    q: np.ndarray                      # float64 [4, ny, nx]: rho, rho*u, rho*v, p
    gx: float = 0.0
    gy: float = -9.81
    beta: float = 1100.0
    bc: tuple = (WALL, WALL, WALL, WALL)   # x-, x+, y-, y+
    solid: np.ndarray | None = None         # uint8 [ny, nx], 1 = solid

    @property
    def fluid_cells(self) -> int:
        n = self.nx * self.ny
        return n if self.solid is None else int(n - np.count_nonzero(self.solid))


@dataclass
class Workload:
    name: str
    tanks: list
    dt: float
    steps: int
    max_pseudo: int
    tol: float = 0.0                  # <= 0: exactly max_pseudo iterations per step
    stages: int = 3
    alpha: tuple = (1.0 / 3.0, 0.5, 1.0)
    cfl: float = 0.48
    k: float = 1.0
    local_dtau: bool = True
    bdf: int = 1
    precision: str = "f64"            # "f64" or "mixed"
    note: dict = field(default_factory=dict)

    @property
    def fluid_cells(self) -> int:
        return sum(t.fluid_cells for t in self.tanks)


def _centres(n: int, length: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


def _state(rho: np.ndarray, u=None, v=None, p=None) -> np.ndarray:
    ny, nx = rho.shape
    q = np.zeros((4, ny, nx), dtype=np.float64)
    q[0] = rho
    if u is not None:
        q[1] = rho * u
    if v is not None:
        q[2] = rho * v
    if p is not None:
        q[3] = p
    return q


def hydrostatic(nx: int = 64, ny: int = 64) -> Workload:
    """Two-layer tank on the unit square: rho = 1000 below y = 0.5, 1 above; g = -9.81,
    beta = 1e3, walls; 10 steps of dt = 1e-3 with exactly 200 pseudo-iterations each; FP64."""
    yc = _centres(ny, 1.0)
    rho = np.where(yc < 0.5, 1000.0, 1.0)[:, None] * np.ones((1, nx))
    t = Tank(nx, ny, 1.0, 1.0, _state(rho), gy=-9.81, beta=1000.0)
    return Workload("hydrostatic_64x64", [t], dt=1e-3, steps=10, max_pseudo=200)


def dam_break(nx: int = 512, ny: int = 256, precision: str = "f64") -> Workload:
    """Dam break on a 4 x 2 domain: water (rho = 1000) at x < 1, y < 1, air (rho = 1)
    elsewhere, g = -9.81, walls, beta = 1100; dt = 1e-4 for 500 steps, up to 100
    pseudo-iterations per step to an RMS residual of 1e-6."""
    xc, yc = _centres(nx, 4.0), _centres(ny, 2.0)
    rho = np.where((xc[None, :] < 1.0) & (yc[:, None] < 1.0), 1000.0, 1.0)
    t = Tank(nx, ny, 4.0, 2.0, _state(rho), gy=-9.81, beta=1100.0)
    return Workload(f"dam_break_{nx}x{ny}", [t], dt=1e-4, steps=500, max_pseudo=100, tol=1e-6,
                    precision=precision)


def rayleigh_taylor(nx: int = 256, ny: int = 1024, seed: int = 3,
                    precision: str = "mixed") -> Workload:
    """Rayleigh-Taylor on a 1 x 4 domain: rho = 3 above y = 2 + 0.05 cos(2 pi x), 1 below;
    seeded uniform noise of amplitude 1e-3 on v; g = -1; periodic in x, walls in y;
    beta = 100; dt = 5e-4 for 2000 steps, up to 100 pseudo-iterations to 1e-6."""
    xc, yc = _centres(nx, 1.0), _centres(ny, 4.0)
    heavy = yc[:, None] > 2.0 + 0.05 * np.cos(2.0 * math.pi * xc[None, :])
    rho = np.where(heavy, 3.0, 1.0)
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1e-3, 1e-3, size=(ny, nx))
    t = Tank(nx, ny, 1.0, 4.0, _state(rho, v=v), gy=-1.0, beta=100.0,
             bc=(PERIODIC, PERIODIC, WALL, WALL))
    return Workload(f"rayleigh_taylor_{nx}x{ny}", [t], dt=5e-4, steps=2000, max_pseudo=100,
                    tol=1e-6, precision=precision)


SLOSH_SIDES = tuple(range(32, 257, 16))   # 32, 48, ..., 256 (15 values)


def sloshing_ensemble(n_tanks: int = 512, seed: int = 4, h: float = 1.0 / 128.0,
                      precision: str = "mixed") -> Workload:
    """Batched sloshing: independent closed tanks at rest with a tilted interface.  Per tank,
    drawn in this order: sides nx, ny from {32, 48, ..., 256}, density ratio log-uniform in
    [1.1, 1000], mean fill level uniform in [0.3, 0.7] of the height, and a tilt a uniform in
    [-0.5, 0.5]: the heavy fluid (rho = ratio) lies below y = ly (fill + 0.2 a (2 x / lx - 1)),
    the light fluid (rho = 1) above, so the interface is displaced by up to 0.1 ly at the side
    walls.  Cell size h, beta = 1100, g = -9.81, dt = 1e-3, 10 steps x 50 pseudo-iterations."""
    rng = np.random.default_rng(seed)
    tanks = []
    for _ in range(n_tanks):
        nx = int(rng.choice(SLOSH_SIDES))
        ny = int(rng.choice(SLOSH_SIDES))
        ratio = float(math.exp(rng.uniform(math.log(1.1), math.log(1000.0))))
        fill = float(rng.uniform(0.3, 0.7))
        tilt = float(rng.uniform(-0.5, 0.5))
        lx, ly = nx * h, ny * h
        xc, yc = _centres(nx, lx), _centres(ny, ly)
        surface = ly * (fill + 0.2 * tilt * (2.0 * xc / lx - 1.0))
        rho = np.where(yc[:, None] < surface[None, :], ratio, 1.0)
        tanks.append(Tank(nx, ny, lx, ly, _state(rho), gy=-9.81, beta=1100.0))
    return Workload(f"sloshing_ensemble_{n_tanks}", tanks, dt=1e-3, steps=10, max_pseudo=50,
                    precision=precision)


def obstacle_dam_break(n: int = 4096, precision: str = "f64") -> Workload:
    """Dam break with an obstacle on a 4 x 4 domain: water at x < 1, y < 2, solid cells at
    2.5 < x < 2.7, y < 0.3 (centre test), density ratio 1000:1, beta = 1100; dt = 2e-5 for 200
    steps with exactly 50 pseudo-iterations each."""
    xc, yc = _centres(n, 4.0), _centres(n, 4.0)
    rho = np.where((xc[None, :] < 1.0) & (yc[:, None] < 2.0), 1000.0, 1.0)
    solid = ((xc[None, :] > 2.5) & (xc[None, :] < 2.7) & (yc[:, None] < 0.3)).astype(np.uint8)
    t = Tank(n, n, 4.0, 4.0, _state(rho), gy=-9.81, beta=1100.0, solid=solid)
    return Workload(f"obstacle_dam_break_{n}x{n}", [t], dt=2e-5, steps=200, max_pseudo=50,
                    precision=precision)


def random_state(nx: int, ny: int, seed: int, rho_range=(1.0, 1000.0), vel=1.0,
                 p_scale=100.0) -> np.ndarray:
    """A seeded rough state for unit tests: two-level density with random velocity and
    pressure fields."""
    rng = np.random.default_rng(seed)
    rho = np.where(rng.random((ny, nx)) < 0.5, rho_range[0], rho_range[1])
    rho = rho * rng.uniform(0.9, 1.1, size=(ny, nx))
    u = rng.uniform(-vel, vel, size=(ny, nx))
    v = rng.uniform(-vel, vel, size=(ny, nx))
    p = rng.uniform(-p_scale, p_scale, size=(ny, nx))
    return _state(rho, u=u, v=v, p=p)
