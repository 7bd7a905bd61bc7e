"""Seeded synthetic workloads: initial states and problem settings.

This module only draws inputs.  It holds none of the lattice Boltzmann
arithmetic and is shared by the CPU oracle's tests, the GPU parity tests and
the benchmark.  Every generator is deterministic in its seed (numpy PCG64).

Conserved variables, one plane per field, cell-centred points
``x_i = x0 + (i + 1/2) dx``:

* scalar advection: ``u``;
* Euler (gamma-law gas): ``(rho, rho u[, rho v], E)`` with
  ``E = p/(gamma-1) + rho |u|^2 / 2``;
* shallow water: ``(h, h u[, h v])``;
* reactive Euler (Section 5.4): ``(rho, rho u[, rho v], rho E, rho Y)`` with
  ``rho E = p/(gamma-1) + rho |u|^2 / 2 + q rho Y``.

Workloads follow the structure of the paper's experiments (Section 5): smooth
periodic sine waves, piecewise-constant Riemann data, four-quadrant 2D Riemann
data, dry-bed and circular dam breaks.  The shallow-water bed of Gaussian
bumps is a synthetic stand-in (the paper's examples use a flat bed).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ADVECTION, EULER, SWE, REACTIVE = 0, 1, 2, 3
PERIODIC, TRANSMISSIVE, REFLECTIVE = 0, 1, 2
GAMMA = 1.4
GRAVITY = 9.81


@dataclasses.dataclass
class Problem:
    """A lattice problem: settings plus conserved initial data."""
    name: str
    system: int
    dim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc: tuple
    cfl: float
    steps: int
    U0: np.ndarray                 # (m, nx) in 1D, (m, ny, nx) in 2D, float64
    bed: Optional[np.ndarray] = None
    t_final: float = 0.0           # > 0: time-targeted run
    gamma: float = GAMMA
    g: float = GRAVITY
    adv: tuple = (1.0, 0.0)
    eps: float = 1e-10
    q_heat: float = 0.0            # reactive: heat release
    k_rate: float = 0.0            # reactive: Arrhenius rate constant
    t_act: float = 0.0             # reactive: activation temperature
    nz: int = 1                    # 3D: cells along z, extent [z0, z1], boundaries (z-lo, z-hi)
    z0: float = 0.0
    z1: float = 1.0
    bc_z: tuple = (PERIODIC, PERIODIC)

    @property
    def cells(self) -> int:
        return self.nx * (self.ny if self.dim >= 2 else 1) * (self.nz if self.dim == 3 else 1)


def centres(n: int, a: float, b: float) -> np.ndarray:
    dx = (b - a) / n
    return a + (np.arange(n) + 0.5) * dx


def euler_conserved(rho, u, v, p, gamma=GAMMA, dim=2):
    rho, u, v, p = (np.asarray(a, dtype=np.float64) for a in (rho, u, v, p))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    if dim == 1:
        return np.stack([rho, rho * u, E])
    return np.stack([rho, rho * u, rho * v, E])


def reactive_conserved(rho, u, v, p, Y, q_heat, gamma, dim=2):
    rho, u, v, p, Y = (np.asarray(a, dtype=np.float64) for a in (rho, u, v, p, Y))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v) + q_heat * rho * Y
    if dim == 1:
        return np.stack([rho, rho * u, E, rho * Y])
    return np.stack([rho, rho * u, rho * v, E, rho * Y])


def swe_conserved(h, u, v, dim=2):
    h, u, v = (np.asarray(a, dtype=np.float64) for a in (h, u, v))
    if dim == 1:
        return np.stack([h, h * u])
    return np.stack([h, h * u, h * v])


# --------------------------------------------------------------------------
# Configuration 1: smooth periodic advection
# --------------------------------------------------------------------------

def advection_sine(n=256, cfl=0.5, steps=512, t_final=0.0) -> Problem:
    x = centres(n, 0.0, 1.0)
    U0 = np.sin(2.0 * np.pi * x)[None, :]
    return Problem("advection_sine", ADVECTION, 1, n, 1, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, steps, U0, t_final=t_final)


def advection_square(n=400, cfl=0.9, t_final=1.0) -> Problem:
    x = centres(n, 0.0, 1.0)
    U0 = ((x >= 0.25) & (x <= 0.75)).astype(np.float64)[None, :]
    return Problem("advection_square", ADVECTION, 1, n, 1, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, 10 ** 9, U0, t_final=t_final)


def advection_sine_2d(n=64, ax=1.0, ay=0.5, cfl=0.5, steps=64, seed=0) -> Problem:
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi)
    U0 = np.sin(2 * np.pi * (X + Y) + ph)[None]
    return Problem("advection_sine_2d", ADVECTION, 2, n, n, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, steps, U0, adv=(ax, ay))


# --------------------------------------------------------------------------
# Configuration 2: 1D Euler Riemann problems
# --------------------------------------------------------------------------

def riemann_states_1d(seed: int):
    rng = np.random.default_rng(seed)
    L = (rng.uniform(0.125, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
    R = (rng.uniform(0.125, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
    return L, R


def euler_riemann_1d(left, right, n=4096, x0=0.0, x1=1.0, xs=0.5, cfl=0.5, steps=2000,
                     t_final=0.0, gamma=GAMMA, name="euler_riemann_1d") -> Problem:
    x = centres(n, x0, x1)
    L = x < xs
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    U0 = euler_conserved(rho, u, 0 * u, p, gamma, dim=1)
    return Problem(name, EULER, 1, n, 1, x0, x1, 0.0, 1.0,
                   (TRANSMISSIVE,) * 4, cfl, steps, U0, t_final=t_final, gamma=gamma)


def euler_seeded_1d(seed=0, n=4096, cfl=0.5, steps=2000) -> Problem:
    L, R = riemann_states_1d(seed)
    return euler_riemann_1d(L, R, n=n, cfl=cfl, steps=steps, name=f"euler1d_seed{seed}")


SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


def euler_entropy_wave_1d(n=400, cfl=0.6, t_final=1.0) -> Problem:
    x = centres(n, 0.0, 1.0)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    U0 = euler_conserved(rho, np.ones(n), np.zeros(n), np.ones(n), dim=1)
    return Problem("euler_entropy_1d", EULER, 1, n, 1, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, 10 ** 9, U0, t_final=t_final)


# --------------------------------------------------------------------------
# Configuration 3: 2D Euler four-quadrant Riemann problems
# --------------------------------------------------------------------------

def _vacuum(uL, cL, uR, cR, gamma):
    return (uR - uL) >= 2.0 * (cL + cR) / (gamma - 1.0)


def quadrant_states(seed: int, gamma=GAMMA):
    """Per-quadrant (rho, u, v, p), redrawn while any interface would create
    vacuum (Toro's pressure-positivity condition).  Order: quadrants
    1 (x>.5,y>.5), 2 (x<.5,y>.5), 3 (x<.5,y<.5), 4 (x>.5,y<.5)."""
    rng = np.random.default_rng(seed)
    while True:
        q = [(rng.uniform(0.1, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1),
              rng.uniform(0.03, 1.5)) for _ in range(4)]
        c = [math.sqrt(gamma * s[3] / s[0]) for s in q]
        bad = (_vacuum(q[1][1], c[1], q[0][1], c[0], gamma) or   # 2 | 1 along x
               _vacuum(q[2][1], c[2], q[3][1], c[3], gamma) or   # 3 | 4 along x
               _vacuum(q[2][2], c[2], q[1][2], c[1], gamma) or   # 3 / 2 along y
               _vacuum(q[3][2], c[3], q[0][2], c[0], gamma))     # 4 / 1 along y
        if not bad:
            return q


def euler_quadrants_2d(states, n=2048, cfl=0.5, steps=1000, bc=(TRANSMISSIVE,) * 4,
                       gamma=GAMMA, name="euler2d_quadrants") -> Problem:
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    quad = np.where(X > 0.5, np.where(Y > 0.5, 0, 3), np.where(Y > 0.5, 1, 2))
    arr = np.array(states, dtype=np.float64)        # (4, 4)
    prim = arr[quad]                                # (n, n, 4)
    U0 = euler_conserved(prim[..., 0], prim[..., 1], prim[..., 2], prim[..., 3], gamma, dim=2)
    return Problem(name, EULER, 2, n, n, 0.0, 1.0, 0.0, 1.0, tuple(bc), cfl, steps, U0,
                   gamma=gamma)


def euler_seeded_2d(seed=0, n=2048, cfl=0.5, steps=1000) -> Problem:
    return euler_quadrants_2d(quadrant_states(seed), n=n, cfl=cfl, steps=steps,
                              name=f"euler2d_seed{seed}")


def euler_entropy_wave_2d(n=40, cfl=0.3, t_final=0.3) -> Problem:
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y))
    one = np.ones_like(rho)
    U0 = euler_conserved(rho, one, one, one, dim=2)
    return Problem("euler_entropy_2d", EULER, 2, n, n, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, 10 ** 9, U0, t_final=t_final)


# --------------------------------------------------------------------------
# Configuration 4: 2D shallow water over a seeded bed of Gaussian bumps
# --------------------------------------------------------------------------

def swe_bed_params(seed: int, bumps: int = 32):
    rng = np.random.default_rng(seed)
    H = rng.uniform(0.0, 0.8, bumps)
    w = rng.uniform(0.02, 0.1, bumps)
    c = rng.uniform(0.0, 1.0, (bumps, 2))
    disc_c = rng.uniform(0.3, 0.7, 2)
    disc_r = rng.uniform(0.15, 0.3)
    return H, w, c, disc_c, disc_r


def swe_bed_2d(seed=0, n=4096, cfl=0.5, steps=2000, level=1.0) -> Problem:
    H, w, cen, dc, dr = swe_bed_params(seed)
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    bed = np.zeros((n, n))
    for Hm, wm, cm in zip(H, w, cen):
        # exp(-|x - c|^2 / w^2) as an outer product of its two 1D factors
        gx = np.exp(-((x - cm[0]) ** 2) / (wm * wm))
        gy = np.exp(-((x - cm[1]) ** 2) / (wm * wm))
        bed += Hm * np.outer(gy, gx)
    inside = (X - dc[0]) ** 2 + (Y - dc[1]) ** 2 <= dr * dr
    h = np.where(inside, np.maximum(0.0, level - bed), 0.0)
    U0 = swe_conserved(h, 0 * h, 0 * h, dim=2)
    return Problem(f"swe2d_bed_seed{seed}", SWE, 2, n, n, 0.0, 1.0, 0.0, 1.0,
                   (REFLECTIVE,) * 4, cfl, steps, U0, bed=bed)


def swe_dam_break_1d(n=600, cfl=0.9, t_final=0.15) -> Problem:
    x = centres(n, -1.0, 1.0)
    h = np.where(x <= 0.0, 2.0, 0.0)
    U0 = swe_conserved(h, 0 * h, 0 * h, dim=1)
    return Problem("swe_dry_dam_break", SWE, 1, n, 1, -1.0, 1.0, 0.0, 1.0,
                   (TRANSMISSIVE,) * 4, cfl, 10 ** 9, U0, t_final=t_final)


def swe_circular_dam_2d(n=64, cfl=0.4, t_final=0.07) -> Problem:
    x = centres(n, -1.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    h = np.where(np.sqrt(X * X + Y * Y) <= 0.5, 2.0, 1.0)
    U0 = swe_conserved(h, 0 * h, 0 * h, dim=2)
    return Problem("swe_circular_dam", SWE, 2, n, n, -1.0, 1.0, -1.0, 1.0,
                   (TRANSMISSIVE,) * 4, cfl, 10 ** 9, U0, t_final=t_final)


def swe_lake_at_rest_2d(n=64, seed=0, steps=50, cfl=0.5) -> Problem:
    """Flat free surface over a smooth bed, closed basin: the lake at rest."""
    rng = np.random.default_rng(seed)
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    bed = np.zeros((n, n))
    for _ in range(4):
        c = rng.uniform(0.3, 0.7, 2)
        bed += rng.uniform(0.1, 0.3) * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / 0.02)
    h = 1.0 - bed
    U0 = swe_conserved(h, 0 * h, 0 * h, dim=2)
    return Problem("swe_lake_at_rest", SWE, 2, n, n, 0.0, 1.0, 0.0, 1.0,
                   (REFLECTIVE,) * 4, cfl, steps, U0, bed=bed)


def swe_bed_1d(n=512, seed=0, steps=200, cfl=0.5) -> Problem:
    rng = np.random.default_rng(seed)
    x = centres(n, 0.0, 1.0)
    bed = np.zeros(n)
    for _ in range(4):
        bed += rng.uniform(0.1, 0.5) * np.exp(-((x - rng.uniform(0.2, 0.8)) ** 2) / 0.003)
    h = np.where(np.abs(x - 0.5) < 0.3, np.maximum(0.0, 1.0 - bed), 0.0)
    U0 = swe_conserved(h, 0 * h, 0 * h, dim=1)
    return Problem(f"swe1d_bed_seed{seed}", SWE, 1, n, 1, 0.0, 1.0, 0.0, 1.0,
                   (REFLECTIVE,) * 4, cfl, steps, U0, bed=bed)


# --------------------------------------------------------------------------
# Configuration 5: serving mix
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str          # "euler1d" | "euler2d" | "swe2d"
    size: int          # cells (1D) or side (2D)
    steps: int
    seed: int

    def problem(self) -> Problem:
        if self.kind == "euler1d":
            return euler_seeded_1d(self.seed, n=self.size, steps=self.steps)
        if self.kind == "euler2d":
            return euler_seeded_2d(self.seed, n=self.size, steps=self.steps)
        return swe_bed_2d(self.seed, n=self.size, steps=self.steps)


def serving_requests(count=512, rate_hz=200.0, seed=0, n1d=(1024, 65536),
                     side2d=(128, 1024), steps=(500, 5000)) -> List[Request]:
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    kinds = ("euler1d", "euler2d", "swe2d")
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        kind = kinds[int(rng.integers(0, 3))]
        size = int(rng.integers(n1d[0], n1d[1] + 1)) if kind == "euler1d" else \
            int(rng.integers(side2d[0], side2d[1] + 1))
        out.append(Request(i, t, kind, size, int(rng.integers(steps[0], steps[1] + 1)),
                           int(rng.integers(0, 2 ** 31))))
    return out


# --------------------------------------------------------------------------
# Reactive Euler (Section 5.4)
# --------------------------------------------------------------------------

# Example 5.11's kinetics.  The example does not state gamma; 1.2 is the value
# of the paper's other reactive examples (a documented reading).
DET1D = dict(q_heat=50.0, k_rate=145.68913, t_act=50.0, gamma=1.2)
DET1D_BURNT = (2.5706, 6.86089, 80.02055, 0.0)   # (rho, u, p, Y) for x < 2
DET1D_FRESH = (1.0, 0.0, 1.0, 1.0)               # x >= 2
CIRC2D = dict(q_heat=50.0, k_rate=2566.4, t_act=50.0, gamma=1.2)


def reactive_detonation_1d(n=15000, x1=100.0, xs=2.0, cfl=0.9, t_final=7.5, steps=10 ** 9) -> Problem:
    """Example 5.11 data: a burnt driver state left of xs, fresh mixture
    right of it, transmissive ends; dx = x1 / n (the paper: 1/150 on [0,100])."""
    x = centres(n, 0.0, x1)
    L = x < xs
    st = [np.where(L, a, b) for a, b in zip(DET1D_BURNT, DET1D_FRESH)]
    U0 = reactive_conserved(st[0], st[1], 0 * st[1], st[2], st[3], DET1D["q_heat"], DET1D["gamma"], dim=1)
    return Problem("reactive_detonation_1d", REACTIVE, 1, n, 1, 0.0, x1, 0.0, 1.0,
                   (TRANSMISSIVE,) * 4, cfl, steps, U0, t_final=t_final, gamma=DET1D["gamma"],
                   q_heat=DET1D["q_heat"], k_rate=DET1D["k_rate"], t_act=DET1D["t_act"])


def reactive_circle_2d(n=400, cfl=0.9, t_final=0.04, steps=10 ** 9) -> Problem:
    """Example 5.12 data on [-1,1]^2: (rho,u,v,p,Y) = (1,0,0,80,0.2) inside
    the circle of radius 0.6, (1,0,0,10,0.8) outside; transmissive."""
    x = centres(n, -1.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    inside = X * X + Y * Y <= 0.36
    p = np.where(inside, 80.0, 10.0)
    Yf = np.where(inside, 0.2, 0.8)
    one = np.ones_like(X)
    U0 = reactive_conserved(one, 0 * one, 0 * one, p, Yf, CIRC2D["q_heat"], CIRC2D["gamma"], dim=2)
    return Problem("reactive_circle_2d", REACTIVE, 2, n, n, -1.0, 1.0, -1.0, 1.0,
                   (TRANSMISSIVE,) * 4, cfl, steps, U0, t_final=t_final, gamma=CIRC2D["gamma"],
                   q_heat=CIRC2D["q_heat"], k_rate=CIRC2D["k_rate"], t_act=CIRC2D["t_act"])


def reactive_seeded_1d(seed=0, n=2048, cfl=0.5, steps=1000) -> Problem:
    """Seeded reactive Riemann data on [0,1]: a hot, partly burnt state left
    of 0.5 and a cool fresh mixture right of it, with kinetics drawn so that
    the left state burns within a few hundred steps."""
    rng = np.random.default_rng(1000 + seed)
    gamma = 1.2
    left = (rng.uniform(1.0, 2.5), rng.uniform(0.0, 2.0), rng.uniform(20.0, 80.0), rng.uniform(0.0, 0.5))
    right = (rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(0.5, 2.0), rng.uniform(0.8, 1.0))
    q_heat = rng.uniform(10.0, 50.0)
    t_act = rng.uniform(10.0, 40.0)
    k_rate = rng.uniform(50.0, 500.0)
    x = centres(n, 0.0, 1.0)
    L = x < 0.5
    st = [np.where(L, a, b) for a, b in zip(left, right)]
    U0 = reactive_conserved(st[0], st[1], 0 * st[1], st[2], st[3], q_heat, gamma, dim=1)
    return Problem(f"reactive1d_seed{seed}", REACTIVE, 1, n, 1, 0.0, 1.0, 0.0, 1.0,
                   (TRANSMISSIVE,) * 4, cfl, steps, U0, gamma=gamma,
                   q_heat=q_heat, k_rate=k_rate, t_act=t_act)


def reactive_seeded_2d(seed=0, n=256, cfl=0.5, steps=200, bc=(TRANSMISSIVE,) * 4) -> Problem:
    """Seeded 2D reactive data on [0,1]^2: hot burnt pockets (Gaussian bumps
    of pressure and burnt fraction) in a fresh mixture, with a shear flow."""
    rng = np.random.default_rng(2000 + seed)
    gamma = 1.2
    q_heat = rng.uniform(10.0, 50.0)
    t_act = rng.uniform(10.0, 40.0)
    k_rate = rng.uniform(50.0, 500.0)
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    p = np.full_like(X, rng.uniform(0.5, 2.0))
    burnt = np.zeros_like(X)
    for _ in range(4):
        cx, cy = rng.uniform(0.2, 0.8, size=2)
        w = rng.uniform(0.04, 0.1)
        g = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / w ** 2)
        p = p + rng.uniform(20.0, 60.0) * g
        burnt = np.maximum(burnt, g)
    Yf = 1.0 - 0.9 * burnt
    rho = rng.uniform(0.8, 1.5) + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    u = rng.uniform(-0.5, 0.5) * np.sin(2 * np.pi * Y)
    v = rng.uniform(-0.5, 0.5) * np.sin(2 * np.pi * X)
    U0 = reactive_conserved(rho, u, v, p, Yf, q_heat, gamma, dim=2)
    return Problem(f"reactive2d_seed{seed}", REACTIVE, 2, n, n, 0.0, 1.0, 0.0, 1.0,
                   bc, cfl, steps, U0, gamma=gamma, q_heat=q_heat, k_rate=k_rate, t_act=t_act)


def reactive_uniform(n=16, dim=1, rho=1.0, u=0.3, v=-0.2, p=1.0, Y=1.0, q_heat=20.0, k_rate=50.0,
                     t_act=5.0, gamma=1.2, cfl=0.5, steps=100) -> Problem:
    """A spatially uniform reacting state with periodic boundaries: every cell
    follows the same ODE for rho Y while rho, rho u and rho E stay fixed."""
    ny = n if dim == 2 else 1
    shape = (ny, n) if dim == 2 else (n,)
    one = np.ones(shape)
    U0 = reactive_conserved(rho * one, u * one, (v if dim == 2 else 0.0) * one, p * one, Y * one,
                            q_heat, gamma, dim=dim)
    return Problem("reactive_uniform", REACTIVE, dim, n, ny, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, steps, U0, gamma=gamma, q_heat=q_heat, k_rate=k_rate, t_act=t_act)


# --------------------------------------------------------------------------
# Three dimensions (D3Q7; the formulation of Section 2.3 is general in d)
# --------------------------------------------------------------------------

def euler3_conserved(rho, u, v, w, p, gamma=GAMMA):
    rho, u, v, w, p = (np.asarray(a, dtype=np.float64) for a in (rho, u, v, w, p))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def _grid3(n):
    x = centres(n, 0.0, 1.0)
    return np.meshgrid(x, x, x, indexing="ij")[::-1]   # X, Y, Z with arrays [z][y][x]


def advection_sine_3d(n=32, a=(1.0, 0.5, 0.25), cfl=0.5, steps=64, amp=1.0) -> Problem:
    Z, Y, X = np.meshgrid(*(centres(n, 0.0, 1.0),) * 3, indexing="ij")
    U0 = amp * np.sin(2 * np.pi * (X + Y + Z))[None]
    return Problem("advection_sine_3d", ADVECTION, 3, n, n, 0.0, 1.0, 0.0, 1.0,
                   (PERIODIC,) * 4, cfl, steps, U0, adv=tuple(a), nz=n, bc_z=(PERIODIC, PERIODIC))


def euler_entropy_wave_3d(n=16, cfl=0.3, t_final=0.2, amp=0.2) -> Problem:
    """rho = 1 + amp sin(2 pi (x + y + z)), u = v = w = p = 1, periodic: the
    exact solution translates by (t, t, t)."""
    Z, Y, X = np.meshgrid(*(centres(n, 0.0, 1.0),) * 3, indexing="ij")
    rho = 1.0 + amp * np.sin(2 * np.pi * (X + Y + Z))
    one = np.ones_like(rho)
    U0 = euler3_conserved(rho, one, one, one, one)
    return Problem("euler_entropy_3d", EULER, 3, n, n, 0.0, 1.0, 0.0, 1.0, (PERIODIC,) * 4, cfl, 10 ** 9,
                   U0, t_final=t_final, nz=n, bc_z=(PERIODIC, PERIODIC))


def octant_states(seed: int, gamma=GAMMA):
    """Eight (rho, u, v, w, p) states drawn like the four-quadrant data."""
    rng = np.random.default_rng(3000 + seed)
    return [(rng.uniform(0.1, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1),
             rng.uniform(0.03, 1.5)) for _ in range(8)]


def euler_octants_3d(seed=0, n=64, cfl=0.5, steps=100, bc=(TRANSMISSIVE,) * 6) -> Problem:
    """3D Riemann data: one seeded state per octant around (0.5, 0.5, 0.5)."""
    st = octant_states(seed)
    Z, Y, X = np.meshgrid(*(centres(n, 0.0, 1.0),) * 3, indexing="ij")
    idx = (X >= 0.5).astype(int) + 2 * (Y >= 0.5).astype(int) + 4 * (Z >= 0.5).astype(int)
    arr = np.array(st)[idx]                       # (n, n, n, 5)
    U0 = euler3_conserved(arr[..., 0], arr[..., 1], arr[..., 2], arr[..., 3], arr[..., 4])
    return Problem(f"euler3d_seed{seed}", EULER, 3, n, n, 0.0, 1.0, 0.0, 1.0, tuple(bc[:4]), cfl, steps, U0,
                   nz=n, bc_z=tuple(bc[4:6]))


def euler_sphere_3d(n=48, cfl=0.5, steps=40, bc=(REFLECTIVE,) * 6) -> Problem:
    """A 3D blast: (rho, p) = (1, 1) inside the sphere of radius 0.25 around
    the centre, (0.125, 0.1) outside, at rest; symmetric under every axis
    permutation and reflection."""
    Z, Y, X = np.meshgrid(*(centres(n, 0.0, 1.0),) * 3, indexing="ij")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    inside = r2 <= 0.0625
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    z = np.zeros_like(rho)
    U0 = euler3_conserved(rho, z, z, z, p)
    return Problem("euler_sphere_3d", EULER, 3, n, n, 0.0, 1.0, 0.0, 1.0, tuple(bc[:4]), cfl, steps, U0,
                   nz=n, bc_z=tuple(bc[4:6]))


def reactive_sphere_3d(n=32, cfl=0.5, steps=30, bc=(TRANSMISSIVE,) * 6) -> Problem:
    """Example 5.12's reactive data on a sphere: (rho,u,v,w,p,Y) = (1,0,0,0,80,0.2)
    inside radius 0.6 of [-1,1]^3, (1,0,0,0,10,0.8) outside."""
    Z, Y, X = np.meshgrid(*(centres(n, -1.0, 1.0),) * 3, indexing="ij")
    inside = X * X + Y * Y + Z * Z <= 0.36
    p = np.where(inside, 80.0, 10.0)
    Yf = np.where(inside, 0.2, 0.8)
    one = np.ones_like(p)
    g = CIRC2D["gamma"]
    E = p / (g - 1.0) + CIRC2D["q_heat"] * one * Yf
    z = np.zeros_like(p)
    U0 = np.stack([one, z, z, z, E, one * Yf])
    return Problem("reactive_sphere_3d", REACTIVE, 3, n, n, -1.0, 1.0, -1.0, 1.0, tuple(bc[:4]), cfl, steps, U0,
                   gamma=g, q_heat=CIRC2D["q_heat"], k_rate=CIRC2D["k_rate"], t_act=CIRC2D["t_act"],
                   nz=n, z0=-1.0, z1=1.0, bc_z=tuple(bc[4:6]))
