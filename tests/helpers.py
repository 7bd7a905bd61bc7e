"""Shared test helpers: build oracle lattices from seeded workloads, norms."""
import math

import numpy as np

import oracle as O


def ora_cfg_from(p, omega_fixed=None, eps=None, cfl=None, bc=None):
    return O.make_cfg(p.system, p.dim, p.nx, p.ny, p.x0, p.x1, p.y0, p.y1,
                      tuple(bc if bc is not None else p.bc) + tuple(p.bc_z),
                      p.cfl if cfl is None else cfl, p.eps if eps is None else eps,
                      p.gamma, p.g, p.adv, has_bed=p.bed is not None,
                      omega_fixed=omega_fixed, q_heat=p.q_heat, k_rate=p.k_rate, t_act=p.t_act,
                      nz=p.nz, z0=p.z0, z1=p.z1)


def ora_from(p, parallel=False, **kw):
    return O.Lattice(ora_cfg_from(p, **kw), parallel=parallel).init(p.U0, p.bed)


def run_until(L, T):
    """Whole steps until t >= T (the reading that reproduces the paper's tables)."""
    while L.t < T:
        L.run(1)
    return L


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(b ** 2)))


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def fsum(a):
    return math.fsum(np.asarray(a, dtype=np.float64).ravel().tolist())
