"""FP64 CPU oracle of the adaptive-relaxation LBM (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``libarlbm_oracle.so`` (plain C, built by
``oracle/build.py``) with ctypes and numpy; it imports nothing from the GPU
library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

ADVECTION, EULER, SWE, REACTIVE = 0, 1, 2, 3
PERIODIC, TRANSMISSIVE, REFLECTIVE = 0, 1, 2


class OraCfg(C.Structure):
    _fields_ = [
        ("system", C.c_int32), ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("bc", C.c_int32 * 4),
        ("cfl", C.c_double), ("eps", C.c_double), ("gamma", C.c_double), ("g", C.c_double),
        ("adv", C.c_double * 3), ("h_dry", C.c_double), ("rho_floor", C.c_double),
        ("p_floor", C.c_double), ("has_bed", C.c_int32), ("omega_fixed_on", C.c_int32),
        ("omega_fixed", C.c_double),
        ("q_heat", C.c_double), ("k_rate", C.c_double), ("t_act", C.c_double),
        ("nz", C.c_int32), ("z0", C.c_double), ("z1", C.c_double), ("bc_z", C.c_int32 * 2),
    ]


_libs = {}


def lib(parallel: bool = False):
    """Load the oracle library, building it first only if it is absent.
    parallel=True: the OpenMP build (same arithmetic, same bits, rows of a
    lattice spread over the host's cores; OMP_NUM_THREADS sets the count)."""
    if parallel not in _libs:
        path = _build.LIB_OMP if parallel else _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.ora_num_fields.argtypes = [C.c_int, C.c_int]
        L.ora_num_fields.restype = C.c_int
        L.ora_create.argtypes = [C.POINTER(OraCfg)]
        L.ora_create.restype = vp
        L.ora_destroy.argtypes = [vp]
        L.ora_init.argtypes = [vp, dp, vp, C.c_double]
        L.ora_init.restype = C.c_int
        L.ora_run.argtypes = [vp, C.c_int64, C.c_double]
        L.ora_run.restype = C.c_int64
        for name in ("ora_moments", "ora_get_f", "ora_last_omega", "ora_omega_field",
                     "ora_nu_field"):
            getattr(L, name).argtypes = [vp, dp]
        L.ora_set_f.argtypes = [vp, dp]
        L.ora_alpha_bar.argtypes = [vp, dp]
        L.ora_threads.argtypes = []
        L.ora_threads.restype = C.c_int
        L.ora_time.argtypes = [vp]
        L.ora_time.restype = C.c_double
        L.ora_steps.argtypes = [vp]
        L.ora_steps.restype = C.c_int64
        L.ora_flags.argtypes = [vp]
        L.ora_flags.restype = C.c_int32
        L.ora_last_scalars.argtypes = [vp, dp, C.POINTER(C.c_double)]
        L.ora_flux.argtypes = [C.POINTER(OraCfg), C.c_int, dp, dp]
        L.ora_max_speed.argtypes = [C.POINTER(OraCfg), C.c_int, dp]
        L.ora_max_speed.restype = C.c_double
        L.ora_left_eigvecs.argtypes = [C.POINTER(OraCfg), C.c_int, dp, dp]
        L.ora_lf_coeffs.argtypes = [C.c_int, dp, C.c_double, dp, dp]
        L.ora_equilibrium.argtypes = [C.POINTER(OraCfg), dp, dp, C.c_double, dp]
        L.ora_source.argtypes = [C.POINTER(OraCfg), dp, dp, dp]
        L.ora_moment_update.argtypes = [C.POINTER(OraCfg), dp, dp, C.c_double, dp]
        _libs[parallel] = L
    return _libs[parallel]


def num_fields(system, dim):
    return lib().ora_num_fields(system, dim)


def make_cfg(system, dim, nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=(PERIODIC,) * 6,
             cfl=0.5, eps=1e-10, gamma=1.4, g=9.81, adv=(1.0, 0.0, 0.0), h_dry=1e-6,
             rho_floor=1e-12, p_floor=1e-12, has_bed=False, omega_fixed=None,
             q_heat=0.0, k_rate=0.0, t_act=0.0, nz=1, z0=0.0, z1=1.0):
    c = OraCfg()
    c.system, c.dim, c.nx, c.ny = system, dim, nx, (ny if dim >= 2 else 1)
    c.nz, c.z0, c.z1 = (nz if dim == 3 else 1), z0, z1
    for i in range(2):
        c.bc_z[i] = bc[4 + i] if len(bc) > 4 else PERIODIC
    c.x0, c.x1, c.y0, c.y1 = x0, x1, y0, y1
    for i in range(4):
        c.bc[i] = bc[i]
    c.cfl, c.eps, c.gamma, c.g = cfl, eps, gamma, g
    for i in range(3):
        c.adv[i] = adv[i] if i < len(adv) else 0.0
    c.h_dry, c.rho_floor, c.p_floor = h_dry, rho_floor, p_floor
    c.has_bed = int(bool(has_bed))
    c.omega_fixed_on = int(omega_fixed is not None)
    c.omega_fixed = float(omega_fixed) if omega_fixed is not None else 0.0
    c.q_heat, c.k_rate, c.t_act = q_heat, k_rate, t_act
    return c


class Lattice:
    """One oracle lattice: ``U0`` has shape (m, nx), (m, ny, nx) or (m, nz, ny, nx)."""

    def __init__(self, cfg: OraCfg, parallel: bool = False):
        self.cfg = cfg
        self._lib = lib(parallel)
        self.d = cfg.dim
        self.m = num_fields(cfg.system, cfg.dim)
        self.Q = 2 * self.d + 1
        self.nx, self.ny, self.nz = cfg.nx, cfg.ny, cfg.nz
        self._h = self._lib.ora_create(C.byref(cfg))
        if not self._h:
            raise ValueError("oracle rejected the configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_destroy(h)
            self._h = None

    def _shape(self, lead):
        if self.d == 3:
            return (lead, self.nz, self.ny, self.nx)
        return (lead, self.ny, self.nx) if self.d == 2 else (lead, self.nx)

    def init(self, U0, bed=None, t0=0.0):
        U0 = np.ascontiguousarray(U0, dtype=np.float64).reshape(self._shape(self.m))
        bp = None
        if bed is not None:
            bed = np.ascontiguousarray(bed, dtype=np.float64)
            self._bed = bed
            bp = bed.ctypes.data_as(C.c_void_p)
        rc = self._lib.ora_init(self._h, U0, bp, float(t0))
        if rc != 0:
            raise RuntimeError(f"ora_init failed: {rc}")
        return self

    def run(self, nsteps, t_final=0.0):
        n = self._lib.ora_run(self._h, int(nsteps), float(t_final))
        if n < 0:
            raise RuntimeError(f"ora_run failed: {n}")
        return n

    def moments(self):
        out = np.empty(self._shape(self.m))
        self._lib.ora_moments(self._h, out)
        return out

    def f(self):
        out = np.empty((self.Q,) + self._shape(self.m))
        self._lib.ora_get_f(self._h, out)
        return out

    def set_f(self, f):
        self._lib.ora_set_f(self._h, np.ascontiguousarray(f, dtype=np.float64))

    def last_omega(self):
        out = np.empty(self._shape(1)[1:])
        self._lib.ora_last_omega(self._h, out)
        return out

    def omega_field(self):
        out = np.empty(self._shape(1)[1:])
        self._lib.ora_omega_field(self._h, out)
        return out

    def nu_field(self):
        out = np.empty(self._shape(1)[1:])
        self._lib.ora_nu_field(self._h, out)
        return out

    def alpha_bar(self):
        out = np.zeros(3)
        self._lib.ora_alpha_bar(self._h, out)
        return out[: self.d]

    @property
    def t(self):
        return self._lib.ora_time(self._h)

    @property
    def steps(self):
        return self._lib.ora_steps(self._h)

    @property
    def flags(self):
        return self._lib.ora_flags(self._h)

    def last_scalars(self):
        ab = np.zeros(3)
        dt = C.c_double()
        self._lib.ora_last_scalars(self._h, ab, C.byref(dt))
        return ab[: self.d], dt.value


def flux(cfg, direction, U):
    m = num_fields(cfg.system, cfg.dim)
    out = np.zeros(m)
    lib().ora_flux(C.byref(cfg), direction, np.ascontiguousarray(U, dtype=np.float64), out)
    return out


def max_speed(cfg, direction, U):
    return lib().ora_max_speed(C.byref(cfg), direction, np.ascontiguousarray(U, dtype=np.float64))


def left_eigvecs(cfg, direction, U):
    m = num_fields(cfg.system, cfg.dim)
    out = np.zeros(m * m)
    lib().ora_left_eigvecs(C.byref(cfg), direction, np.ascontiguousarray(U, dtype=np.float64), out)
    return out.reshape(m, m)


def lf_coeffs(dim, alpha, lam):
    Q = 2 * dim + 1
    a = np.zeros(Q)
    b = np.zeros(Q * dim)
    lib().ora_lf_coeffs(dim, np.ascontiguousarray(alpha, dtype=np.float64), float(lam), a, b)
    return a, b.reshape(Q, dim)


def equilibrium(cfg, U, alpha, lam):
    m = num_fields(cfg.system, cfg.dim)
    Q = 2 * cfg.dim + 1
    out = np.zeros(Q * m)
    lib().ora_equilibrium(C.byref(cfg), np.ascontiguousarray(U, dtype=np.float64),
                          np.ascontiguousarray(alpha, dtype=np.float64), float(lam), out)
    return out.reshape(Q, m)


def source(cfg, U, db=(0.0, 0.0)):
    m = num_fields(cfg.system, cfg.dim)
    out = np.zeros(m)
    lib().ora_source(C.byref(cfg), np.ascontiguousarray(U, dtype=np.float64),
                     np.ascontiguousarray(db, dtype=np.float64), out)
    return out


def moment_update(cfg, sumF, half_dt, db=(0.0, 0.0)):
    """(2.8) for one cell: U = sumF + (dt/2) S(U)."""
    m = num_fields(cfg.system, cfg.dim)
    out = np.zeros(m)
    lib().ora_moment_update(C.byref(cfg), np.ascontiguousarray(sumF, dtype=np.float64),
                            np.ascontiguousarray(db, dtype=np.float64), float(half_dt), out)
    return out


def threads(parallel: bool = False) -> int:
    """Threads the given build runs a step on."""
    return lib(parallel).ora_threads()
