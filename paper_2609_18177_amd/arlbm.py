"""Thin ctypes binding of libarlbm (the C ABI in include/arlbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (caller-owned buffers) and the HIP stream.
The library must be built (``__graft_entry__.build()``); loading fails loudly
otherwise, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libarlbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "arlbm.h")

ADVECTION, EULER, SWE, REACTIVE = 0, 1, 2, 3
PERIODIC, TRANSMISSIVE, REFLECTIVE = 0, 1, 2
F32, F64 = 0, 1
OMEGA_ADAPTIVE, OMEGA_FIXED = 0, 1
ABI_VERSION = 4

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EPOSITIVITY, EDEGENERATE, EBUSY, EBUDGET = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
FLAG_NONFINITE, FLAG_POSITIVITY, FLAG_DEGENERATE = 1, 2, 4


class ArlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"arlbm error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("system", C.c_int32), ("dim", C.c_int32), ("precision", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("z0", C.c_double), ("z1", C.c_double),
        ("bc", C.c_int32 * 6),
        ("cfl", C.c_double), ("eps", C.c_double), ("gamma", C.c_double), ("g", C.c_double),
        ("adv_speed", C.c_double * 3), ("h_dry", C.c_double), ("rho_floor", C.c_double),
        ("p_floor", C.c_double), ("has_bed", C.c_int32), ("omega_mode", C.c_int32),
        ("omega_fixed", C.c_double),
        ("q_heat", C.c_double), ("k_rate", C.c_double), ("t_act", C.c_double),
    ]


class Sizes(C.Structure):
    _fields_ = [("f_bytes", C.c_size_t), ("u_bytes", C.c_size_t), ("bed_bytes", C.c_size_t),
                ("scalar_bytes", C.c_size_t), ("omega_bytes", C.c_size_t), ("total_bytes", C.c_size_t),
                ("alignment", C.c_size_t), ("m", C.c_int32), ("q", C.c_int32)]


class Buffers(C.Structure):
    _fields_ = [("f", C.c_void_p * 2), ("u", C.c_void_p * 2), ("bed", C.c_void_p),
                ("scalars", C.c_void_p), ("omega", C.c_void_p)]


class Status(C.Structure):
    _fields_ = [("t", C.c_double), ("last_dt", C.c_double), ("abar", C.c_double * 3),
                ("step", C.c_int64), ("first_bad_step", C.c_int64), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]


class Completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("flags", C.c_uint32), ("steps", C.c_int64),
                ("first_bad_step", C.c_int64), ("t", C.c_double), ("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("U", C.POINTER(C.c_double)), ("u_count", C.c_int64)]


_lib = None


def lib():
    """Load libarlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        sig = {
            "arlbm_config_init": ([C.POINTER(Config)], C.c_int),
            "arlbm_query_sizes": ([C.POINTER(Config), C.POINTER(Sizes)], C.c_int),
            "arlbm_create": ([C.POINTER(Config), C.POINTER(Buffers), vp, C.POINTER(vp)], C.c_int),
            "arlbm_set_state": ([vp, dp, dp, C.c_double], C.c_int),
            "arlbm_set_state_device": ([vp, vp, vp, C.c_double], C.c_int),
            "arlbm_step": ([vp, C.c_int64], C.c_int),
            "arlbm_sync": ([vp, C.POINTER(Status)], C.c_int),
            "arlbm_step_until": ([vp, C.c_double, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
            "arlbm_read_moments": ([vp, dp], C.c_int),
            "arlbm_set_omega_export": ([vp, C.c_int], C.c_int),
            "arlbm_read_omega": ([vp, dp], C.c_int),
            "arlbm_conservation": ([vp, dp], C.c_int),
            "arlbm_conservation_noalloc": ([vp, dp], C.c_int),
            "arlbm_state_bytes": ([vp, C.POINTER(C.c_size_t)], C.c_int),
            "arlbm_save_state": ([vp, vp, C.c_size_t], C.c_int),
            "arlbm_load_state": ([vp, vp, C.c_size_t], C.c_int),
            "arlbm_destroy": ([vp], C.c_int),
            "arlbm_last_error": ([vp], C.c_char_p),
            "arlbm_server_create": ([C.c_size_t, C.c_int32, vp, C.POINTER(vp)], C.c_int),
            "arlbm_server_submit": ([vp, C.POINTER(Config), dp, dp, C.c_int64, C.POINTER(C.c_uint64)], C.c_int),
            "arlbm_server_submit_state": ([vp, C.POINTER(Config), vp, C.c_size_t, C.c_int64,
                                           C.POINTER(C.c_uint64)], C.c_int),
            "arlbm_server_iterate": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
            "arlbm_server_iterate_n": ([vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32)], C.c_int),
            "arlbm_server_result_into": ([vp, C.c_uint64, dp, C.c_int64], C.c_int),
            "arlbm_server_poll": ([vp, C.POINTER(Completion), C.c_int32, C.POINTER(C.c_int32)], C.c_int),
            "arlbm_server_memory": ([vp, C.POINTER(C.c_size_t)], C.c_int),
            "arlbm_server_pool_bytes": ([vp, C.POINTER(C.c_size_t)], C.c_int),
            "arlbm_server_destroy": ([vp], C.c_int),
            "arlbm_step_kernel_vgprs": ([C.c_int32, C.c_int32, C.c_int32], C.c_int),
            "arlbm_plan_schedule": ([C.POINTER(Config), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)], C.c_int),
            "arlbm_plan_groups": ([C.POINTER(Config), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32)], C.c_int),
            "arlbm_kernel_exp": ([C.c_double], C.c_double),
            "arlbm_kernel_expf": ([C.c_float], C.c_float),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def last_error(handle=None) -> str:
    s = lib().arlbm_last_error(handle)
    return s.decode() if s else ""


def _check(rc, handle=None):
    if rc != OK:
        raise ArlbmError(rc, last_error(handle))
    return rc


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def config_from(problem=None, precision=F32, omega_fixed=None, **over) -> Config:
    """Build an arlbm_config from a workloads.Problem (or keywords)."""
    c = Config()
    _check(lib().arlbm_config_init(C.byref(c)))
    if problem is not None:
        c.system, c.dim = problem.system, problem.dim
        c.nx, c.ny = problem.nx, (problem.ny if problem.dim >= 2 else 1)
        c.nz = problem.nz if problem.dim == 3 else 1
        c.x0, c.x1, c.y0, c.y1 = problem.x0, problem.x1, problem.y0, problem.y1
        c.z0, c.z1 = problem.z0, problem.z1
        for i in range(4):
            c.bc[i] = problem.bc[i]
        c.bc[4], c.bc[5] = problem.bc_z
        c.cfl, c.eps, c.gamma, c.g = problem.cfl, problem.eps, problem.gamma, problem.g
        for i in range(3):
            c.adv_speed[i] = problem.adv[i] if i < len(problem.adv) else 0.0
        c.has_bed = int(problem.bed is not None)
        c.q_heat, c.k_rate, c.t_act = problem.q_heat, problem.k_rate, problem.t_act
    c.precision = precision
    if omega_fixed is not None:
        c.omega_mode, c.omega_fixed = OMEGA_FIXED, float(omega_fixed)
    for k, v in over.items():
        if k == "bc":
            for i in range(len(v)):
                c.bc[i] = v[i]
        else:
            setattr(c, k, v)
    return c


def query_sizes(cfg: Config) -> Sizes:
    s = Sizes()
    _check(lib().arlbm_query_sizes(C.byref(cfg), C.byref(s)))
    return s


class Lattice:
    """One lattice on the GPU.

    owner="torch": the device buffers are torch tensors (caller-owned, kept
    alive here); owner="library": libarlbm allocates them.  The HIP stream is
    torch's current stream unless one is given.
    """

    def __init__(self, cfg: Config, owner: str = "torch", stream=None):
        import torch  # device memory and streams only

        self.cfg = cfg
        self.sizes = query_sizes(cfg)
        self.m, self.q = self.sizes.m, self.sizes.q
        self.dim, self.nx, self.ny, self.nz = cfg.dim, cfg.nx, cfg.ny, cfg.nz
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        raw_stream = C.c_void_p(stream.cuda_stream)
        self._tensors = []
        bufs = None
        if owner == "torch":
            def alloc(nbytes):
                t = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device="cuda")
                p = t.data_ptr()
                off = (-p) % 256
                self._tensors.append(t)
                return p + off
            b = Buffers()
            for i in range(2):
                b.f[i] = alloc(self.sizes.f_bytes)
                b.u[i] = alloc(self.sizes.u_bytes)
            b.bed = alloc(self.sizes.bed_bytes) if cfg.has_bed else None
            b.scalars = alloc(self.sizes.scalar_bytes)
            b.omega = None
            bufs = C.byref(b)
        h = C.c_void_p()
        _check(lib().arlbm_create(C.byref(cfg), bufs, raw_stream, C.byref(h)))
        self._h = h

    # ------------------------------------------------------------------
    def _shape(self, lead):
        if self.dim == 3:
            return (lead, self.nz, self.ny, self.nx)
        return (lead, self.ny, self.nx) if self.dim == 2 else (lead, self.nx)

    def set_state(self, U0: np.ndarray, bed: Optional[np.ndarray] = None, t0: float = 0.0):
        U0 = np.ascontiguousarray(U0, dtype=np.float64).reshape(self._shape(self.m))
        bed = None if bed is None else np.ascontiguousarray(bed, dtype=np.float64)
        _check(lib().arlbm_set_state(self._h, _dptr(U0), _dptr(bed), float(t0)), self._h)
        return self

    def set_state_device(self, U0_dev, bed_dev=None, t0: float = 0.0):
        """U0_dev / bed_dev: float64 CUDA tensors (m planes / one plane)."""
        _check(lib().arlbm_set_state_device(self._h, C.c_void_p(U0_dev.data_ptr()),
                                            C.c_void_p(bed_dev.data_ptr()) if bed_dev is not None else None,
                                            float(t0)), self._h)
        return self

    def step(self, n: int = 1):
        _check(lib().arlbm_step(self._h, int(n)), self._h)

    def step_until(self, t_final: float, max_steps: int = 10 ** 9) -> int:
        """Whole steps until t >= t_final; returns the number of steps taken."""
        n = C.c_int64()
        _check(lib().arlbm_step_until(self._h, float(t_final), int(max_steps), C.byref(n)), self._h)
        return n.value

    def sync(self, check: bool = True, strict: bool = False) -> dict:
        """Wait for the stream.  With check, raise on a non-finite or
        degenerate state (and, with strict, on the advisory positivity flag)."""
        st = Status()
        rc = lib().arlbm_sync(self._h, C.byref(st))
        if check and (rc != EPOSITIVITY or strict):
            _check(rc, self._h)
        return {"rc": rc, "t": st.t, "last_dt": st.last_dt, "abar": [st.abar[0], st.abar[1], st.abar[2]][: self.dim],
                "step": st.step, "flags": st.flags, "first_bad_step": st.first_bad_step}

    def moments(self) -> np.ndarray:
        out = np.empty(self._shape(self.m))
        _check(lib().arlbm_read_moments(self._h, _dptr(out)), self._h)
        return out

    def set_omega_export(self, on: bool = True):
        _check(lib().arlbm_set_omega_export(self._h, int(bool(on))), self._h)

    def omega(self) -> np.ndarray:
        out = np.empty(self._shape(1)[1:])
        _check(lib().arlbm_read_omega(self._h, _dptr(out)), self._h)
        return out

    def conservation(self) -> np.ndarray:
        out = np.empty(self.m)
        _check(lib().arlbm_conservation(self._h, _dptr(out)), self._h)
        return out

    def conservation_noalloc(self) -> np.ndarray:
        """arlbm_conservation with the library's device scratch array."""
        out = np.empty(self.m)
        _check(lib().arlbm_conservation_noalloc(self._h, _dptr(out)), self._h)
        return out

    def save_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().arlbm_state_bytes(self._h, C.byref(n)), self._h)
        buf = C.create_string_buffer(n.value)
        _check(lib().arlbm_save_state(self._h, buf, n.value), self._h)
        return buf.raw

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().arlbm_load_state(self._h, buf, len(blob)), self._h)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().arlbm_destroy(h)
            self._h = None
        self._tensors = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server: resident lattices advance together, one
    batched launch per iteration; admission is bounded by an HBM budget."""

    def __init__(self, hbm_budget: int, precision: int = F32, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(lib().arlbm_server_create(int(hbm_budget), precision, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h
        self._dst = {}  # request id -> the array its result is written into

    def _result_into(self, rid: int, count: int):
        dst = np.empty(count)
        _check(lib().arlbm_server_result_into(self._h, rid, _dptr(dst), count))
        self._dst[rid] = dst

    def submit(self, cfg: Config, U0: np.ndarray, bed: Optional[np.ndarray], nsteps: int,
               result_into: bool = True) -> int:
        """Queue a request; with result_into the server writes its result
        into an array of this object's, which poll hands back uncopied."""
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        bed = None if bed is None else np.ascontiguousarray(bed, dtype=np.float64)
        rid = C.c_uint64()
        _check(lib().arlbm_server_submit(self._h, C.byref(cfg), _dptr(U0), _dptr(bed), int(nsteps), C.byref(rid)))
        if result_into:
            self._result_into(rid.value, U0.size)
        return rid.value

    def submit_state(self, cfg: Config, blob: bytes, nsteps: int, result_into: bool = True) -> int:
        """Queue a request that resumes a state saved by Lattice.save_state."""
        buf = C.create_string_buffer(blob, len(blob))
        rid = C.c_uint64()
        _check(lib().arlbm_server_submit_state(self._h, C.byref(cfg), buf, len(blob), int(nsteps), C.byref(rid)))
        if result_into:
            self._result_into(rid.value, query_sizes(cfg).m * cfg.nx * cfg.ny * cfg.nz)
        return rid.value

    def iterate(self, max_launches: int = 1):
        """Admit, launch (up to max_launches batched steps, never past a
        resident lattice's step count), retire; returns (resident, queued)."""
        r, q = C.c_int32(), C.c_int32()
        if max_launches == 1:
            _check(lib().arlbm_server_iterate(self._h, C.byref(r), C.byref(q)))
        else:
            _check(lib().arlbm_server_iterate_n(self._h, int(max_launches), C.byref(r), C.byref(q), None))
        return r.value, q.value

    def poll(self, max_items: int = 64):
        arr = (Completion * max_items)()
        n = C.c_int32()
        _check(lib().arlbm_server_poll(self._h, arr, max_items, C.byref(n)))
        out = []
        for i in range(n.value):
            c = arr[i]
            dst = self._dst.pop(c.id, None)
            U = None
            if c.status == OK and c.u_count:
                if dst is not None and C.cast(c.U, C.c_void_p).value == dst.ctypes.data:
                    U = dst
                else:
                    U = np.ctypeslib.as_array(c.U, shape=(c.u_count,)).copy()
            out.append({"id": c.id, "status": c.status, "flags": c.flags, "steps": c.steps,
                        "first_bad_step": c.first_bad_step, "t": c.t,
                        "submit_s": c.submit_s,
                        "admit_s": c.admit_s, "done_s": c.done_s, "U": U})
        return out

    def memory(self) -> int:
        """Device bytes charged to resident lattices."""
        b = C.c_size_t()
        _check(lib().arlbm_server_memory(self._h, C.byref(b)))
        return b.value

    def pool_bytes(self) -> int:
        """Device bytes the pool holds for lattices (in use and free)."""
        b = C.c_size_t()
        _check(lib().arlbm_server_pool_bytes(self._h, C.byref(b)))
        return b.value

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().arlbm_server_destroy(h)
            self._h = None
        self._dst = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_kernel_vgprs(precision: int, system: int, dim: int) -> int:
    return lib().arlbm_step_kernel_vgprs(precision, system, dim)


def plan_schedule(cfgs, waves: int):
    """The batched launch's work list for these configurations (host only):
    (queue_start, 9 entries: queue q holds items queue_start[q] ..
    queue_start[q+1]-1; items as an (nsegs, 4) array of (lattice, strip,
    first row, end row), or (lattice, first strip, 0, end strip) for 1D;
    the number of waves the launch takes)."""
    arr = (Config * max(len(cfgs), 1))(*cfgs)
    ns, nw = C.c_int32(), C.c_int32()
    qs = np.zeros(9, dtype=np.int32)
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
    lib().arlbm_plan_schedule(arr, len(cfgs), int(waves), ip(qs), None, 0, C.byref(ns), C.byref(nw))
    sg = np.zeros(4 * max(ns.value, 1), dtype=np.int32)
    _check(lib().arlbm_plan_schedule(arr, len(cfgs), int(waves), ip(qs), ip(sg), ns.value, C.byref(ns),
                                     C.byref(nw)))
    return qs, sg[:4 * ns.value].reshape(-1, 4), nw.value


def plan_groups(cfgs, waves: int):
    """How the server splits these configurations into batched launches
    (host only): (group of each lattice, -1 for 3D; number of groups)."""
    arr = (Config * max(len(cfgs), 1))(*cfgs)
    grp = np.zeros(max(len(cfgs), 1), dtype=np.int32)
    ng = C.c_int32()
    _check(lib().arlbm_plan_groups(arr, len(cfgs), int(waves), grp.ctypes.data_as(C.POINTER(C.c_int32)),
                                   C.byref(ng)))
    return grp[:len(cfgs)], ng.value


def kernel_exp(x: float, precision: int = F64) -> float:
    """The Arrhenius factor's exponential as the FP64 (or FP32) kernels
    evaluate it, on the host."""
    return lib().arlbm_kernel_exp(float(x)) if precision == F64 else lib().arlbm_kernel_expf(float(x))
