"""Host checks of an initial state (arlbm_set_state), on the CPU: a lattice
made with caller buffers needs no GPU, and a state that fails the checks is
rejected before any transfer.  The checks of a large state run over several
threads; what they report must be what one sequential pass over the cells
reports: a non-finite value of U0 anywhere first, then a non-finite bed,
then the first cell (lowest index) with density <= 0 or pressure <= 0
(Euler), or depth < 0 (shallow water)."""
import ctypes as C

import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W


class HostLattice:
    """A lattice whose "device" buffers are host arrays: enough for the
    checks, which run before the first transfer."""

    def __init__(self, p):
        self.cfg = A.config_from(p, precision=A.F32)
        sz = A.query_sizes(self.cfg)
        self._keep = []
        b = A.Buffers()
        b.f[0], b.f[1] = self._buf(sz.f_bytes), self._buf(sz.f_bytes)
        b.u[0], b.u[1] = self._buf(sz.u_bytes), self._buf(sz.u_bytes)
        b.scalars = self._buf(sz.scalar_bytes)
        b.bed = self._buf(sz.bed_bytes) if sz.bed_bytes else None
        self.h = C.c_void_p()
        A._check(A.lib().arlbm_create(C.byref(self.cfg), C.byref(b), None, C.byref(self.h)))

    def _buf(self, nbytes):
        a = np.empty(nbytes + 256, dtype=np.uint8)
        self._keep.append(a)
        return a.ctypes.data + (-a.ctypes.data) % 256

    def reject(self, U0, bed=None):
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        bed = None if bed is None else np.ascontiguousarray(bed, dtype=np.float64)
        rc = A.lib().arlbm_set_state(self.h, A._dptr(U0), A._dptr(bed), 0.0)
        return rc, A.last_error(self.h)

    def close(self):
        A.lib().arlbm_destroy(self.h)


def sequential_verdict(U0, bed, system, gamma):
    """The rule written out with whole-array operations."""
    if not np.all(np.isfinite(U0)):
        return "initial state is not finite"
    if bed is not None and not np.all(np.isfinite(bed)):
        return "bed is not finite"
    if system == W.SWE:
        bad = ~(U0[0] >= 0.0)
        return "initial depth must be >= 0" if bad.any() else None
    rho = U0[0]
    with np.errstate(all="ignore"):
        ke = sum(0.5 * U0[1 + d] * U0[1 + d] / rho for d in range(U0.shape[0] - 2))
        p = (gamma - 1.0) * (U0[-1] - ke)
    bad = ~(rho > 0.0) | ~(p > 0.0)
    if not bad.any():
        return None
    i = int(np.argmax(bad.ravel()))
    return "initial density must be > 0" if not rho.ravel()[i] > 0.0 else "initial pressure must be > 0"


@pytest.mark.parametrize("seed", range(6))
def test_euler_checks_match_a_sequential_pass(seed):
    rng = np.random.default_rng(seed)
    p = W.euler_seeded_2d(seed % 4, n=1024, steps=1)
    L = HostLattice(p)
    try:
        for case in range(8):
            U = p.U0.copy()
            for _ in range(int(rng.integers(1, 4))):
                y, x = int(rng.integers(0, 1024)), int(rng.integers(0, 1024))
                kind = int(rng.integers(0, 4))
                if kind == 0:
                    U[0, y, x] = -float(rng.random())          # density <= 0
                elif kind == 1:
                    U[3, y, x] = 0.0                           # pressure <= 0
                elif kind == 2:
                    U[int(rng.integers(0, 4)), y, x] = np.nan  # not finite
                else:
                    U[0, y, x] = 0.0                           # zero density
            want = sequential_verdict(U, None, W.EULER, p.gamma)
            rc, msg = L.reject(U)
            assert want is not None
            assert rc == A.EPOSITIVITY and msg == want, (seed, case, msg, want)
    finally:
        L.close()


def test_shallow_water_checks_match_a_sequential_pass():
    q = W.swe_bed_2d(0, n=1100, steps=1)
    L = HostLattice(q)
    try:
        U = q.U0.copy()
        U[0, 1000, 3] = -1e-3
        U[0, 600, 7] = -2e-3
        assert L.reject(U, q.bed) == (A.EPOSITIVITY, "initial depth must be >= 0")
        bed = q.bed.copy()
        bed[900, 900] = np.inf
        assert L.reject(U, bed) == (A.EPOSITIVITY, "bed is not finite")
        U[2, 1099, 1099] = np.nan
        assert L.reject(U, bed) == (A.EPOSITIVITY, "initial state is not finite")
        for U_, b_ in ((U, bed),):
            assert sequential_verdict(U_, b_, W.SWE, q.gamma) == "initial state is not finite"
    finally:
        L.close()
