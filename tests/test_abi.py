"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/arlbm.h, and validates configurations on the host."""
import ctypes as C
import re

import pytest

from paper_2609_18177_amd import arlbm as A

# elements added after every plane (staggers power-of-two planes over the
# memory interleave)
PAD = 1088


def declared_functions():
    src = open(A.HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(arlbm_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = A.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_config_defaults():
    c = A.Config()
    assert A.lib().arlbm_config_init(C.byref(c)) == 0
    assert c.abi_version == A.ABI_VERSION and c.eps == 1e-10 and c.cfl == 0.5 and c.gamma == 1.4


def _cfg(**kw):
    c = A.Config()
    A.lib().arlbm_config_init(C.byref(c))
    for k, v in kw.items():
        if k == "bc":
            for i in range(4):
                c.bc[i] = v[i]
        else:
            setattr(c, k, v)
    return c


def test_query_sizes_layout():
    c = _cfg(system=A.EULER, dim=2, nx=100, ny=60, y1=0.6, precision=A.F32)
    s = A.query_sizes(c)
    assert (s.m, s.q) == (4, 5)
    ps = (6000 + 63) // 64 * 64 + PAD         # plane stride: nx ny rounded up to 64, plus the pad
    assert s.f_bytes == (20 * ps * 4 + 255) // 256 * 256
    assert s.u_bytes == (4 * ps * 4 + 255) // 256 * 256
    assert s.total_bytes == 2 * s.f_bytes + 2 * s.u_bytes + s.scalar_bytes
    c.precision = A.F64
    assert A.query_sizes(c).f_bytes == (20 * ps * 8 + 255) // 256 * 256
    c2 = _cfg(system=A.SWE, dim=2, nx=64, ny=64, has_bed=1)
    assert A.query_sizes(c2).bed_bytes == (64 * 64 + PAD) * 4


@pytest.mark.parametrize("bad", [
    dict(cfl=1.0), dict(cfl=0.0), dict(eps=0.0), dict(dim=3), dict(nx=3),
    dict(system=A.ADVECTION, bc=(A.REFLECTIVE,) * 4), dict(bc=(A.PERIODIC, A.TRANSMISSIVE, 1, 1)),
    dict(dim=2, nx=64, ny=32),                     # dx != dy on the unit square
    dict(has_bed=1), dict(system=A.SWE, g=0.0), dict(gamma=1.0), dict(omega_mode=1, omega_fixed=2.5),
    dict(abi_version=99), dict(precision=5), dict(dim=1, ny=2),
])
def test_query_sizes_rejects(bad):
    c = _cfg(**bad)
    s = A.Sizes()
    rc = A.lib().arlbm_query_sizes(C.byref(c), C.byref(s))
    assert rc == A.EINVAL
    assert A.last_error()
