"""GPU checks of 2D lattices whose population buffer exceeds 4 GiB.

Below 4 GiB the 2D step addresses the populations through buffer resources
with 32-bit offsets; above it, through 64-bit plane pointers.  Every other
GPU test runs the first path, so these run the second at 6000^2 in FP64
(5.8 GB of populations for Euler, 4.3 GB for shallow water):

* Euler, one column per lane: one step, compared bit for bit with the oracle
  on a 70 x 70 window around the centre of the four-quadrant data.  After one
  step a cell depends on the data within three cells and on the wave-speed
  bound of the initial state, which the window holds (all four states), so
  the window's cells three or more from its edge are exact;
* shallow water over a bed, two columns per lane: two steps, compared bit for
  bit with the same lattice in the batched server (one column per lane,
  64-bit pointers; FP64 results do not depend on the path).
"""
import dataclasses

import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W
from gpu_common import require_gpu, say, gpu_lattice
from helpers import ora_from

pytestmark = pytest.mark.gpu

N = 6000


def test_euler_fp64_over_4gib_window():
    require_gpu()
    p = W.euler_seeded_2d(0, n=N, steps=1)
    f_bytes = A.query_sizes(A.config_from(p, precision=A.F64)).f_bytes
    say(f"[large euler] {N}^2 FP64, population buffer {f_bytes / 2**30:.2f} GiB")
    assert f_bytes > 2 ** 32
    G = gpu_lattice(p, A.F64)
    G.step(1)
    st = G.sync()
    a = N // 2 - 35
    Ug = G.moments()[:, a:a + 70, a:a + 70].copy()
    G.close()
    # the window keeps the cell size bit for bit (its position does not enter
    # the update): [0, 70 dx] with dx = 1/N
    dx = 1.0 / N
    assert (70 * dx) / 70 == dx
    win = dataclasses.replace(p, nx=70, ny=70, x0=0.0, x1=70 * dx, y0=0.0, y1=70 * dx,
                              U0=np.ascontiguousarray(p.U0[:, a:a + 70, a:a + 70]))
    del p
    Lo = ora_from(win)
    Lo.run(1)
    Uo = Lo.moments()
    inner = (slice(None), slice(3, 67), slice(3, 67))
    ok = np.array_equal(Ug[inner], Uo[inner])
    say(f"[large euler] window interior bitwise={ok} t gpu {st['t']!r} oracle {Lo.t!r} "
        f"max diff {np.max(np.abs(Ug[inner] - Uo[inner])):.3e}")
    assert st["t"] == Lo.t
    assert ok


def test_swe_fp64_over_4gib_vs_server():
    require_gpu()
    p = W.swe_bed_2d(3, n=N, steps=2)
    cfg = A.config_from(p, precision=A.F64)
    f_bytes = A.query_sizes(cfg).f_bytes
    say(f"[large swe] {N}^2 FP64, population buffer {f_bytes / 2**30:.2f} GiB")
    assert f_bytes > 2 ** 32
    G = gpu_lattice(p, A.F64)
    G.step(2)
    G.sync()
    U1 = G.moments()
    G.close()
    srv = A.Server(24 << 30, A.F64)
    rid = srv.submit(cfg, p.U0, p.bed, 2)
    res = None
    while res is None:
        srv.iterate()
        for c in srv.poll(4):
            if c["id"] == rid:
                res = c
    srv.close()
    assert res["status"] == 0
    U2 = res["U"].reshape(U1.shape)
    ok = np.array_equal(U1, U2)
    say(f"[large swe] single (two columns per lane) vs batched (one) bitwise={ok}")
    assert ok
