"""GPU checks of the 2D strip geometries of the fused step.

A 2D advection or shallow-water lattice of even nx runs its step with two
adjacent columns per lane (strips of 120 output columns, 8-byte row accesses
in FP32; shallow water also in FP64), in the single-lattice kernel and in the
batched server alike; odd nx and the other systems run one column per lane
(strips of 58).  Every cell does the
same arithmetic in both, so the two must agree; the cases below span several
strips with a ragged last strip, the lattice edges where a lane's two columns
map to mirror-ghost cells in descending order (transmissive and reflective
walls), the bed source, reactive Euler, the smallest lattice (nx = 4), the
omega export, and null steps of a time-targeted run.

Checks per case: FP64 bit for bit with the oracle (reactive Euler: within
1e-12 pointwise, see test_gpu_reactive.py); FP32 against the oracle
(relative L1 over all fields, bound below); the exported FP32 relaxation
parameter of the first step against the oracle's; FP32 single lattice
against the same lattice in the FP32 batched server (its own strip width,
row segments of the server's schedule), bit for bit: FP32 rounds every expression as written
(no contraction, the hardware reciprocal and root named explicitly), so the
strip width, the band decomposition and the kernel do not change the bits.  A further test fills both population buffers with a byte
pattern and checks that the steps write nothing outside the lattice cells
of each plane (the masked halo lanes and warm-up rows).
"""
import dataclasses

import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W
from gpu_common import require_gpu, say, gpu_lattice, rel_l1, fp64_parity_ok
from helpers import ora_from

pytestmark = pytest.mark.gpu

# FP32 against the FP64 oracle after 60 steps on these small crops, where
# the quadrant shocks cover a large share of the cells: measured 1.8e-4 for
# the Euler crop with either strip geometry (the FP32 rounding floor, as in
# the full-size checks); the bound leaves a margin of about 5x.
TOL_FP32 = 1e-3
# After one step the FP32 relaxation parameter differs from the oracle's only
# through the rounding of the initial data and of the indicator arithmetic;
# the indicator divides small differences (measured up to 4.5e-4 over the
# shallow-water lake and 2.9e-3 for reactive Euler, 7e-8 for gas dynamics).
TOL_OMEGA32_1 = 1e-2


def crop(p, nx, ny, bc=None, ox=0, oy=0, steps=60):
    """The nx x ny window at cell (ox, oy) of a square problem (same cell
    size), run for a fixed number of steps."""
    dx = (p.x1 - p.x0) / p.nx
    U0 = np.ascontiguousarray(p.U0[:, oy:oy + ny, ox:ox + nx])
    bed = None if p.bed is None else np.ascontiguousarray(p.bed[oy:oy + ny, ox:ox + nx])
    x0, y0 = p.x0 + ox * dx, p.y0 + oy * dx
    return dataclasses.replace(p, nx=nx, ny=ny, x0=x0, x1=x0 + nx * dx, y0=y0, y1=y0 + ny * dx, U0=U0, bed=bed,
                               bc=tuple(bc) if bc is not None else p.bc, steps=steps, t_final=0.0)


def _served(p, steps):
    srv = A.Server(1 << 28, A.F32)
    rid = srv.submit(A.config_from(p, precision=A.F32), p.U0, p.bed, steps)
    res = None
    while res is None:
        srv.iterate()
        for c in srv.poll(4):
            if c["id"] == rid:
                res = c
    srv.close()
    assert res["status"] == 0
    return res["U"].reshape((-1, p.ny, p.nx))


T, R, P = W.TRANSMISSIVE, W.REFLECTIVE, W.PERIODIC
CASES = {
    "euler 250x70 transmissive": lambda: crop(W.euler_seeded_2d(0, n=256, steps=60), 250, 70),
    "euler 250x70 reflective": lambda: crop(W.euler_seeded_2d(1, n=256, steps=60), 250, 70, bc=(R,) * 4),
    "euler 240x64 periodic": lambda: crop(W.euler_seeded_2d(2, n=256, steps=60), 240, 64, bc=(P,) * 4),
    "euler 251x70 odd nx": lambda: crop(W.euler_seeded_2d(0, n=256, steps=60), 251, 70),
    "euler 4x40 reflective": lambda: crop(W.euler_seeded_2d(3, n=64, steps=60), 4, 40, bc=(R, R, T, T)),
    "swe bed 250x250 reflective": lambda: crop(W.swe_bed_2d(0, n=256, steps=60), 250, 250),
    "swe bed 249x250 odd nx": lambda: crop(W.swe_bed_2d(0, n=256, steps=60), 249, 250),
    "swe bed 240x256 periodic": lambda: crop(W.swe_bed_2d(1, n=256, steps=60), 240, 256, bc=(P,) * 4),
    "swe lake 122x64 reflective": lambda: crop(W.swe_lake_at_rest_2d(n=128, steps=60), 122, 64),
    "swe dam 250x128 transmissive": lambda: crop(W.swe_circular_dam_2d(n=256), 250, 128),
    "swe dam 4x128 transmissive": lambda: crop(W.swe_circular_dam_2d(n=256), 4, 128, ox=62, oy=64),
    "advection 130x40 periodic": lambda: crop(W.advection_sine_2d(n=130, steps=60), 130, 40),
    "advection 250x70 transmissive": lambda: crop(W.advection_sine_2d(n=256, steps=60), 250, 70, bc=(T,) * 4),
    "advection 251x70 odd nx": lambda: crop(W.advection_sine_2d(n=256, steps=60), 251, 70, bc=(T,) * 4),
    "reactive 250x70 transmissive": lambda: crop(W.reactive_seeded_2d(0, n=256, steps=60), 250, 70),
    "reactive 244x70 reflective": lambda: crop(W.reactive_seeded_2d(1, n=256, steps=60), 244, 70, bc=(R,) * 4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_strip_geometry(name):
    require_gpu()
    p = CASES[name]()
    steps = p.steps
    two = p.nx % 2 == 0 and p.system in (W.ADVECTION, W.SWE)
    say(f"[strips {name}] nx={p.nx} ny={p.ny} steps={steps} columns per lane {2 if two else 1}")
    Lo = ora_from(p)
    Lo.run(steps)
    Uo = Lo.moments()
    L1 = ora_from(p)
    L1.run(1)
    om_ref = L1.last_omega()
    G = gpu_lattice(p, A.F64, omega_export=True)
    G.step(1)
    G.sync()
    om64_ok = np.array_equal(G.omega(), om_ref)
    G.step(steps - 1)
    st64 = G.sync()
    U64 = G.moments()
    G.close()
    G = gpu_lattice(p, A.F32, omega_export=True)
    G.step(1)
    G.sync()
    eom = float(np.max(np.abs(G.omega() - om_ref)))
    G.step(steps - 1)
    st32 = G.sync()
    U32 = G.moments()
    G.close()
    Us = _served(p, steps)
    e32 = rel_l1(U32, Uo)
    say(f"[strips {name}] fp64 bitwise={np.array_equal(U64, Uo)} fp32 rel L1 {e32:.2e} "
        f"single vs batched bitwise={np.array_equal(U32, Us)} rel L1 {rel_l1(U32, Us):.2e} "
        f"step-1 omega fp64 bitwise={om64_ok} fp32 max diff {eom:.2e} flags {st64['flags']}/{st32['flags']}")
    assert om64_ok
    assert fp64_parity_ok(U64, Uo, p.system)
    assert st64["t"] == pytest.approx(Lo.t, rel=1e-13)
    assert e32 <= TOL_FP32, e32
    assert np.array_equal(U32, Us)
    assert eom <= TOL_OMEGA32_1, eom


@pytest.mark.parametrize("maker,n", [(W.euler_seeded_2d, 1024), (W.swe_bed_2d, 1024), (W.reactive_seeded_2d, 512)])
def test_fp32_single_equals_served_at_size(maker, n):
    """FP32 bit for bit between a single lattice (bands of equal height,
    one per wave) and the same lattice in the batched server (row segments
    of the server's schedule, cut where the balance of work falls), at a
    size where the decompositions differ."""
    require_gpu()
    p = maker(0, n=n, steps=20)
    G = gpu_lattice(p, A.F32)
    G.step(p.steps)
    st = G.sync()
    U1 = G.moments()
    G.close()
    U2 = _served(p, p.steps)
    say(f"[strips {p.name} {n}^2] FP32 single vs served bitwise={np.array_equal(U1, U2)} "
        f"max diff {float(np.max(np.abs(U1 - U2))):.3e} t {st['t']}")
    assert np.array_equal(U1, U2)


def test_two_columns_null_steps():
    """A time-targeted FP32 shallow-water run (its surplus launches are null
    steps that copy the populations with two columns per lane) equals
    stepping exactly."""
    require_gpu()
    p = crop(W.swe_bed_2d(2, n=256), 250, 250)
    G = gpu_lattice(p, A.F32)
    k = G.step_until(0.02)
    st = G.sync()
    U1 = G.moments()
    G.close()
    H = gpu_lattice(p, A.F32)
    H.step(k)
    st2 = H.sync()
    U2 = H.moments()
    H.close()
    say(f"[strips null steps] k={k} t={st['t']} bitwise={np.array_equal(U1, U2)}")
    assert k > 0 and st["step"] == k and st["t"] >= 0.02
    assert np.array_equal(U1, U2) and st["t"] == st2["t"]


SENTINEL = 0xA5  # byte pattern of the padding (0xA5A5A5A5 is a finite float32, -2.9e-16)


@pytest.mark.parametrize("name,prec", [
    ("euler 250x70 transmissive", A.F32), ("euler 251x70 odd nx", A.F64),
    ("swe bed 250x250 reflective", A.F32), ("swe bed 240x256 periodic", A.F64),
    ("advection 130x40 periodic", A.F32), ("reactive 244x70 reflective", A.F32),
])
def test_steps_write_only_lattice_cells(name, prec):
    """Masked lanes (halo lanes, warm-up rows) store nothing: after the step,
    every byte of both population buffers outside the nx ny cells of each
    plane (the pad after every plane, the tail of the buffer) still holds
    the byte pattern written before, and the results equal a run on
    buffers that were not pre-filled, bit for bit."""
    require_gpu()
    p = dataclasses.replace(CASES[name](), steps=7)
    cfg = A.config_from(p, precision=prec)
    size = 8 if prec == A.F64 else 4
    planes = cfg.nx * cfg.ny
    nplanes = (5 if p.dim == 2 else 3) * A.query_sizes(cfg).m
    ref = gpu_lattice(p, prec)
    ref.step(p.steps)
    ref.sync()
    Uref = ref.moments()
    ref.close()
    L = A.Lattice(cfg, owner="torch")
    f_bytes = L.sizes.f_bytes
    # the binding allocates f[0], u[0], f[1], u[1] in this order, each at a
    # 256-byte aligned offset of its tensor
    fts = [L._tensors[0], L._tensors[2]]
    views = []
    for t in fts:
        off = (-t.data_ptr()) % 256
        views.append(t[off:off + f_bytes])
    views[0].fill_(SENTINEL)
    L.set_state(p.U0, p.bed)
    views[1].fill_(SENTINEL)  # f[1] holds nothing before the first step
    L.step(p.steps)
    st = L.sync()
    # read the buffers before the moments: FP32 read-back converts the moments
    # to FP64 in the population buffer the next step would write
    raw = [v.cpu().numpy() for v in views]
    U = L.moments()
    ps = (planes + 63) // 64 * 64 + 1088
    ok = True
    for bi, b in enumerate(raw):
        body = b[:nplanes * ps * size].reshape(nplanes, ps * size)
        pad = body[:, planes * size:]
        pad_ok = bool(np.all(pad == SENTINEL))
        tail_ok = bool(np.all(b[nplanes * ps * size:] == SENTINEL))
        if not (pad_ok and tail_ok):
            bad = np.argwhere(pad != SENTINEL)
            el = np.unique(bad[:, 1] // size)
            dt = np.float64 if size == 8 else np.float32
            vals = pad.view(dt)[bad[0, 0], el[:6]] if len(bad) else []
            say(f"[pads {name}] buffer f[{bi}]: {len(bad)} bytes changed in the pads of planes "
                f"{np.unique(bad[:, 0])[:8]}..., element offsets after the plane {el[:12]}..., values {vals}; "
                f"tail ok={tail_ok}")
        ok = ok and pad_ok and tail_ok
    L.close()
    say(f"[pads {name} prec={prec}] pads and tails untouched={ok} results bitwise={np.array_equal(U, Uref)} "
        f"flags {st['flags']}")
    assert ok
    assert np.array_equal(U, Uref)
