"""GPU parity: the HIP library against the FP64 CPU oracle (MI355X only).

FP64 path: the kernels are compiled without contraction and keep the
oracle's operation order, so the results agree to the last bit and are
compared bit for bit.  FP32 path: per field, relative L1 and the largest
pointwise difference over the field's largest magnitude (a local error at a
wall or a front cannot hide in the norm), bounds below.
"""
import numpy as np
import pytest

import oracle as O
from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W
from gpu_common import (require_gpu, say, gpu_lattice, rel_l2_per_comp, oracle_run, rel_l1_per_comp,
                        rel_max_per_comp)

pytestmark = pytest.mark.gpu

T, R, P = W.TRANSMISSIVE, W.REFLECTIVE, W.PERIODIC

# FP32 against the oracle after 60 steps of these cases, per field: measured
# at most 1.1e-5 relative L1 and 6.1e-5 pointwise (the shallow-water cases
# with a wet/dry edge); the bounds keep a margin of about 8x.
TOL_FP32_L1, TOL_FP32_MAX = 1e-4, 5e-4


def small_problem(kind, bcs, n=(131, 45)):
    nx, ny = n
    if kind == "adv1":
        p = W.advection_sine(n=nx, cfl=0.5)
        p.U0 = p.U0 + 0.3 * (W.centres(nx, 0, 1) > 0.6)[None]
    elif kind == "eul1":
        p = W.euler_seeded_1d(4, n=nx)
    elif kind == "swe1":
        p = W.swe_bed_1d(n=nx)
    elif kind == "adv2":
        p = W.advection_sine_2d(n=ny, ax=0.8, ay=-0.5)
        x = W.centres(nx, 0, 1)
        X, Y = np.meshgrid(x, W.centres(ny, 0, 1), indexing="xy")
        p.nx, p.ny, p.x1, p.y1 = nx, ny, 1.0, ny / nx
        p.U0 = (np.sin(2 * np.pi * (X + 2 * Y)) + (X > 0.5))[None]
    elif kind == "eul2":
        p = W.euler_quadrants_2d(W.quadrant_states(5), n=ny)
        x = W.centres(nx, 0, 1)
        X, Y = np.meshgrid(x, W.centres(ny, 0, ny / nx), indexing="xy")
        st = np.array(W.quadrant_states(5))
        quad = np.where(X > 0.5, np.where(Y > 0.5 * ny / nx, 0, 3), np.where(Y > 0.5 * ny / nx, 1, 2))
        pr = st[quad]
        p.U0 = W.euler_conserved(pr[..., 0], pr[..., 1], pr[..., 2], pr[..., 3])
        p.nx, p.ny, p.x1, p.y1 = nx, ny, 1.0, ny / nx
    elif kind == "swe2":
        p = W.swe_bed_2d(seed=2, n=ny)
        x = W.centres(nx, 0, 1)
        X, Y = np.meshgrid(x, W.centres(ny, 0, ny / nx), indexing="xy")
        bed = 0.5 * np.exp(-((X - 0.3) ** 2 + (Y - 0.2) ** 2) / 0.01)
        h = np.where((X - 0.55) ** 2 + (Y - 0.18) ** 2 < 0.04, np.maximum(0, 1 - bed), 0.0)
        p.U0 = W.swe_conserved(h, 0 * h + 0.1 * (h > 0), 0 * h)
        p.bed = bed
        p.nx, p.ny, p.x1, p.y1 = nx, ny, 1.0, ny / nx
    p.bc = bcs
    return p


CASES = [
    ("adv1", (P,) * 4), ("adv1", (T,) * 4),
    ("eul1", (T,) * 4), ("eul1", (R,) * 4), ("eul1", (P,) * 4),
    ("swe1", (R,) * 4), ("swe1", (T,) * 4),
    ("adv2", (P,) * 4), ("adv2", (T, T, P, P)),
    ("eul2", (T,) * 4), ("eul2", (R,) * 4), ("eul2", (P, P, R, R)), ("eul2", (R, R, T, T)),
    ("swe2", (R,) * 4), ("swe2", (T, T, R, R)), ("swe2", (P,) * 4),
]


@pytest.mark.parametrize("kind,bcs", CASES)
def test_first_step_fields_fp64(kind, bcs):
    require_gpu()
    p = small_problem(kind, bcs)
    say(f"[first-step] {kind} bc={bcs} nx={p.nx} ny={p.ny}")
    G = gpu_lattice(p, A.F64, omega_export=True)
    Lo = oracle_run(p, 1)
    G.step(1)
    st = G.sync()
    assert st["step"] == 1
    Ug, Uo = G.moments(), Lo.moments()
    err = rel_l2_per_comp(Ug, Uo)
    say("  U1 rel err", err, "bitwise", bool(np.array_equal(Ug, Uo)))
    assert np.array_equal(Ug, Uo)
    wg, wo = G.omega(), Lo.last_omega()
    say("  omega max abs diff", float(np.abs(wg - wo).max()))
    assert np.array_equal(wg, wo)
    assert st["t"] == Lo.t
    ab = Lo.alpha_bar()
    assert list(st["abar"]) == list(ab)
    G.close()


@pytest.mark.parametrize("kind,bcs", CASES)
def test_multi_step_parity_fp64(kind, bcs):
    require_gpu()
    p = small_problem(kind, bcs)
    say(f"[multi-step] {kind} bc={bcs}")
    G = gpu_lattice(p, A.F64)
    Lo = oracle_run(p, 60)
    G.step(60)
    st = G.sync()
    Ug, Uo = G.moments(), Lo.moments()
    err = rel_l2_per_comp(Ug, Uo)
    say("  U60 rel err", err, "bitwise", bool(np.array_equal(Ug, Uo)), "t", st["t"], Lo.t)
    assert np.array_equal(Ug, Uo)
    assert st["t"] == Lo.t
    G.close()


@pytest.mark.parametrize("kind,bcs", CASES)
def test_multi_step_parity_fp32(kind, bcs):
    require_gpu()
    p = small_problem(kind, bcs)
    say(f"[fp32] {kind} bc={bcs}")
    G = gpu_lattice(p, A.F32)
    Lo = oracle_run(p, 60)
    G.step(60)
    G.sync()
    Ug, Uo = G.moments(), Lo.moments()
    e1, em = rel_l1_per_comp(Ug, Uo), rel_max_per_comp(Ug, Uo)
    say("  fp32 rel L1 per field", e1, "pointwise", em)
    assert max(e1) <= TOL_FP32_L1, e1
    assert max(em) <= TOL_FP32_MAX, em
    G.close()
