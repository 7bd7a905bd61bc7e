"""GPU runs to a target time and with a fixed relaxation parameter, against
the FP64 oracle and the values the paper prints.

* ``step_until``: whole steps until t >= T (the last step is not shortened),
  the reading under which the oracle reproduces Table 5.1; the GPU FP64 path
  must take the same number of steps and give the oracle's moments bit for
  bit, whatever batching of launches the library chose;
* Tables 5.1, 5.2 and 5.5 recomputed on the GPU (FP64 exact to the oracle,
  FP32 within the stated bounds of the printed values);
* fixed omega (omega = 1, the first-order Lax-Friedrichs limit of Example 5.6,
  and omega in (1, 2)) on the GPU against the oracle in the same mode.
"""
import json
import math
import os

import numpy as np
import pytest

import exact as X
from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W
from gpu_common import require_gpu, say, gpu_lattice, rel_l2_per_comp, rel_l1
from helpers import ora_from, run_until, rel_l2

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _gpu_until(p, T, precision, **kw):
    G = gpu_lattice(p, precision, **kw)
    n = G.step_until(T)
    st = G.sync()
    U = G.moments()
    G.close()
    return U, n, st


@pytest.mark.parametrize("n", [400, 800, 1600, 6400])
def test_table_5_1_on_gpu(n):
    """Example 5.1 / Table 5.1: smooth advection, CFL 0.9, t = 1."""
    require_gpu()
    t = GOLD["t_adv"]
    ref = t["err"][t["N"].index(n)]
    p = W.advection_sine(n=n, cfl=0.9)
    Lo = run_until(ora_from(p), 1.0)
    x = W.centres(n, 0.0, 1.0)
    U64, k, st = _gpu_until(p, 1.0, A.F64)
    e64 = rel_l2(U64[0], np.sin(2 * np.pi * (x - st["t"])))
    U32, k32, st32 = _gpu_until(p, 1.0, A.F32)
    e32 = rel_l2(U32[0], np.sin(2 * np.pi * (x - st32["t"])))
    say(f"[table 5.1 N={n}] steps gpu={k} oracle={Lo.steps} t={st['t']!r} err fp64={e64:.5e} "
        f"fp32={e32:.5e} printed={ref:.5e}")
    assert k == Lo.steps and st["step"] == Lo.steps
    assert st["t"] == Lo.t
    assert np.array_equal(U64, Lo.moments())
    assert abs(e64 / ref - 1.0) < 0.08
    if n == 6400:
        assert abs(e64 / ref - 1.0) < 1e-4
    # FP32 has a rounding floor near 1e-4 relative L2 here (omega close to 2
    # leaves the non-equilibrium modes undamped; a correctly rounded float32
    # emulation of the same scheme gives 0.97e-4 at N=800 and 0.91e-4 at
    # N=1600; the GPU measures 2.9e-4 at N=6400, where the run is 7112
    # steps long), so only the coarsest row is a discretisation-error check.
    assert e32 <= e64 + (5e-4 if n == 6400 else 1.5e-4), (e32, e64)
    if n == 400:
        assert abs(e32 / ref - 1.0) < 0.1, (e32, ref)
    assert k32 == k


@pytest.mark.parametrize("n", [400, 800])
def test_table_5_2_on_gpu(n):
    """Example 5.3 / Table 5.2: 1D Euler entropy wave, CFL 0.6, t = 1."""
    require_gpu()
    t = GOLD["t_ent1"]
    ref = t["err"][t["N"].index(n)]
    p = W.euler_entropy_wave_1d(n=n)
    Lo = run_until(ora_from(p), 1.0)
    x = W.centres(n, 0.0, 1.0)
    U64, k, st = _gpu_until(p, 1.0, A.F64)
    e64 = rel_l2(U64[0], 1 + 0.2 * np.sin(2 * np.pi * (x - st["t"])))
    U32, k32, st32 = _gpu_until(p, 1.0, A.F32)
    e32 = rel_l2(U32[0], 1 + 0.2 * np.sin(2 * np.pi * (x - st32["t"])))
    say(f"[table 5.2 N={n}] steps gpu={k} oracle={Lo.steps} err fp64={e64:.5e} fp32={e32:.5e} printed={ref:.5e}")
    assert k == Lo.steps
    assert np.array_equal(U64, Lo.moments())
    assert abs(e64 / ref - 1.0) < 0.05
    assert e32 <= e64 + 1.5e-4, (e32, e64)  # FP32 rounding floor, as for Table 5.1


def test_table_5_3_on_gpu():
    """Example 5.4 / Table 5.3: 2D diagonal entropy wave, CFL 0.3, with the
    3x3 box of (2.15), run to t = 0.2, where the printed errors and orders are
    reproduced (the example states t = 0.3, at which every error is about
    1.5 times the printed one); FP64 bit for bit with the oracle."""
    require_gpu()
    t = GOLD["t_ent2"]
    T = t["t_reproduced"]
    errs = []
    for n, ref in zip(t["N"][:3], t["err"][:3]):
        p = W.euler_entropy_wave_2d(n=n)
        Lo = run_until(ora_from(p, parallel=True), T)
        U64, k, st = _gpu_until(p, T, A.F64)
        x = W.centres(n, 0.0, 1.0)
        X_, Y_ = np.meshgrid(x, x, indexing="xy")
        errs.append(rel_l2(U64[0], 1 + 0.2 * np.sin(2 * np.pi * (X_ + Y_ - 2 * st["t"]))))
        say(f"[table 5.3 N={n}] steps gpu={k} oracle={Lo.steps} err={errs[-1]:.5e} printed {ref:.5e}")
        assert k == Lo.steps and np.array_equal(U64, Lo.moments())
        assert abs(errs[-1] / ref - 1.0) < 0.03
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for o, ref in zip(orders, t["order"][1:3]):
        assert abs(o - ref) < 0.02, orders


def test_fixed_omega_two_smooth():
    """omega = 2 (the upper end of (2.12)) on smooth data: advection (Example
    5.1 data) and the 1D entropy wave, FP64 bit for bit with the oracle."""
    require_gpu()
    for p, steps in ((W.advection_sine(n=256, cfl=0.5), 512), (W.euler_entropy_wave_1d(n=200), 400)):
        Lo = ora_from(p, omega_fixed=2.0)
        Lo.run(steps)
        G = gpu_lattice(p, A.F64, omega_fixed=2.0)
        G.step(steps)
        st = G.sync()
        U = G.moments()
        G.close()
        say(f"[omega=2 {p.system}] bitwise={np.array_equal(U, Lo.moments())} t={st['t']}")
        assert np.array_equal(U, Lo.moments()) and st["t"] == Lo.t


def test_table_5_5_sod_on_gpu():
    """Example 5.6 / Table 5.5: local total variation of the Sod solution,
    N = 600, CFL 0.3, t = 0.2; the fixed omega = 1 run is more dissipative."""
    require_gpu()
    t = GOLD["t_sod"]
    p = W.euler_riemann_1d(*W.SOD, n=600, cfl=0.3)
    Lo = run_until(ora_from(p), 0.2)
    x = W.centres(600, 0.0, 1.0)
    I = (x >= 0.15) & (x <= 0.35)
    refs = (t["tv_rho"], t["tv_u"], t["tv_p"])
    U64, k, st = _gpu_until(p, 0.2, A.F64)
    assert k == Lo.steps and np.array_equal(U64, Lo.moments())
    for prec, tol in ((A.F64, 0.01), (A.F32, 0.01)):
        U, _, st = _gpu_until(p, 0.2, prec)
        tv = [X.total_variation(q[I]) for q in X.euler_primitive(U)]
        say(f"[sod tv {'f64' if prec == A.F64 else 'f32'}] {tv} printed {refs}")
        for v, ref in zip(tv, refs):
            assert abs(v - ref) < tol, (tv, refs)
    U1, k1, st1 = _gpu_until(p, 0.2, A.F64, omega_fixed=1.0)
    L1 = run_until(ora_from(p, omega_fixed=1.0), 0.2)
    assert k1 == L1.steps and np.array_equal(U1, L1.moments())
    re, _, _ = X.riemann_sample(*W.SOD, (x - 0.5) / st["t"])
    err_adapt = np.mean(np.abs(U64[0] - re))
    err_one = np.mean(np.abs(U1[0] - re))
    say(f"[sod] L1 density error adaptive {err_adapt:.4e} omega=1 {err_one:.4e}")
    assert err_adapt < 0.6 * err_one


def test_step_until_is_independent_of_batching():
    """One call, one step at a time, and a capped call followed by the rest
    reach the same state and the same step count; a later plain step
    continues from it as the oracle does."""
    require_gpu()
    p = W.euler_riemann_1d(*W.LAX, n=1000, cfl=0.5)
    T = 0.14
    Lo = run_until(ora_from(p), T)
    A1 = gpu_lattice(p, A.F64)
    k1 = A1.step_until(T)
    U1 = A1.moments()
    A2 = gpu_lattice(p, A.F64)
    k2 = 0
    while A2.sync()["t"] < T:
        A2.step(1)
        k2 += 1
    U2 = A2.moments()
    A3 = gpu_lattice(p, A.F64)
    k3a = A3.step_until(T, max_steps=17)
    st3 = A3.sync()
    assert k3a == 17 and st3["step"] == 17 and st3["t"] < T
    k3b = A3.step_until(T)
    U3 = A3.moments()
    say(f"[batching] steps {k1} {k2} {k3a}+{k3b} oracle {Lo.steps}")
    assert k1 == k2 == k3a + k3b == Lo.steps
    assert np.array_equal(U1, Lo.moments()) and np.array_equal(U2, U1) and np.array_equal(U3, U1)
    # already there: no step
    assert A1.step_until(T) == 0
    # continuing with plain steps after a batch that ended in surplus launches
    A1.step(5)
    st = A1.sync()
    Lo.run(5)
    assert st["step"] == Lo.steps and st["t"] == Lo.t
    assert np.array_equal(A1.moments(), Lo.moments())
    for G in (A1, A2, A3):
        G.close()


def test_step_until_2d_and_checkpoint():
    """2D Euler to a target time, with a checkpoint taken after a batch that
    ended in surplus launches and resumed in a fresh lattice."""
    require_gpu()
    p = W.euler_seeded_2d(seed=3, n=96)
    Lo = ora_from(p)
    run_until(Lo, 0.05)
    G = gpu_lattice(p, A.F64)
    k = G.step_until(0.05)
    assert k == Lo.steps and np.array_equal(G.moments(), Lo.moments())
    blob = G.save_state()
    H = gpu_lattice(p, A.F64)
    H.load_state(blob)
    run_until(Lo, 0.1)
    kh = H.step_until(0.1)
    stH = H.sync()
    say(f"[2d until] steps {k}+{kh} oracle {Lo.steps} t {stH['t']!r} {Lo.t!r}")
    assert k + kh == Lo.steps and stH["step"] == Lo.steps and stH["t"] == Lo.t
    assert np.array_equal(H.moments(), Lo.moments())
    G.close()
    H.close()


@pytest.mark.parametrize("omega", [1.0, 1.5, 1.9])
@pytest.mark.parametrize("kind", ["euler1d", "euler2d", "swe2d"])
def test_fixed_omega_parity(kind, omega):
    """Fixed omega in place of (2.12)/(2.16): FP64 bit for bit against the
    oracle.  FP32 within the relative L1 bound of the adaptive runs, except
    shallow water over the dry bed with omega > 1: there the fixed-omega
    scheme is ill-conditioned at the wet/dry front (the FP64 oracle itself
    moves by 1e-2 (omega 1.5) and 3e-2 (omega 1.9) relative L1 when the
    initial state is perturbed by 1e-7), so FP32 is checked on what must
    hold at any rounding: the water volume, conserved by reflective walls."""
    require_gpu()
    if kind == "euler1d":
        p, steps = W.euler_seeded_1d(seed=2, n=777), 300
    elif kind == "euler2d":
        p, steps = W.euler_seeded_2d(seed=1, n=131), 100
    else:
        p, steps = W.swe_bed_2d(seed=0, n=131), 100
    Lo = ora_from(p, omega_fixed=omega)
    Lo.run(steps)
    Uo = Lo.moments()
    G = gpu_lattice(p, A.F64, omega_fixed=omega, omega_export=True)
    G.step(steps)
    st = G.sync()
    U64 = G.moments()
    om = G.omega()
    G.close()
    G = gpu_lattice(p, A.F32, omega_fixed=omega)
    G.step(steps)
    G.sync()
    U32 = G.moments()
    e32 = rel_l1(U32, Uo)
    G.close()
    say(f"[fixed omega {omega} {kind}] fp64 bitwise={np.array_equal(U64, Uo)} "
        f"rel L2 {rel_l2_per_comp(U64, Uo)} fp32 rel L1 {e32:.3e}")
    assert np.array_equal(U64, Uo)
    assert st["t"] == Lo.t
    assert np.all(om == omega)
    if kind == "swe2d" and omega > 1.0:
        v0 = math.fsum(p.U0[0].ravel().tolist())
        v32 = math.fsum(U32[0].ravel().tolist())
        assert abs(v32 / v0 - 1.0) < 1e-5, (v32, v0)
    else:
        assert e32 < 3e-4
