"""GPU checks of the D3Q7 path (Section 2.3 with d = 3) against the FP64 oracle.

FP64 bit for bit on 3D Euler (seeded octant data; a centred sphere with
reflective walls; periodic, transmissive and mixed boundaries; a ragged
non-cubic lattice) and 3D advection, within 1e-12 pointwise on 3D reactive
Euler (its exponential and the root of (2.8) are computed independently on
each side); FP32 within the
stated bound; time-targeted runs, the omega export, conservation sums,
checkpoint/resume, and 3D lattices in the server's mix.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2609_18177_amd import arlbm as A
from paper_2609_18177_amd import workloads as W
from gpu_common import (require_gpu, say, gpu_lattice, rel_l2_per_comp, rel_l1, rel_l1_per_comp, fp64_parity_ok,
                        oracle_run)
from helpers import ora_from, run_until, fsum

pytestmark = pytest.mark.gpu

# FP32 against the FP64 oracle, relative L1 over all fields (3D shock data
# after 20-30 steps; the bound keeps about a 3x margin over the measured
# values printed by the tests).
TOL_FP32 = 3e-5


def _cmp(p, steps, tag, tol32=TOL_FP32, omega_export=False):
    Lo = ora_from(p)
    Lo.run(steps)
    Uo = Lo.moments()
    G = gpu_lattice(p, A.F64, omega_export=omega_export)
    G.step(steps)
    st = G.sync()
    U64 = G.moments()
    om = G.omega() if omega_export else None
    G.close()
    G = gpu_lattice(p, A.F32)
    G.step(steps)
    G.sync()
    e32 = rel_l1(G.moments(), Uo)
    G.close()
    say(f"[3d {tag}] cells {p.cells} steps {steps} bitwise={np.array_equal(U64, Uo)} "
        f"rel L2 {rel_l2_per_comp(U64, Uo)} fp32 rel L1 {e32:.3e}")
    assert fp64_parity_ok(U64, Uo, p.system)
    assert st["t"] == pytest.approx(Lo.t, rel=1e-13) and st["step"] == steps
    assert e32 < tol32, e32
    if omega_export:
        assert np.array_equal(om, Lo.last_omega())
    return U64


@pytest.mark.parametrize("seed", [0, 1])
def test_euler3d_octants_transmissive(seed):
    require_gpu()
    _cmp(W.euler_octants_3d(seed=seed, n=24, steps=20), 20, f"octants seed {seed}", omega_export=seed == 0)


def test_euler3d_periodic_and_mixed():
    require_gpu()
    _cmp(W.euler_octants_3d(seed=2, n=20, steps=20, bc=(A.PERIODIC,) * 6), 20, "octants periodic")
    bc = (A.TRANSMISSIVE, A.REFLECTIVE, A.PERIODIC, A.PERIODIC, A.REFLECTIVE, A.TRANSMISSIVE)
    _cmp(W.euler_octants_3d(seed=3, n=20, steps=20, bc=bc), 20, "octants mixed")


def test_euler3d_sphere_reflective_symmetric():
    require_gpu()
    U = _cmp(W.euler_sphere_3d(n=20, steps=15), 15, "sphere reflective")
    rho = U[0]
    for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
        assert np.max(np.abs(rho - rho.transpose(perm))) < 1e-12


def test_euler3d_ragged_noncubic():
    """17 x 13 x 11 cells of spacing 1/16 (not a multiple of any tile)."""
    require_gpu()
    h = 1.0 / 16
    base = W.euler_octants_3d(seed=4, n=17)
    Z, Y, X = np.meshgrid(*(W.centres(n, 0.0, n * h) for n in (11, 13, 17)), indexing="ij")
    st = W.octant_states(4)
    idx = (X >= 0.5).astype(int) + 2 * (Y >= 0.4).astype(int) + 4 * (Z >= 0.3).astype(int)
    arr = np.array(st)[idx]
    U0 = W.euler3_conserved(arr[..., 0], arr[..., 1], arr[..., 2], arr[..., 3], arr[..., 4])
    p = W.Problem("ragged3d", W.EULER, 3, 17, 13, 0.0, 17 * h, 0.0, 13 * h, base.bc, 0.5, 15, U0,
                  nz=11, z0=0.0, z1=11 * h, bc_z=base.bc_z)
    _cmp(p, 15, "ragged 17x13x11")


@pytest.mark.parametrize("bc", [
    (A.PERIODIC,) * 6,
    (A.REFLECTIVE, A.TRANSMISSIVE, A.PERIODIC, A.PERIODIC, A.TRANSMISSIVE, A.REFLECTIVE),
    (A.PERIODIC, A.PERIODIC, A.TRANSMISSIVE, A.REFLECTIVE, A.REFLECTIVE, A.REFLECTIVE),
])
def test_euler3d_several_tiles_and_chunks(bc):
    """70 x 37 x 33 cells: three tiles across x and five along y (each of
    them ragged at the far side) and plane chunks, with every kind of face."""
    require_gpu()
    h = 1.0 / 32
    base = W.euler_octants_3d(seed=5, n=16)
    nx, ny, nz = 70, 37, 33
    Z, Y, X = np.meshgrid(*(W.centres(m, 0.0, m * h) for m in (nz, ny, nx)), indexing="ij")
    st = W.octant_states(5)
    idx = (X >= 1.1).astype(int) + 2 * (Y >= 0.5).astype(int) + 4 * (Z >= 0.6).astype(int)
    arr = np.array(st)[idx]
    U0 = W.euler3_conserved(arr[..., 0], arr[..., 1], arr[..., 2], arr[..., 3], arr[..., 4])
    p = W.Problem("tiles3d", W.EULER, 3, nx, ny, 0.0, nx * h, 0.0, ny * h, bc[:4], 0.5, 12, U0,
                  nz=nz, z0=0.0, z1=nz * h, bc_z=bc[4:])
    _cmp(p, 12, f"tiles {nx}x{ny}x{nz} bc {bc}", omega_export=True)


def test_euler3d_full_size_first_steps():
    """256^3, the lattice and launch the benchmark times (128 tiles in two
    plane chunks): two steps against the oracle, FP64 bit for bit, FP32
    within the 3D bound per field."""
    require_gpu()
    p = W.euler_octants_3d(seed=0, n=256, steps=2)
    Lo = oracle_run(p, 2, parallel=True)
    Uo = Lo.moments()
    for prec in (A.F64, A.F32):
        G = gpu_lattice(p, prec)
        G.step(2)
        st = G.sync()
        U = G.moments()
        G.close()
        e = rel_l1_per_comp(U, Uo)
        say(f"[3d 256^3] prec={prec} 2 steps bitwise={np.array_equal(U, Uo)} rel L1 per field {e}")
        if prec == A.F64:
            assert np.array_equal(U, Uo) and st["t"] == Lo.t
        else:
            assert max(e) <= TOL_FP32, e
        del U


def test_advection3d_periodic():
    require_gpu()
    _cmp(W.advection_sine_3d(n=20, steps=20), 20, "advection", tol32=1e-5)


def test_reactive3d_sphere():
    require_gpu()
    _cmp(W.reactive_sphere_3d(n=20, steps=10), 10, "reactive sphere", tol32=2e-3)


def test_euler3d_step_until_and_checkpoint():
    require_gpu()
    p = W.euler_octants_3d(seed=6, n=16)
    Lo = ora_from(p)
    run_until(Lo, 0.03)
    G = gpu_lattice(p, A.F64)
    k = G.step_until(0.03)
    assert k == Lo.steps and np.array_equal(G.moments(), Lo.moments())
    blob = G.save_state()
    H = gpu_lattice(p, A.F64)
    H.load_state(blob)
    run_until(Lo, 0.06)
    kh = H.step_until(0.06)
    st = H.sync()
    say(f"[3d until] steps {k}+{kh} oracle {Lo.steps}")
    assert k + kh == Lo.steps and st["t"] == Lo.t
    assert np.array_equal(H.moments(), Lo.moments())
    G.close()
    H.close()


@pytest.mark.parametrize("system", ["euler", "reactive"])
def test_conservation_sums_3d(system):
    """arlbm_conservation over 5 (Euler) and 6 (reactive) fields equals the
    compensated sums of the read-back moments; rho, m, E stay conserved."""
    require_gpu()
    if system == "euler":
        p = W.euler_octants_3d(seed=7, n=16, bc=(A.PERIODIC,) * 6)
    else:
        p = W.reactive_sphere_3d(n=16, bc=(A.PERIODIC,) * 6)
    m = p.U0.shape[0]
    G = gpu_lattice(p, A.F64)
    G.step(12)
    sums = G.conservation()
    U = G.moments()
    for c in range(m):
        ref = fsum(U[c])
        assert abs(sums[c] - ref) <= 1e-12 * max(1.0, fsum(np.abs(U[c]))), (c, sums[c], ref)
    for c in range(m - (1 if system == "reactive" else 0)):
        # a field that starts at zero (momentum of data at rest) is scaled by
        # its magnitude at the end
        scale = max(fsum(np.abs(p.U0[c])), fsum(np.abs(U[c])))
        assert abs(sums[c] - fsum(p.U0[c])) <= 1e-12 * scale, c
    G.close()


def _serve(probs, precision, one_at_a_time, max_launches=1):
    srv = A.Server(1 << 30, precision)
    ids, res = [], {}
    pending = list(probs)
    while pending or len(res) < len(probs):
        if pending and (not one_at_a_time or len(res) == len(ids)):
            p = pending.pop(0)
            ids.append(srv.submit(A.config_from(p, precision=precision), p.U0, p.bed, p.steps))
        srv.iterate(max_launches)
        for c in srv.poll(16):
            res[c["id"]] = c
    srv.close()
    return [res[i] for i in ids]


def test_3d_in_serving_mix():
    """3D lattices served beside 1D and 2D ones (their passes launched after
    the batched step): FP32 the same bits alone and in the mix and as a
    single lattice; FP64 bit for bit with the oracle."""
    require_gpu()
    probs = [dataclasses.replace(W.euler_octants_3d(seed=1, n=24), steps=12),
             W.euler_seeded_1d(3, n=3000, steps=40),
             dataclasses.replace(W.reactive_sphere_3d(n=20), steps=9),
             W.euler_seeded_2d(2, n=90, steps=30),
             dataclasses.replace(W.advection_sine_3d(n=16), steps=15)]
    mix, alone = _serve(probs, A.F32, False), _serve(probs, A.F32, True)
    # several launches per call: the 3D passes run after each batched launch
    many = _serve(probs, A.F32, False, max_launches=5)
    for p, a, b, c in zip(probs, alone, mix, many):
        assert a["status"] == 0 and b["status"] == 0 and c["status"] == 0, p.name
        assert np.array_equal(a["U"], b["U"]), p.name
        assert np.array_equal(a["U"], c["U"]) and a["t"] == c["t"] and c["steps"] == p.steps, p.name
        if p.dim == 3:
            G = gpu_lattice(p, A.F32)
            G.step(p.steps)
            G.sync()
            assert np.array_equal(G.moments().reshape(-1), a["U"]), p.name
            G.close()
    mix64 = _serve(probs, A.F64, False)
    for p, r in zip(probs, mix64):
        Lo = ora_from(p)
        Lo.run(p.steps)
        assert r["status"] == 0 and r["steps"] == p.steps, p.name
        assert fp64_parity_ok(r["U"], Lo.moments(), p.system), p.name
        assert r["t"] == pytest.approx(Lo.t, rel=1e-13), p.name
    say("[3d serving] alone == mix == 5 launches per call == single (FP32); FP64 served == oracle, 3D and 1D/2D")
