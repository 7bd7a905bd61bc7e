"""Oracle pins: smoothness indicator (2.9)/(2.13), nu (2.10)/(2.14), box sum
(2.11)/(2.15) and relaxation parameter (2.12)/(2.16), on inputs whose values
follow in closed form (CPU)."""
import numpy as np
import pytest

import oracle as O
from paper_2609_18177_amd import workloads as W
from helpers import ora_cfg_from


def _lat(system, d, U0, n, bc=O.TRANSMISSIVE, x0=0.0, x1=1.0, adv=(1.0, 0.5)):
    cfg = O.make_cfg(system, d, n, n if d == 2 else 1, x0=x0, x1=x1, y0=x0, y1=x1,
                     bc=(bc,) * 4, adv=adv)
    return O.Lattice(cfg).init(U0)


def theta(dm, dp, dx):
    """Scalar indicator written out for closed-form expectations."""
    return abs(dp - dm) / (abs(dm) + abs(dp) + dx) + abs(dm) + abs(dp)


@pytest.mark.parametrize("bc", [O.PERIODIC, O.TRANSMISSIVE, O.REFLECTIVE])
def test_constant_state_gives_omega_two(bc):
    n = 16
    U0 = W.euler_conserved(np.full((n, n), 0.7), np.zeros((n, n)) if bc == O.REFLECTIVE else np.full((n, n), 0.3),
                           np.zeros((n, n)) if bc == O.REFLECTIVE else np.full((n, n), -0.2), np.full((n, n), 1.1))
    L = _lat(O.EULER, 2, U0, n, bc)
    assert np.all(L.nu_field() == 0.0)
    assert np.all(L.omega_field() == 2.0)


def test_linear_profile_1d():
    n, s = 32, -0.8
    x = W.centres(n, 0.0, 1.0)
    dx = 1.0 / n
    L = _lat(O.ADVECTION, 1, (s * x)[None], n)
    nu = L.nu_field()
    np.testing.assert_allclose(nu[2:n - 2], 2 * abs(s) * dx, rtol=1e-12)
    om = L.omega_field()
    np.testing.assert_allclose(om[3:n - 3], 1 + 1 / (1 + 6 * abs(s) * dx), rtol=1e-14)
    assert np.all((om > 1.0) & (om <= 2.0))


def test_linear_profile_2d_full_box():
    """nu = 2|s_x| dx + 2|s_y| dx on a linear field, and the 3x3 box of (2.15)
    sums nine equal values."""
    n, sx, sy = 20, 0.6, -1.1
    x = W.centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    dx = 1.0 / n
    L = _lat(O.ADVECTION, 2, (sx * X + sy * Y)[None], n)
    nu = L.nu_field()
    nu0 = 2 * abs(sx) * dx + 2 * abs(sy) * dx
    np.testing.assert_allclose(nu[2:-2, 2:-2], nu0, rtol=1e-12)
    om = L.omega_field()
    np.testing.assert_allclose(om[3:-3, 3:-3], 1 + 1 / (1 + 9 * nu0), rtol=1e-13)


def test_step_function_1d():
    n = 12
    U0 = np.where(np.arange(n) >= 6, 1.0, 0.0)[None]
    dx = 1.0 / n
    L = _lat(O.ADVECTION, 1, U0, n)
    nu = L.nu_field()
    jump = 1.0 / (1.0 + dx) + 1.0
    expect = np.zeros(n)
    expect[5] = expect[6] = jump
    np.testing.assert_allclose(nu, expect, rtol=1e-15, atol=0)
    nut = np.array([expect[max(i - 1, 0):i + 2].sum() if 0 < i < n - 1 else 0 for i in range(n)])
    np.testing.assert_allclose(L.omega_field(), 1 + 1 / (1 + nut), rtol=1e-15)


def test_euler_entropy_profile_projects_to_density():
    """With u, p uniform, U_i - U_{i-1} = (rho_i - rho_{i-1}) r_entropy and
    Toro's normalisation maps it to the density jump itself: nu of the Euler
    system equals the scalar nu of the density profile."""
    rng = np.random.default_rng(3)
    n = 24
    rho = 1.0 + 0.3 * rng.standard_normal(n).clip(-2, 2)
    Ue = W.euler_conserved(rho, np.full(n, 0.4), 0 * rho, np.full(n, 0.9), dim=1)
    nu_e = _lat(O.EULER, 1, Ue, n, O.PERIODIC).nu_field()
    nu_s = _lat(O.ADVECTION, 1, rho[None], n, O.PERIODIC).nu_field()
    np.testing.assert_allclose(nu_e, nu_s, rtol=1e-12, atol=1e-15)


def test_euler_pressure_jump_closed_form():
    """At rest, a pressure jump dp gives L dU = (dp/2c^2, -dp/c^2, dp/2c^2)
    with c^2 = gamma p_i / rho at the cell whose L is used."""
    n, g = 12, 1.4
    pL, pR, rho = 1.0, 0.4, 0.8
    p = np.where(np.arange(n) >= 6, pR, pL)
    U = W.euler_conserved(np.full(n, rho), 0 * p, 0 * p, p, dim=1)
    dx = 1.0 / n
    nu = _lat(O.EULER, 1, U, n).nu_field()
    dpj = pR - pL
    c2L, c2R = g * pL / rho, g * pR / rho
    cellL = sum(theta(0.0, w, dx) for w in (dpj / (2 * c2L), -dpj / c2L, dpj / (2 * c2L)))
    cellR = sum(theta(w, 0.0, dx) for w in (dpj / (2 * c2R), -dpj / c2R, dpj / (2 * c2R)))
    np.testing.assert_allclose(nu[5], cellL, rtol=1e-13)
    np.testing.assert_allclose(nu[6], cellR, rtol=1e-13)
    assert np.all(nu[:4] == 0) and np.all(nu[8:] == 0)


def test_swe_velocity_jump_closed_form():
    """At uniform depth, a velocity jump du gives L dU = h du (-1/2c, 1/2c)."""
    n, g, h = 12, 9.81, 1.3
    u = np.where(np.arange(n) >= 6, 0.5, -0.25)
    U = W.swe_conserved(np.full(n, h), u, 0 * u, dim=1)
    dx = 1.0 / n
    nu = _lat(O.SWE, 1, U, n).nu_field()
    a = h * 0.75 / (2 * np.sqrt(g * h))
    expect = theta(0.0, a, dx) * 2
    np.testing.assert_allclose(nu[5], expect, rtol=1e-13)
    np.testing.assert_allclose(nu[6], expect, rtol=1e-13)


def test_omega_range_on_shock_data():
    p = W.euler_seeded_2d(3, n=32, steps=10)
    L = O.Lattice(ora_cfg_from(p)).init(p.U0)
    L.run(5)
    om = L.last_omega()
    assert np.all(om > 1.0) and np.all(om <= 2.0)
    assert om.min() < 1.5 and om.max() == 2.0
