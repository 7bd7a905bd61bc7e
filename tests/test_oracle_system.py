"""Oracle pins: per-state system functions and the equilibrium (CPU).

* (2.4)/(2.7): moment and coefficient identities of the Lax-Friedrichs-type
  equilibrium (2.20) in the general form (2.5), including the source split (2.6);
* left eigenvectors: L R = I against Toro's right eigenvectors and
  L A R = diag(lambda) with A from finite differences of the flux;
* eigenvalue bound of (2.17)/(2.19) against numpy's eigenvalues of A;
* Theorem 4.1's proof structure: the equilibrium Jacobian E is a projection.
"""
import numpy as np
import pytest

import oracle as O
import physics as P

CASES = [(O.EULER, 1), (O.EULER, 2), (O.SWE, 1), (O.SWE, 2), (O.ADVECTION, 1), (O.ADVECTION, 2)]


def _state(rng, system, d):
    if system == O.EULER:
        return P.random_euler_state(rng, d)
    if system == O.SWE:
        return P.random_swe_state(rng, d)
    return np.array([rng.uniform(-2, 2)])


def _flux_fn(system, cfg):
    if system == O.EULER:
        return lambda U, j: P.euler_flux(U, j, cfg.gamma)
    if system == O.SWE:
        return lambda U, j: P.swe_flux(U, j, cfg.g)
    return lambda U, j: np.array([cfg.adv[j] * U[0]])


@pytest.mark.parametrize("system,d", CASES)
def test_moment_identities(system, d):
    rng = np.random.default_rng(10 + 3 * system + d)
    cfg = O.make_cfg(system, d, 8, 8, adv=(0.7, -1.3))
    Q = 2 * d + 1
    e = np.zeros((Q, d))
    for j in range(d):
        e[1 + j, j] = 1.0
        e[1 + d + j, j] = -1.0
    for _ in range(20):
        U = _state(rng, system, d)
        alpha = rng.uniform(0.5, 3.0, d)
        lam = rng.uniform(1.0, 2.0) * alpha.sum()
        a, b = O.lf_coeffs(d, alpha, lam)
        v = lam * e
        # (2.7)
        assert abs(a.sum() - 1.0) < 1e-14
        np.testing.assert_allclose(b.sum(axis=0), 0.0, atol=1e-15)
        np.testing.assert_allclose(v.T @ a, 0.0, atol=1e-13)
        np.testing.assert_allclose(v.T @ b, np.eye(d), atol=1e-13)
        # (2.4)
        feq = O.equilibrium(cfg, U, alpha, lam)
        np.testing.assert_allclose(feq.sum(axis=0), U, rtol=1e-14, atol=1e-14)
        for j in range(d):
            Fj = _flux_fn(system, cfg)(U, j)
            np.testing.assert_allclose((v[:, j:j + 1] * feq).sum(axis=0), Fj, rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(O.flux(cfg, j, U), Fj, rtol=1e-14, atol=1e-14)
        # (2.20) written out: f_0 = (1 - sum alpha/lam) U, f_{+-j} = (alpha_j U +- F_j)/(2 lam)
        np.testing.assert_allclose(feq[0], (1 - alpha.sum() / lam) * U, rtol=1e-13, atol=1e-14)
        for j in range(d):
            Fj = _flux_fn(system, cfg)(U, j)
            np.testing.assert_allclose(feq[1 + j], (alpha[j] * U + Fj) / (2 * lam), rtol=1e-13, atol=1e-14)
            np.testing.assert_allclose(feq[1 + d + j], (alpha[j] * U - Fj) / (2 * lam), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("system,d", [c for c in CASES if c[0] != O.ADVECTION])
def test_left_eigenvectors(system, d):
    rng = np.random.default_rng(20 + 3 * system + d)
    cfg = O.make_cfg(system, d, 8, 8)
    for _ in range(20):
        U = _state(rng, system, d)
        for j in range(d):
            L = O.left_eigvecs(cfg, j, U)
            if system == O.EULER:
                R, lam = P.euler_right_eigvecs(U, j)
                A = P.jacobian_fd(lambda V, jj: P.euler_flux(V, jj), U, j)
            else:
                R, lam = P.swe_right_eigvecs(U, j)
                A = P.jacobian_fd(lambda V, jj: P.swe_flux(V, jj), U, j)
            np.testing.assert_allclose(L @ R, np.eye(len(U)), atol=1e-12)
            np.testing.assert_allclose(L @ A @ R, np.diag(lam), atol=1e-6)
            # eigenvalue bound |u_n| + c equals the largest |eigenvalue| of A
            ev = np.linalg.eigvals(A)
            assert abs(O.max_speed(cfg, j, U) - np.max(np.abs(ev))) < 1e-6


def test_advection_speed_and_projection():
    cfg = O.make_cfg(O.ADVECTION, 2, 8, 8, adv=(0.7, -1.3))
    U = np.array([0.3])
    assert O.max_speed(cfg, 0, U) == 0.7
    assert O.max_speed(cfg, 1, U) == 1.3
    assert O.left_eigvecs(cfg, 1, U).tolist() == [[1.0]]


@pytest.mark.parametrize("system,d", [(O.EULER, 2), (O.SWE, 2), (O.EULER, 1)])
def test_equilibrium_jacobian_is_projection(system, d):
    """E_k = a_k I + sum_j b_kj A_j and E = [E_k](I,...,I): sum_k E_k = I makes
    E a rank-m projection (proof of Theorem 4.1), so E @ E == E."""
    rng = np.random.default_rng(5)
    cfg = O.make_cfg(system, d, 8, 8)
    U = _state(rng, system, d)
    m, Q = len(U), 2 * d + 1
    alpha = np.array([1.3, 0.9][:d])
    lam = 2.5 * alpha.sum()
    # Jacobian of the equilibrium by finite differences of the oracle's f^eq
    Ek = np.zeros((Q, m, m))
    for c in range(m):
        h = 1e-6 * max(1.0, abs(U[c]))
        up, um = U.copy(), U.copy()
        up[c] += h
        um[c] -= h
        Ek[:, :, c] = (O.equilibrium(cfg, up, alpha, lam) - O.equilibrium(cfg, um, alpha, lam)) / (2 * h)
    E = np.concatenate([np.tile(Ek[k], (1, Q)) for k in range(Q)], axis=0)
    np.testing.assert_allclose(Ek.sum(axis=0), np.eye(m), atol=1e-8)
    np.testing.assert_allclose(E @ E, E, atol=1e-7)
    assert np.linalg.matrix_rank(E, tol=1e-6) == m
