"""Test-side physics of the balance laws (Section 5 systems), in numpy.

Fluxes written from the PDEs, Jacobians by central finite differences, and
right eigenvectors in Toro's textbook form.  Independent of the oracle; used
to pin its per-state functions and to build textbook special cases.
"""
import numpy as np


def euler_flux(U, j, gamma=1.4):
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 2
    rho, E = U[0], U[d + 1]
    vel = [U[1 + i] / rho for i in range(d)]
    p = (gamma - 1.0) * (E - 0.5 * rho * sum(v * v for v in vel))
    F = [rho * vel[j]]
    for i in range(d):
        F.append(rho * vel[j] * vel[i] + (p if i == j else 0.0))
    F.append(vel[j] * (E + p))
    return np.array(F)


def swe_flux(U, j, g=9.81):
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 1
    h = U[0]
    vel = [U[1 + i] / h for i in range(d)]
    F = [h * vel[j]]
    for i in range(d):
        F.append(h * vel[j] * vel[i] + (0.5 * g * h * h if i == j else 0.0))
    return np.array(F)


def jacobian_fd(flux, U, j, rel=1e-6):
    U = np.asarray(U, dtype=np.float64)
    m = U.shape[0]
    A = np.zeros((m, m))
    for c in range(m):
        h = rel * max(1.0, abs(U[c]))
        up, um = U.copy(), U.copy()
        up[c] += h
        um[c] -= h
        A[:, c] = (flux(up, j) - flux(um, j)) / (2 * h)
    return A


def euler_right_eigvecs(U, j, gamma=1.4):
    """Columns: u_n - c, entropy, shear (one per tangential direction),
    u_n + c (Toro's form, 1D to 3D)."""
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 2
    rho, E = U[0], U[d + 1]
    vel = np.array([U[1 + i] / rho for i in range(d)])
    q2 = float(vel @ vel)
    p = (gamma - 1.0) * (E - 0.5 * rho * q2)
    c = np.sqrt(gamma * p / rho)
    H = (E + p) / rho
    un = vel[j]
    e = np.zeros(d)
    e[j] = 1.0
    cols = [np.concatenate([[1.0], vel - c * e, [H - un * c]]),
            np.concatenate([[1.0], vel, [0.5 * q2]])]
    for t in range(d):          # shear columns, tangential directions in order
        if t == j:
            continue
        et = np.zeros(d)
        et[t] = 1.0
        cols.append(np.concatenate([[0.0], et, [vel[t]]]))
    cols.append(np.concatenate([[1.0], vel + c * e, [H + un * c]]))
    lam = [un - c, un] + [un] * (d - 1) + [un + c]
    return np.array(cols).T, np.array(lam)


def swe_right_eigvecs(U, j, g=9.81):
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 1
    h = U[0]
    vel = np.array([U[1 + i] / h for i in range(d)])
    c = np.sqrt(g * h)
    un = vel[j]
    e = np.zeros(d)
    e[j] = 1.0
    cols = [np.concatenate([[1.0], vel - c * e])]
    if d == 2:
        t = 1 - j
        et = np.zeros(2)
        et[t] = 1.0
        cols.append(np.concatenate([[0.0], et]))
    cols.append(np.concatenate([[1.0], vel + c * e]))
    lam = [un - c] + ([un] if d == 2 else []) + [un + c]
    return np.array(cols).T, np.array(lam)


def euler_max_speed(U, j, gamma=1.4):
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 2
    rho, E = U[0], U[d + 1]
    vel = [U[1 + i] / rho for i in range(d)]
    p = (gamma - 1.0) * (E - 0.5 * rho * sum(v * v for v in vel))
    return np.abs(vel[j]) + np.sqrt(gamma * p / rho)


def swe_max_speed(U, j, g=9.81):
    U = np.asarray(U, dtype=np.float64)
    h = U[0]
    return np.abs(U[1 + j] / h) + np.sqrt(g * h)


def random_euler_state(rng, d, gamma=1.4):
    rho = rng.uniform(0.2, 2.0)
    vel = rng.uniform(-1.5, 1.5, d)
    p = rng.uniform(0.1, 2.0)
    E = p / (gamma - 1) + 0.5 * rho * float(vel @ vel)
    return np.concatenate([[rho], rho * vel, [E]])


def random_swe_state(rng, d):
    h = rng.uniform(0.1, 2.0)
    vel = rng.uniform(-1.5, 1.5, d)
    return np.concatenate([[h], h * vel])


def reactive_flux(U, j, gamma=1.2, q_heat=0.0):
    """Reactive Euler flux (Section 5.4): Euler flux with rho E including
    q rho Y, plus rho Y u_j."""
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 3
    rho, E, Z = U[0], U[d + 1], U[d + 2]
    vel = [U[1 + i] / rho for i in range(d)]
    p = (gamma - 1.0) * (E - 0.5 * rho * sum(v * v for v in vel) - q_heat * Z)
    F = [rho * vel[j]]
    for i in range(d):
        F.append(rho * vel[j] * vel[i] + (p if i == j else 0.0))
    F.append(vel[j] * (E + p))
    F.append(Z * vel[j])
    return np.array(F)


def reactive_right_eigvecs(U, j, gamma=1.2, q_heat=0.0):
    """Columns in the order u_n - c, entropy, [shear], species, u_n + c.

    With E' = E - q rho Y the system is Euler plus an advected scalar; its
    right eigenvectors in (rho, m, E', rho Y) are Toro's columns extended by
    Y (acoustic, entropy), 0 (shear) and the unit species column; mapping
    back to (rho, m, E, rho Y) adds q times the last entry to the energy."""
    U = np.asarray(U, dtype=np.float64)
    d = U.shape[0] - 3
    rho, E, Z = U[0], U[d + 1], U[d + 2]
    Y = Z / rho
    vel = np.array([U[1 + i] / rho for i in range(d)])
    q2 = float(vel @ vel)
    p = (gamma - 1.0) * (E - 0.5 * rho * q2 - q_heat * Z)
    c = np.sqrt(gamma * p / rho)
    Ep = E - q_heat * Z
    H = (Ep + p) / rho
    un = vel[j]
    e = np.zeros(d)
    e[j] = 1.0
    cols = [np.concatenate([[1.0], vel - c * e, [H - un * c], [Y]]),
            np.concatenate([[1.0], vel, [0.5 * q2], [Y]])]
    for t in range(d):
        if t == j:
            continue
        sh = np.zeros(d + 3)
        sh[1 + t] = 1.0
        sh[d + 1] = vel[t]
        cols.append(sh)
    sp = np.zeros(d + 3)
    sp[d + 2] = 1.0
    cols.append(sp)
    cols.append(np.concatenate([[1.0], vel + c * e, [H + un * c], [Y]]))
    R = np.array(cols).T
    R[d + 1, :] = R[d + 1, :] + q_heat * R[d + 2, :]
    return R


def random_reactive_state(rng, d, gamma=1.2, q_heat=30.0):
    rho = rng.uniform(0.5, 2.0)
    vel = rng.uniform(-1.0, 1.0, size=d)
    p = rng.uniform(0.5, 5.0)
    Y = rng.uniform(0.0, 1.0)
    E = p / (gamma - 1.0) + 0.5 * rho * float(vel @ vel) + q_heat * rho * Y
    return np.concatenate([[rho], rho * vel, [E], [rho * Y]])
