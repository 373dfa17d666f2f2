"""Per-Fourier-mode model of the linearised scheme (von Neumann analysis).

TEST INFRASTRUCTURE, independent of ``lbm_oracle.c``: it shares no code with
it and works in a different representation (one complex Fourier amplitude
per field instead of real fields on a grid), in lattice units
(dX = dt = rho0 = 1, C_s^2 = 1/3, mu_L = 1/3, lam_L = lam / (3 mu)).

On a periodic lattice one step of the method (Algorithm 1 with readings R1/R2)
maps the Fourier amplitudes of the state (f_0..f_8, u_x, u_y, j_x, j_y) at
wave vector k linearly onto themselves once the neo-Hooke law is linearised
about F = I, P ~ mu (H + H^T) + lam tr(H) I. In Fourier space:

* a central difference d_b becomes multiplication by i sin(k_b);
* pull streaming f_i(X, n+1) = f_i^col(X - e_i, n) multiplies f_i by
  exp(-i k . e_i).

The step matrix G(k) (13 x 13 complex) is assembled column by column from the
image of each unit state. Its eigenvalues give the per-step amplification and
phase of every mode: stability, wave speeds and damping.

Velocity order here: (ex, ey) over the list below; it differs from the
oracle's own order on purpose.
"""
from __future__ import annotations

import numpy as np

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
NSTATE = 13


def _stress_sum_hat(u_hat, sk, lam_l, mu_l):
    """K = P(H) + Pbar(H) for the linearised law, H_ab = i sin(k_b) u_a."""
    H = np.array([[1j * sk[b] * u_hat[a] for b in range(2)] for a in range(2)])
    tr = H[0, 0] + H[1, 1]
    P = mu_l * (H + H.T) + lam_l * tr * np.eye(2)
    Pb = -mu_l * (H + H.T + tr * np.eye(2))
    return P + Pb


def _source_hat(u_hat, sk, lam_l, mu_l):
    K = _stress_sum_hat(u_hat, sk, lam_l, mu_l)
    return np.array([sum(1j * sk[b] * K[a, b] for b in range(2)) for a in range(2)])


def step_map(state, k, lam_over_mu, tau_over_dt, scheme="pc"):
    """Apply one step to a 13-vector of Fourier amplitudes.

    scheme: "pc" (reading R2), "explicit" (the source time level printed in
    Algorithm 1), both with the populations' own second moment in the
    equilibrium (reading R1); or "literal": Algorithm 1 as printed, whose
    equilibrium takes the Poisson stress Pbar(H(u)) of the current
    displacement (eq. (15)) in place of the populations' second moment, with
    the explicit source."""
    mu_l = 1.0 / 3.0
    lam_l = lam_over_mu / 3.0
    omega = 1.0 / tau_over_dt
    sk = np.sin(np.asarray(k, dtype=float))
    f = state[0:9].astype(complex)
    u = state[9:11].astype(complex)
    j = state[11:13].astype(complex)

    S = _source_hat(u, sk, lam_l, mu_l)
    r = f.sum()
    if scheme == "literal":
        H = np.array([[1j * sk[b] * u[a] for b in range(2)] for a in range(2)])
        Pi = -mu_l * (H + H.T + (H[0, 0] + H[1, 1]) * np.eye(2))
    else:
        Pi = np.einsum("i,ia,ib->ab", f, E, E)
    A = Pi - r / 3.0 * np.eye(2)
    feq = np.array([W[i] * (r + 3.0 * E[i] @ j + 4.5 * np.sum(A * (np.outer(E[i], E[i]) - np.eye(2) / 3.0)))
                    for i in range(9)])
    psi = 3.0 * W * (E @ S)
    fcol = f - omega * (f - feq) + (1.0 - 0.5 * omega) * psi
    fnew = fcol * np.exp(-1j * (E @ np.asarray(k, dtype=float)))
    jf = E.T @ fnew
    if scheme == "pc":
        jp = jf + 0.5 * S
        up = u + 0.5 * (jp + j)
        Sp = _source_hat(up, sk, lam_l, mu_l)
    else:
        Sp = S
    jnew = jf + 0.5 * Sp
    unew = u + 0.5 * (jnew + j)
    return np.concatenate([fnew, unew, jnew])


def step_matrix(k, lam_over_mu, tau_over_dt, scheme="pc"):
    G = np.zeros((NSTATE, NSTATE), dtype=complex)
    for c in range(NSTATE):
        e = np.zeros(NSTATE, dtype=complex)
        e[c] = 1.0
        G[:, c] = step_map(e, k, lam_over_mu, tau_over_dt, scheme)
    return G


def initial_state(k, u_hat, j_hat, lam_over_mu):
    """f = f^eq(r0, j0, Pbar(H(u0))) with r0 = -div u0 (lattice units)."""
    mu_l = 1.0 / 3.0
    sk = np.sin(np.asarray(k, dtype=float))
    u_hat = np.asarray(u_hat, dtype=complex)
    j_hat = np.asarray(j_hat, dtype=complex)
    H = np.array([[1j * sk[b] * u_hat[a] for b in range(2)] for a in range(2)])
    tr = H[0, 0] + H[1, 1]
    Pb = -mu_l * (H + H.T + tr * np.eye(2))
    r = -tr
    A = Pb - r / 3.0 * np.eye(2)
    f = np.array([W[i] * (r + 3.0 * E[i] @ j_hat + 4.5 * np.sum(A * (np.outer(E[i], E[i]) - np.eye(2) / 3.0)))
                  for i in range(9)])
    return np.concatenate([f, u_hat, j_hat])


def max_amplification(lam_over_mu, tau_over_dt, scheme="pc", nk=33):
    """Largest |eigenvalue| of G(k) over an nk x nk grid of wave vectors."""
    ks = np.linspace(-np.pi, np.pi, nk)
    best = 0.0
    for kx in ks:
        for ky in ks:
            ev = np.linalg.eigvals(step_matrix((kx, ky), lam_over_mu, tau_over_dt, scheme))
            best = max(best, float(np.max(np.abs(ev))))
    return best
