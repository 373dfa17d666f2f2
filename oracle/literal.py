"""Algorithm 1 read literally, on a periodic lattice, in plain NumPy.

TEST INFRASTRUCTURE. It exists to show, inside the test suite, why the oracle
and the GPU path depart from the printed algorithm in one place (reading R1):
read literally, the equilibrium of Algorithm 1 takes the Poisson stress
Pbar(H(u)) of eq. (15), recomputed from the displacement at the end of every
step, in place of the populations' own second moment, and that scheme grows
without bound. It shares no code with ``lbm_oracle.c`` or ``modal.py``.

Periodic edges only, lattice units (dX = dt = rho0 = 1, C_s^2 = 1/3, so
mu_L = 1/3 and lam_L = (lam/mu)/3), no body force. One step, in the printed
order:

1. source 1S = div(Pbar + P) from the stresses of the last update (explicit);
2. equilibrium (20) with r, j and Pbar, source populations (22), collision (4);
3. streaming (5);
4. r = sum f, j = sum C f + 1S/2 (6) with the same 1S;
5. u += (j_new + j_old)/2 (24), then H = grad u, P(H) (neo-Hooke, eq. (27))
   and Pbar(H) (eq. (15)) for the next step.

Central differences are np.roll differences; the velocity set is listed
below in an order of its own.
"""
from __future__ import annotations

import numpy as np

# (ex, ey) and weights of D2Q9 (Sec. 3)
VEL = np.array([(1, 1), (0, 1), (-1, 1), (1, 0), (0, 0), (-1, 0), (1, -1), (0, -1), (-1, -1)])
WGT = np.array([1 / 36, 1 / 9, 1 / 36, 1 / 9, 4 / 9, 1 / 9, 1 / 36, 1 / 9, 1 / 36])


def _dx(a):
    return 0.5 * (np.roll(a, -1, axis=-1) - np.roll(a, 1, axis=-1))


def _dy(a):
    return 0.5 * (np.roll(a, -1, axis=-2) - np.roll(a, 1, axis=-2))


def _stresses(u, lam, mu):
    """P(H) of the compressible neo-Hooke law and Pbar(H), [2][2][ny][nx]."""
    H = np.array([[_dx(u[0]), _dy(u[0])], [_dx(u[1]), _dy(u[1])]])
    F = H + np.eye(2)[:, :, None, None]
    J = F[0, 0] * F[1, 1] - F[0, 1] * F[1, 0]
    # F^-T = cof F / J
    FiT = np.array([[F[1, 1], -F[1, 0]], [-F[0, 1], F[0, 0]]]) / J
    P = mu * (F - FiT) + 0.5 * lam * (J * J - 1.0) * FiT
    tr = H[0, 0] + H[1, 1]
    Pb = -mu * (H + H.transpose(1, 0, 2, 3) + tr * np.eye(2)[:, :, None, None])
    return P, Pb


def _feq(r, j, Pb):
    s2 = 1.0 / 3.0
    out = np.empty((9,) + r.shape)
    for i, (ex, ey) in enumerate(VEL):
        c = (ex, ey)
        quad = sum((Pb[a, b] - (r * s2 if a == b else 0.0)) * (c[a] * c[b] - (s2 if a == b else 0.0))
                   for a in range(2) for b in range(2))
        out[i] = WGT[i] * (r + (ex * j[0] + ey * j[1]) / s2 + quad / (2.0 * s2 * s2))
    return out


class Literal:
    """State of one periodic plate under the printed Algorithm 1."""

    def __init__(self, u0, v0, lam_over_mu, tau_over_dt):
        self.mu = 1.0 / 3.0
        self.lam = lam_over_mu / 3.0
        self.omega = 1.0 / tau_over_dt
        self.u = np.array(u0, dtype=np.float64)
        self.j = np.array(v0, dtype=np.float64)
        self.P, self.Pb = _stresses(self.u, self.lam, self.mu)
        # initial moments: r = -rho0 div u (eq. (18)), j = rho0 v, Pbar(H(u0))
        self.r = -(_dx(self.u[0]) + _dy(self.u[1]))
        self.f = _feq(self.r, self.j, self.Pb)

    def step(self):
        K = self.Pb + self.P
        S = np.array([_dx(K[a, 0]) + _dy(K[a, 1]) for a in range(2)])
        feq = _feq(self.r, self.j, self.Pb)
        psi = np.array([3.0 * WGT[i] * (VEL[i, 0] * S[0] + VEL[i, 1] * S[1]) for i in range(9)])
        fcol = self.f - self.omega * (self.f - feq) + (1.0 - 0.5 * self.omega) * psi
        self.f = np.array([np.roll(fcol[i], (VEL[i, 1], VEL[i, 0]), axis=(0, 1)) for i in range(9)])
        self.r = self.f.sum(axis=0)
        jnew = np.array([np.tensordot(VEL[:, a], self.f, axes=1) for a in range(2)]) + 0.5 * S
        self.u = self.u + 0.5 * (jnew + self.j)
        self.j = jnew
        self.P, self.Pb = _stresses(self.u, self.lam, self.mu)
