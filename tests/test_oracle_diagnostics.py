"""Pins of the oracle's diagnostics (momentum, mass moment, energy, min J,
largest Green-Lagrange strain, unstable flag) against values computed here
without the oracle's reduction code:

- a uniform translation has momentum N rho0 v and kinetic energy
  N rho0 |v|^2 / 2 dX^2 exactly, and no strain;
- on a smooth prescribed periodic state the displacement gradient is taken
  here by np.roll central differences; det F comes from np.linalg.det, the
  largest strain from np.linalg.eigvalsh of E = (F^T F - I)/2, and the energy
  density from the oracle's pointwise W (pinned separately as the potential
  of P, eq. (27)) summed here;
- the mass moment is the plain sum of the oracle's own populations;
- a state with J <= 0 somewhere raises the flag.
"""
import numpy as np

from oracle import oracle as O


def _smooth_state(n, dx, amp):
    y, x = np.mgrid[0:n, 0:n] * (2 * np.pi / n)
    u = amp * n * dx * np.array([0.3 * np.sin(x + 2 * y) + 0.1 * np.cos(3 * y),
                                 0.2 * np.cos(2 * x - y) - 0.15 * np.sin(x)])
    v = np.array([0.01 * np.cos(x) * np.sin(y), -0.02 * np.sin(2 * x + y)])
    return u, v


def _grad(u, dx):
    """H[a][b] = d_b u_a by periodic central differences."""
    d = lambda a, ax: (np.roll(a, -1, axis=ax) - np.roll(a, 1, axis=ax)) / (2 * dx)
    return np.array([[d(u[a], 1), d(u[a], 0)] for a in range(2)])


def test_uniform_translation_energy_and_momentum():
    n, dx, rho0 = 12, 0.5, 1.3
    vel = np.array([0.031, -0.017])
    p = O.Params(nx=n, ny=n, dx=dx, rho0=rho0, lam=0.1, mu=0.05)
    s = O.Solver(p, np.zeros((2, n, n)), np.broadcast_to(vel[:, None, None], (2, n, n)).copy())
    d = s.diagnostics()
    assert np.allclose(d["momentum"], n * n * rho0 * vel, rtol=1e-14, atol=0)
    assert abs(d["energy"] - n * n * 0.5 * rho0 * vel @ vel * dx * dx) <= 1e-14 * d["energy"]
    assert d["min_J"] == 1.0 and d["max_strain"] == 0.0 and not d["unstable"]


def test_diagnostics_of_a_prescribed_smooth_state():
    n, dx, rho0, lam, mu = 24, 0.25, 0.9, 0.13, 0.05
    u, v = _smooth_state(n, dx, 0.02)
    p = O.Params(nx=n, ny=n, dx=dx, rho0=rho0, lam=lam, mu=mu)
    s = O.Solver(p, u, v)
    d = s.diagnostics()
    H = _grad(u, dx)
    F = H + np.eye(2)[:, :, None, None]
    Fm = F.transpose(2, 3, 0, 1)  # [y][x][2][2]
    J = np.linalg.det(Fm)
    E = 0.5 * (np.swapaxes(Fm, -1, -2) @ Fm - np.eye(2))
    emax = np.abs(np.linalg.eigvalsh(E)).max()
    W = sum(O.strain_energy(lam, mu, Fm[yy, xx] - np.eye(2)) for yy in range(n) for xx in range(n))
    kin = 0.5 * rho0 * (v ** 2).sum()
    assert abs(d["min_J"] - J.min()) <= 1e-14
    assert abs(d["max_strain"] - emax) <= 1e-13 * emax
    assert abs(d["energy"] - (kin + W) * dx * dx) <= 1e-12 * d["energy"]
    assert np.allclose(d["momentum"], rho0 * v.sum(axis=(1, 2)), rtol=0, atol=1e-15 * n * n)
    assert W > 0.1 * kin  # the check covers both parts of the energy
    assert not d["unstable"]


def test_mass_moment_is_the_sum_of_the_populations_after_steps():
    n = 20
    u, v = _smooth_state(n, 1.0, 0.01)
    s = O.Solver(O.Params(nx=n, ny=n), u, v)
    s.step(7)
    d = s.diagnostics()
    total = s.f.sum()
    assert abs(d["mass_moment"] - total) <= 1e-13 * np.abs(s.f).sum()
    # and it moves with the state (not a constant of the run)
    assert np.abs(s.f.sum(axis=0)).max() > 1e-6


def test_unstable_flag_on_inverted_elements():
    n = 16
    x = np.arange(n)[None, :] * np.ones((n, 1))
    u = np.zeros((2, n, n))
    # du_x/dx reaches -1.5 near x = n/2: F11 < 0 there, so J < 0
    u[0] = -1.5 * n / (2 * np.pi) * np.sin(2 * np.pi * x / n)
    s = O.Solver(O.Params(nx=n, ny=n), u, np.zeros((2, n, n)))
    d = s.diagnostics()
    assert d["unstable"] and d["min_J"] < 0
