"""Pin of a momentum wall whose value changes during a run (Sec. 6, eq. (25)
with a load history).

A momentum wall is a rigid boundary driven by its prescribed momentum j*: it
moves with velocity j*/rho0, so its displacement is the time integral of the
values in effect, continuous when j* changes. In a shear strip (periodic in
x, momentum walls at both y edges) a tangential displacement u_x(y) makes
the stress sum K = P + Pbar vanish exactly (F = [[1, g], [0, 1]], J = 1), so
the step is the linear scheme, and the numerical viscosity damps every mode.
Once both walls stop, the strip settles to a simple shear whose profile is
the straight line between the walls' final displacements, placed half a
spacing beyond the outer node rows:
  u_x(y) = U_lo + (U_hi - U_lo) (y + 1/2) / N,
with U = sum over steps of j* dt / rho0. A wall displacement taken as j* t
with the current j* would put both walls back at zero once they stop.
"""
import numpy as np

from oracle import oracle as O

D = O.DIRICHLET_J


def test_walls_stopped_after_a_load_history_hold_the_integrated_displacement():
    nx, ny, rho0 = 5, 16, 1.2
    p = O.Params(nx=nx, ny=ny, rho0=rho0, lam=0.1, mu=0.05, tau_over_dt=0.8,
                 bc_ymin=D, bc_ymax=D)
    z = np.zeros((2, ny, nx))
    s = O.Solver(p, z, z.copy())
    dt = O.dt(p)
    a, c = 2e-4, -1.5e-4
    history = [  # (steps, j* of the bottom wall, j* of the top wall)
        (150, (0.0, 0.0), (a, 0.0)),
        (100, (c, 0.0), (-0.5 * a, 0.0)),
        (80, (c, 0.0), (0.0, 0.0)),
    ]
    U_lo = U_hi = 0.0
    for n, lo, hi in history:
        s.set_boundary_value("ymin", lo)
        s.set_boundary_value("ymax", hi)
        s.step(n)
        U_lo += lo[0] * n * dt / rho0
        U_hi += hi[0] * n * dt / rho0
    s.set_boundary_value("ymin", (0.0, 0.0))
    s.set_boundary_value("ymax", (0.0, 0.0))
    s.step(8000)
    u, v, P = s.fields()
    expect = U_lo + (U_hi - U_lo) * (np.arange(ny) + 0.5) / ny
    scale = max(abs(U_lo), abs(U_hi))
    assert abs(U_hi) > 0.5 * scale and abs(U_lo) > 0.5 * scale
    assert np.abs(u[0] - expect[:, None]).max() <= 1e-9 * scale
    assert np.abs(u[1]).max() <= 1e-12 * scale
    assert np.abs(v).max() <= 1e-12 * scale
    # the walls' displacements the oracle carries are the integrals
    assert abs(s.wall[2, 0] - U_lo) <= 1e-15 * scale * 400 and abs(s.wall[3, 0] - U_hi) <= 1e-15 * scale * 400


def test_uniform_translation_between_moving_walls_is_exact():
    """Both walls and the material move with one velocity: u = v t exactly,
    for momentum walls on every edge (the wall displacement enters the
    ghost displacements of every edge)."""
    n, steps = 9, 60
    vel = np.array([0.011, -0.006])
    rho0 = 0.8
    js = tuple(rho0 * vel)
    p = O.Params(nx=n, ny=n, rho0=rho0, lam=0.1, mu=0.05, bc_xmin=D, bc_xmax=D, bc_ymin=D, bc_ymax=D,
                 val_xmin=js, val_xmax=js, val_ymin=js, val_ymax=js)
    v0 = np.broadcast_to(vel[:, None, None], (2, n, n)).copy()
    s = O.Solver(p, np.zeros((2, n, n)), v0)
    s.step(steps)
    u, v, P = s.fields()
    t = steps * O.dt(p)
    assert np.abs(v - v0).max() <= 1e-15
    assert np.abs(u - v0 * t).max() <= 1e-13 * np.abs(vel).max() * t
    assert np.abs(P).max() <= 1e-13
