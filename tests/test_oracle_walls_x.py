"""Pins of the oracle's walls on the x edges and at corners (Sec. 6; readings
Q11 and Q20), against properties that do not use the new code's formulas:

- Transposition: a plate with walls on its y edges (periodic in x) and the
  transposed plate with the same walls on its x edges (periodic in y) solve
  the same problem with the axes swapped; the D2Q9 lattice, the central
  differences and the isotropic material are symmetric under the swap. The
  y-wall code is itself pinned (resonance tests), so the x-wall code must
  reproduce its results transposed.
- A uniformly translating block bounded by four traction-free walls is an
  exact solution (no strain, no stress): the anti-bounce-back rule returns
  the equilibrium populations, corners included.
- A block pulled symmetrically at its top and bottom edges, free at its
  sides, stays mirror-symmetric about both centre lines.
- A block at rest between walls with zero loads stays at rest.
- Loaded blocks settle to the homogeneous states of the continuum problem:
  slow uniaxial tension to the neo-Hooke uniaxial-stress stretch (one scalar
  equation, solved here with a root finder), pure shear to F = cI + g(e1e2 +
  e2e1) with J = 1 and g = tau / (2 mu) (closed form). The nonlinear parts of
  both answers are larger than the tolerances, so a linear or wrong material
  response at the walls fails them.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O

N_, D_ = O.NEUMANN_T, O.DIRICHLET_J


def _run(p, u0, v0, n, loads=None):
    s = O.Solver(p, u0, v0)
    for k in range(n):
        if loads:
            for edge, val in loads(k).items():
                s.set_boundary_value(edge, val)
        s.step(1)
    u, v, P = s.fields()
    return u, v, P, s


def _T(a):
    """transpose a [2][ny][nx] vector field: swap components and axes"""
    return np.ascontiguousarray(a[::-1].transpose(0, 2, 1))


def _T2(P):
    return np.ascontiguousarray(P[::-1, ::-1].transpose(0, 1, 3, 2))


@pytest.mark.parametrize("scheme", [O.PC, O.EXPLICIT])
@pytest.mark.parametrize("lo,hi", [(D_, N_), (N_, N_), (D_, D_)])
def test_x_walls_are_the_transposed_y_walls(scheme, lo, hi):
    nx, ny, n = 30, 14, 60
    rng = np.random.Generator(np.random.PCG64(4))
    u0 = 0.02 * rng.standard_normal((2, ny, nx))
    v0 = 0.01 * rng.standard_normal((2, ny, nx))
    vlo = (0.001, -0.002) if lo == D_ else (0.004, 0.003)
    vhi = (0.0, 0.002) if hi == D_ else (-0.003, 0.005)
    py = O.Params(nx=nx, ny=ny, lam=0.07, mu=0.05, tau_over_dt=0.9, scheme=scheme, body=(0.001, -0.002),
                  bc_ymin=lo, bc_ymax=hi, val_ymin=vlo, val_ymax=vhi)
    px = O.Params(nx=ny, ny=nx, lam=0.07, mu=0.05, tau_over_dt=0.9, scheme=scheme, body=(-0.002, 0.001),
                  bc_xmin=lo, bc_xmax=hi, val_xmin=vlo[::-1], val_xmax=vhi[::-1])
    uy, vy, Py, _ = _run(py, u0, v0, n)
    ux, vx, Px, _ = _run(px, _T(u0), _T(v0), n)
    for a, b in ((ux, _T(uy)), (vx, _T(vy)), (Px, _T2(Py))):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_translation_between_four_free_walls_is_exact():
    nx, ny, n = 20, 16, 50
    vel = np.array([0.013, -0.007])
    p = O.Params(nx=nx, ny=ny, lam=0.1, mu=0.05, tau_over_dt=0.8, bc_xmin=N_, bc_xmax=N_, bc_ymin=N_, bc_ymax=N_)
    v0 = np.broadcast_to(vel[:, None, None], (2, ny, nx)).copy()
    u, v, P, s = _run(p, np.zeros((2, ny, nx)), v0, n)
    t = n * O.dt(p)
    assert np.abs(v - v0).max() <= 1e-14
    assert np.abs(u - v0 * t).max() <= 1e-13 * np.abs(vel).max() * t
    assert np.abs(P).max() <= 1e-14


def test_symmetric_tension_keeps_both_mirror_symmetries():
    n, steps, T = 24, 120, 0.02
    p = O.Params(nx=n, ny=n, dx=1.0 / n, lam=1.0, mu=1.0, tau_over_dt=0.8,
                 bc_xmin=N_, bc_xmax=N_, bc_ymin=N_, bc_ymax=N_)
    dt = O.dt(p)

    def loads(k):
        f = T * min(k * dt, 1.0)
        return {"ymax": (0.0, f), "ymin": (0.0, -f)}

    z = np.zeros((2, n, n))
    u, v, P, s = _run(p, z, z.copy(), steps, loads)
    scale = np.abs(u).max()
    assert scale > 1e-4
    # mirror x -> -x: u_x odd, u_y even; mirror y -> -y: u_x even, u_y odd
    assert np.abs(u[0] + u[0][:, ::-1]).max() <= 1e-12 * scale
    assert np.abs(u[1] - u[1][:, ::-1]).max() <= 1e-12 * scale
    assert np.abs(u[0] - u[0][::-1, :]).max() <= 1e-12 * scale
    assert np.abs(u[1] + u[1][::-1, :]).max() <= 1e-12 * scale
    # the block is pulled apart: top moves up, bottom down, sides move in
    assert u[1][-1, n // 2] > 0 > u[1][0, n // 2]
    assert u[0][n // 2, 0] > 0 > u[0][n // 2, -1]


@pytest.mark.parametrize("kinds", [(D_, D_, D_, D_), (N_, N_, N_, N_), (D_, N_, N_, D_)])
def test_rest_between_walls_stays_at_rest(kinds):
    p = O.Params(nx=12, ny=10, lam=0.1, mu=0.05, bc_xmin=kinds[0], bc_xmax=kinds[1], bc_ymin=kinds[2],
                 bc_ymax=kinds[3])
    z = np.zeros((2, 10, 12))
    u, v, P, s = _run(p, z, z.copy(), 30)
    assert np.abs(u).max() == 0.0 and np.abs(v).max() == 0.0


def test_unpaired_periodic_edges_are_rejected():
    p = O.Params(nx=12, ny=10, bc_xmin=N_, bc_xmax=O.PERIODIC)
    with pytest.raises(ValueError):
        O.Solver(p, np.zeros((2, 10, 12)), np.zeros((2, 10, 12)))


def _edge_stretch(u, n):
    """mean stretches (x, y) between the outermost node columns / rows"""
    L = 1.0 - 1.0 / n
    return (1.0 + (u[0][:, -1].mean() - u[0][:, 0].mean()) / L,
            1.0 + (u[1][-1, :].mean() - u[1][0, :].mean()) / L)


def test_slow_tension_settles_to_uniaxial_stress():
    """Top and bottom pulled with T = 0.2 mu, ramped over t = 10, sides free,
    tau/dt = 0.55 (the Sec. 7 value, reading Q24); the stretches averaged
    over t in [10, 16] against the homogeneous solution F = diag(a, b) with
    P11 = 0, P22 = T of the Sec. 7 energy, to a few per cent of their
    nonlinear parts (the traction walls pass T* exactly, reading Q11)."""
    n, T, lam, mu, t_ramp, t_end = 40, 0.2, 1.0, 1.0, 10.0, 16.0
    # P11 = 0 gives a^2 = (mu + lam/2) / (mu + lam b^2 / 2); then P22(b) = T
    a_of = lambda b: np.sqrt((mu + lam / 2) / (mu + lam * b * b / 2))
    P22 = lambda b: mu * (b - 1 / b) + lam / 2 * ((a_of(b) * b) ** 2 - 1) / b - T
    b = brentq(P22, 1.0, 1.5, xtol=1e-15)
    a = a_of(b)
    # linear elasticity (plane strain): eps_yy = T (lam + 2mu) / (4 mu (lam + mu)), eps_xx = -T lam / (4 mu (lam + mu))
    b_lin, a_lin = 1 + T * (lam + 2 * mu) / (4 * mu * (lam + mu)), 1 - T * lam / (4 * mu * (lam + mu))
    p = O.Params(nx=n, ny=n, dx=1.0 / n, lam=lam, mu=mu, tau_over_dt=0.55,
                 bc_xmin=N_, bc_xmax=N_, bc_ymin=N_, bc_ymax=N_)
    s = O.Solver(p, np.zeros((2, n, n)), np.zeros((2, n, n)))
    dt = O.dt(p)
    hist = []
    for k in range(int(round(t_end / dt))):
        f = T * min(k * dt / t_ramp, 1.0)
        s.set_boundary_value("ymax", (0.0, f))
        s.set_boundary_value("ymin", (0.0, -f))
        s.step(1)
        if k * dt > t_ramp and k % 3 == 0:
            hist.append(_edge_stretch(s.u, n))
    ax, by = np.mean(hist, axis=0)
    assert abs(by - b) < 0.02 * abs(b - b_lin)
    assert abs(ax - a) < 0.05 * abs(a - a_lin)


def test_pure_shear_settles_to_the_homogeneous_state():
    """The shear workload of Sec. 7.1 read as pure shear (tangential traction
    tau = 0.05 mu on all four edges, ramped over t = 1), run to t = 16: the
    shear H12 = H21 averaged over t in [12, 16] against g = tau / (2 mu), and
    the normal strains against the second-order c - 1 = sqrt(1 + g^2) - 1."""
    n, tau, t_end = 40, 0.05, 16.0
    g = tau / 2.0
    c1 = np.sqrt(1.0 + g * g) - 1.0
    p = O.Params(nx=n, ny=n, dx=1.0 / n, lam=1.0, mu=1.0, tau_over_dt=0.8,
                 bc_xmin=N_, bc_xmax=N_, bc_ymin=N_, bc_ymax=N_)
    s = O.Solver(p, np.zeros((2, n, n)), np.zeros((2, n, n)))
    dt = O.dt(p)
    L = 1.0 - 1.0 / n
    hist = []
    for k in range(int(round(t_end / dt))):
        f = tau * min(k * dt, 1.0)
        s.set_boundary_value("ymax", (f, 0.0))
        s.set_boundary_value("ymin", (-f, 0.0))
        s.set_boundary_value("xmax", (0.0, f))
        s.set_boundary_value("xmin", (0.0, -f))
        s.step(1)
        if k * dt > t_end - 4.0 and k % 3 == 0:
            u = s.u
            hist.append(((u[0][-1, :].mean() - u[0][0, :].mean()) / L, (u[1][:, -1].mean() - u[1][:, 0].mean()) / L,
                         _edge_stretch(u, n)[0] - 1.0, _edge_stretch(u, n)[1] - 1.0))
    H12, H21, H11, H22 = np.mean(hist, axis=0)
    assert abs(H12 - g) < 0.03 * g and abs(H21 - g) < 0.03 * g
    # J = 1: no volume change to first order; the normal strains are the nonlinear c - 1
    assert abs(H11 - c1) < 0.4 * c1 and abs(H22 - c1) < 0.4 * c1
