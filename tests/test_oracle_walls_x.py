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
"""
import numpy as np
import pytest

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
