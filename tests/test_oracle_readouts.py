"""Pins of the oracle's read-outs (Cauchy stress, Green-Lagrange strain,
strain-energy density) against closed forms that do not use its formulas.

- Cauchy stress of the compressible neo-Hooke law (the energy of Sec. 7):
  sigma = (mu / J)(F F^T - I) + lam (J^2 - 1) / (2 J) I, which follows from
  P = mu (F - F^-T) + lam/2 (J^2 - 1) F^-T and sigma = J^-1 P F^T; the oracle
  forms the matrix product, the pin uses the left Cauchy-Green form.
- Objectivity: a rigid rotation carries no stress and no strain.
- Simple shear and uniaxial stretch: E and sigma in closed form.
- The field routine applies the point functions to the central-difference
  gradient (Sec. 5); the pin recomputes that gradient with numpy.
"""
import numpy as np
import pytest

from oracle import oracle as O

LAM, MU = 0.7, 0.4


def _F(H):
    return np.eye(2) + np.asarray(H).reshape(2, 2)


def test_cauchy_matches_left_cauchy_green_form():
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(50):
        H = 0.3 * rng.standard_normal((2, 2))
        F = _F(H)
        J = np.linalg.det(F)
        if J < 0.3:
            continue
        expect = MU / J * (F @ F.T - np.eye(2)) + LAM * (J * J - 1.0) / (2.0 * J) * np.eye(2)
        got = O.cauchy(LAM, MU, H)
        assert np.allclose(got, expect, rtol=1e-13, atol=1e-14)
        assert abs(got[0, 1] - got[1, 0]) < 1e-14


@pytest.mark.parametrize("theta", [0.3, np.pi / 2, 2.5])
def test_rotation_is_free_of_stress_and_strain(theta):
    R = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
    H = R - np.eye(2)
    assert np.abs(O.cauchy(LAM, MU, H)).max() < 1e-15
    assert np.abs(O.green_lagrange(H)).max() < 1e-15


def test_simple_shear_strain():
    g = 0.37
    H = np.array([[0.0, g], [0.0, 0.0]])
    E = O.green_lagrange(H)
    assert np.allclose(E, [[0.0, g / 2], [g / 2, g * g / 2]], rtol=0, atol=1e-16)


def test_uniaxial_stretch():
    s = 1.23
    H = np.array([[s - 1.0, 0.0], [0.0, 0.0]])
    E = O.green_lagrange(H)
    assert np.allclose(E, [[(s * s - 1) / 2, 0], [0, 0]], rtol=0, atol=1e-16)
    sig = O.cauchy(LAM, MU, H)
    assert np.isclose(sig[0, 0], MU / s * (s * s - 1) + LAM * (s * s - 1) / (2 * s), rtol=1e-14)
    assert np.isclose(sig[1, 1], LAM * (s * s - 1) / (2 * s), rtol=1e-14)
    assert sig[0, 1] == 0.0


def test_derived_fields_use_the_central_difference_gradient():
    nx, ny = 24, 16
    rng = np.random.Generator(np.random.PCG64(3))
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    u0 = np.zeros((2, ny, nx))
    u0[0] = 0.4 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)
    u0[1] = 0.3 * np.cos(4 * np.pi * x / nx) + 0.1 * rng.standard_normal((ny, nx))
    p = O.Params(nx=nx, ny=ny, lam=LAM, mu=MU, tau_over_dt=0.8)
    s = O.Solver(p, u0, np.zeros((2, ny, nx)))
    sig, E, W = s.derived()
    # central differences on the periodic grid, component-major H[a][b] = du_a/dX_b
    H = np.empty((2, 2, ny, nx))
    for a in range(2):
        H[a, 0] = 0.5 * (np.roll(u0[a], -1, axis=1) - np.roll(u0[a], 1, axis=1))
        H[a, 1] = 0.5 * (np.roll(u0[a], -1, axis=0) - np.roll(u0[a], 1, axis=0))
    for yy, xx in [(0, 0), (5, 17), (15, 23), (9, 2)]:
        h = H[:, :, yy, xx]
        F = _F(h)
        J = np.linalg.det(F)
        expect_sig = MU / J * (F @ F.T - np.eye(2)) + LAM * (J * J - 1.0) / (2.0 * J) * np.eye(2)
        assert np.allclose(sig[:, :, yy, xx], expect_sig, rtol=1e-12, atol=1e-14)
        assert np.allclose(E[:, :, yy, xx], 0.5 * (F.T @ F - np.eye(2)), rtol=1e-12, atol=1e-15)
        IC = np.trace(F.T @ F)
        expect_W = MU / 2 * (IC - 2) + LAM / 4 * (J * J - 1) - LAM / 2 * np.log(J) - MU * np.log(J)
        assert np.isclose(W[yy, xx], expect_W, rtol=1e-12, atol=1e-15)
