"""Why the oracle departs from the printed Algorithm 1 (reading R1).

Algorithm 1 as printed feeds the equilibrium (20) with the Poisson stress
Pbar(H(u)) of eq. (15), recomputed from the displacement after every step.
The oracle and the GPU path feed it the populations' own second moment
instead (Sec. 4-5: the LBM evolves Pbar through the chain (19)). These tests
keep the evidence for that reading in the suite:

- the per-mode model with the literal equilibrium grows about 1.5 times per
  step at lambda = mu, tau/dt = 0.8 (any lambda/mu and tau/dt probed), while
  reading R1 with the predictor-corrector is neutral;
- an independent real-space NumPy stepper of the printed algorithm
  (``oracle/literal.py``) follows the per-mode model's literal step on a
  single Fourier mode (two codes, one answer);
- run on a grid from a tiny seeded disturbance, the literal scheme grows by
  many orders of magnitude within a hundred steps, where the oracle on the
  same input stays at its start amplitude.
"""
import numpy as np
import pytest

from oracle import literal as L
from oracle import modal as M
from oracle import oracle as O


@pytest.mark.parametrize("lam_over_mu", [0.5, 1.0, 2.0, 5.0])
def test_literal_equilibrium_grows_where_reading_r1_is_neutral(lam_over_mu):
    lit = M.max_amplification(lam_over_mu, 0.8, "literal", nk=17)
    pc = M.max_amplification(lam_over_mu, 0.8, "pc", nk=17)
    assert lit > 1.2, lit
    assert abs(pc - 1.0) < 1e-12, pc


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.5])
def test_literal_grows_for_every_relaxation_time(tau):
    assert M.max_amplification(1.0, tau, "literal", nk=17) > 1.2


def _mode_fields(n, k, hat):
    """Real fields Re(hat e^{i k . X}) on an n x n grid, [len(hat)][n][n]."""
    y, x = np.mgrid[0:n, 0:n]
    ph = np.exp(1j * (k[0] * x + k[1] * y))
    return np.real(np.asarray(hat)[:, None, None] * ph[None])


@pytest.mark.parametrize("modes", [(1, 2), (3, -1), (0, 5)])
def test_real_space_literal_step_follows_the_mode_model(modes):
    n = 16
    k = (2 * np.pi * modes[0] / n, 2 * np.pi * modes[1] / n)
    lam_over_mu, tau = 2.0, 0.8
    u_hat = 1e-8 * np.array([0.7 + 0.2j, -0.4 + 0.5j])
    j_hat = 1e-8 * np.array([0.1 - 0.3j, 0.6 + 0.1j])
    state = M.initial_state(k, u_hat, j_hat, lam_over_mu)
    nxt = M.step_map(state, k, lam_over_mu, tau, "literal")
    lit = L.Literal(_mode_fields(n, k, u_hat), _mode_fields(n, k, j_hat), lam_over_mu, tau)
    # populations in the mode model's velocity order
    order = [int(np.flatnonzero((L.VEL == M.E[i].astype(int)).all(axis=1))[0]) for i in range(9)]
    f0 = _mode_fields(n, k, state[0:9])
    assert np.abs(lit.f[order] - f0).max() <= 1e-6 * np.abs(f0).max()
    lit.step()
    ref_f, ref_u, ref_j = _mode_fields(n, k, nxt[0:9]), _mode_fields(n, k, nxt[9:11]), _mode_fields(n, k, nxt[11:13])
    assert np.abs(lit.f[order] - ref_f).max() <= 1e-6 * np.abs(ref_f).max()
    assert np.abs(lit.u - ref_u).max() <= 1e-6 * np.abs(ref_u).max()
    assert np.abs(lit.j - ref_j).max() <= 1e-6 * np.abs(ref_j).max()


def test_literal_scheme_blows_up_where_the_oracle_does_not():
    n, steps = 32, 120
    rng = np.random.Generator(np.random.PCG64(7))
    x = np.arange(n)
    v0 = np.zeros((2, n, n))
    v0[1] = 1e-6 * np.sin(2 * np.pi * x / n)[None, :]
    v0 += 1e-12 * rng.standard_normal((2, n, n))
    u0 = np.zeros((2, n, n))
    # lattice units: dx = rho0 = 1, mu = 1/3 gives dt = 1; lambda = mu
    lit = L.Literal(u0, v0, 1.0, 0.8)
    blown = None
    with np.errstate(all="ignore"):
        for k in range(steps):
            lit.step()
            g = np.abs(lit.j).max() / np.abs(v0).max()
            if not np.isfinite(g) or g > 1e6:
                blown = k + 1
                break
    p = O.Params(nx=n, ny=n, dx=1.0, rho0=1.0, lam=1.0 / 3.0, mu=1.0 / 3.0, tau_over_dt=0.8)
    assert abs(O.dt(p) - 1.0) < 1e-15
    ref = O.Solver(p, u0, v0)
    ref.step(steps)
    grow_ref = np.abs(ref.j).max() / np.abs(v0).max()
    assert blown is not None and blown < steps, blown
    assert grow_ref < 1.01, grow_ref
