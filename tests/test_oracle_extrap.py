"""Pins of the oracle's extrapolation variant (the closing paragraphs of
Sec. 5): the source of the moment step is taken at t + dt from a predictor
displacement whose j at t + dt is extrapolated linearly, 2 j(t) - j(t - dt).

- A standing P-wave (the only kind the source acts on when lam != mu) keeps
  second-order phase convergence against the continuum frequency
  w = k sqrt((lam + 2 mu) / rho0). Its phase error agrees with the
  predictor-corrector's to 2 % and differs from the explicit level's (source
  at t) by more than 40 %, so the variant evaluates the source at t + dt.
- Growth for lam > mu, which the extrapolation brings and the
  predictor-corrector does not (a property of the method, recorded here).
"""
import numpy as np

from oracle import oracle as O


def _pwave_phase_errors(scheme, lam, mu=0.05, sizes=(64, 128, 256)):
    L, A, m_cross = 64.0, 1e-4, 16
    k = 2 * np.pi / L
    w = np.sqrt((lam + 2 * mu) / 1.0) * k
    errs = []
    for N in sizes:
        dx = L / N
        p = O.Params(nx=N, ny=5, dx=dx, lam=lam, mu=mu, scheme=scheme)
        dt = O.dt(p)
        x = np.arange(N) * dx
        v0 = np.zeros((2, 5, N))
        v0[0] = A * np.sin(k * x)[None, :]
        s = O.Solver(p, np.zeros((2, 5, N)), v0)
        probe = N // 4
        crossings, prev = [], 0.0
        while len(crossings) < m_cross:
            s.step(1)
            cur = s.u[0, 0, probe]
            if s.step_index > 1 and np.sign(cur) != np.sign(prev) and prev != 0.0:
                crossings.append((s.step_index - 1 + prev / (prev - cur)) * dt)
            prev = cur
        t_exact = m_cross * np.pi / w
        errs.append((crossings[-1] - t_exact) / t_exact)
    return np.array(errs)


def test_extrapolated_source_keeps_second_order_phase():
    ex = _pwave_phase_errors(O.EXTRAP, 0.025)
    pc = _pwave_phase_errors(O.PC, 0.025)
    exp_ = _pwave_phase_errors(O.EXPLICIT, 0.025, sizes=(64,))
    order = np.log2(np.abs(ex[:-1]) / np.abs(ex[1:]))
    assert np.all(order > 1.9), (ex, order)
    assert np.all(np.abs(ex - pc) < 0.02 * np.abs(pc)), (ex, pc)
    assert abs(exp_[0] - pc[0]) > 0.4 * abs(pc[0]), (exp_, pc)


def test_extrapolation_grows_for_lambda_above_mu():
    n, steps = 16, 200
    rng = np.random.Generator(np.random.PCG64(9))
    u0 = 1e-8 * rng.standard_normal((2, n, n))
    out = {}
    for scheme in (O.EXTRAP, O.PC):
        p = O.Params(nx=n, ny=n, lam=0.1, mu=0.05, scheme=scheme)
        s = O.Solver(p, u0, np.zeros((2, n, n)))
        s.step(steps)
        out[scheme] = np.abs(s.u).max() / np.abs(u0).max()
    assert out[O.EXTRAP] > 1e3
    assert out[O.PC] < 10.0
