"""Accuracy of the storage precisions on the 1024 x 1024 standing shear wave
(v_y = 1e-4 sin(2 pi x / 1024), lam = 0.1, mu = 0.05, tau/dt = 0.8, 5000
steps), against the FP64 oracle.

The field is uniform in y and the grid is periodic, so the exact (FP64)
solution has identical rows: the oracle runs a 1024 x 8 plate and each of its
rows is the reference for every row of the 1024 x 1024 GPU run.

Every case asserts the contract bound of its storage form (rel-L2 on u and
P: 1e-5 for FP32 storage, 1e-3 for 16-bit storage; FP64 is held to its
1e-12 scaled to the run length). Known misses are marked xfail with the
measured error:
- FP32 populations drift over 5000 steps: a slowly varying population
  rounds the same way step after step, so the error in the conserved
  momentum, and hence in u, grows with the step count (u 6e-5); plain FP32
  also rounds the accumulated displacement (P 1.8e-4), which FP32_U64 (a
  double displacement) removes (P 6e-5);
- 16-bit populations are stored as deviations from the reference
  equilibrium of their state, which is within a fraction of a percent of
  them in this smooth wave, so their rounding no longer drifts visibly.

A second case is the large-strain workload at a quarter of its size: a
1024 x 1024 periodic plate, the same calibrated peak velocity (a wave's
strain is about v / c, whatever its length) with the Gaussian filter width
scaled to 8 cells, 500 steps, peak Green-Lagrange strain about 0.2.
"""
import numpy as np
import pytest

from paper_2208_13769_amd import inputs
from tests.helpers import oracle_run

pytestmark = pytest.mark.gpu

N, STEPS = 1024, 5000


@pytest.fixture(scope="module")
def reference():
    u0, v0 = inputs.shear_wave(N, 8, 1e-4, N)
    u, v, P, _ = oracle_run(N, 8, u0, v0, STEPS)
    return u[:, :1, :], v[:, :1, :], P[:, :, :1, :]


@pytest.fixture(scope="module")
def errors(gpu, reference):
    from paper_2208_13769_amd import lbm

    ru, rv, rP = reference
    u0, v0 = inputs.shear_wave(N, N, 1e-4, N)
    out = {}

    def rel(x, r):
        return float(np.linalg.norm(x - r) / (np.linalg.norm(r) * np.sqrt(x.shape[-2])))

    for prec, rnd in [("fp64", "nearest"), ("fp32", "nearest"), ("fp32u64", "nearest"), ("fp16", "nearest"),
                      ("fp16", "stochastic"), ("bf16", "nearest"), ("bf16", "stochastic")]:
        s = lbm.Solver(N, N, 1.0, prec, "pc")
        s.set_material(1.0, 0.1, 0.05, 0.8)
        s.set_rounding(rnd, 2024)
        s.set_fields(u0, v0)
        s.step(STEPS)
        u, v, P, d, st = s.read()
        s.close()
        assert st == 0 and d.steps == STEPS
        out[prec, rnd] = (rel(u, ru), rel(v, rv), rel(P, rP))
        print(prec, rnd, "rel-L2 u %.3e v %.3e P %.3e" % out[prec, rnd], flush=True)
    return out


def _miss(reason):
    return pytest.mark.xfail(reason=reason, strict=False)


@pytest.mark.parametrize("prec,rnd,tol", [
    ("fp64", "nearest", 3e-11),
    pytest.param("fp32", "nearest", 1e-5, marks=_miss("FP32 drift over 5000 steps: u 6.0e-5, P 1.8e-4")),
    pytest.param("fp32u64", "nearest", 1e-5, marks=_miss("FP32 population drift over 5000 steps: u 6e-5, P 6e-5")),
    ("fp16", "nearest", 1e-3),
    ("fp16", "stochastic", 1e-3),
    ("bf16", "nearest", 1e-3),
    ("bf16", "stochastic", 1e-3),
])
def test_storage_precision_error_after_5000_steps(errors, prec, rnd, tol):
    eu, ev, eP = errors[prec, rnd]
    assert eu < tol and eP < tol, (prec, rnd, eu, eP)


def test_stochastic_rounding_removes_the_drift(errors):
    """BF16 (8 significant bits) still shows the drift of rounding to
    nearest; stochastic rounding takes it out."""
    assert errors["bf16", "stochastic"][0] < 0.5 * errors["bf16", "nearest"][0]


def _large_strain_case():
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "large_strain_amplitude.json")
    with open(path) as fh:
        peak = float(json.load(fh)["peak_velocity"])
    return inputs.filtered_random_velocity(1024, 1024, 8.0, 2, peak)


@pytest.fixture(scope="module")
def large_strain_reference():
    u0, v0 = _large_strain_case()
    u, v, P, d = oracle_run(1024, 1024, u0, v0, 500)
    return u, v, P


# The contract bounds on this large-strain field. Plain FP32 misses 1e-5 on
# P (1.5e-5: P differences a float displacement of a few lattice units).
@pytest.mark.parametrize("prec,tol_u,tol_P", [
    pytest.param("fp32", 1e-5, 1e-5, marks=_miss("plain FP32: P 1.5e-5 (float displacement)")),
    ("fp32u64", 1e-5, 1e-5), ("fp16", 1e-3, 1e-3), ("bf16", 1e-3, 1e-3)])
def test_large_strain_500_steps(gpu, large_strain_reference, prec, tol_u, tol_P):
    from paper_2208_13769_amd import lbm

    ru, rv, rP = large_strain_reference
    u0, v0 = _large_strain_case()
    s = lbm.Solver(1024, 1024, 1.0, prec, "pc")
    s.set_material(1.0, 0.1, 0.05, 0.8)
    s.set_fields(u0, v0)
    s.step(500)
    u, v, P, d, st = s.read()
    s.close()
    assert st == 0
    eu, ev, eP = (float(np.linalg.norm(x - r) / np.linalg.norm(r)) for x, r in ((u, ru), (v, rv), (P, rP)))
    print(prec, "large strain 500 steps: max strain %.3f rel-L2 u %.3e v %.3e P %.3e" % (d.max_strain, eu, ev, eP),
          flush=True)
    assert d.max_strain > 0.1
    assert eu < tol_u and eP < tol_P
