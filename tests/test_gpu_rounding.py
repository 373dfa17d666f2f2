"""Stochastic rounding of 16-bit population stores.

The random bits are a hash of (seed, state index, site, population), so a
run is reproducible for a seed and must not depend on the launch shape, the
number of steps fused per launch or batching. Rounding up or down in
proportion to the distance makes the stored populations unbiased; the
uniform-translation test measures that through the conserved momentum."""
import numpy as np
import pytest

from paper_2208_13769_amd import inputs
from tests.helpers import BC_NAMES

pytestmark = pytest.mark.gpu


def _run(nx, ny, u0, v0, nsteps, precision, rounding, seed=0, tiling=None, spl=1, walled=False, lam=0.1,
         mu=0.05):
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(nx, ny, 1.0, precision, "pc")
    s.set_material(1.0, lam, mu, 0.8)
    if walled:
        s.set_boundary(lbm.LBM_EDGE_YMIN, BC_NAMES["dirichlet"], (0.0, 0.0))
        s.set_boundary(lbm.LBM_EDGE_YMAX, BC_NAMES["neumann"], (0.0, 0.0005))
    s.set_steps_per_launch(spl)
    if tiling:
        s.set_tiling(*tiling)
    s.set_rounding(rounding, seed)
    s.set_fields(u0, v0)
    s.step(nsteps)
    u, v, P, d, st = s.read()
    s.close()
    assert st == 0 and d.steps == nsteps
    return u, v


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
@pytest.mark.parametrize("walled", [False, True])
def test_stochastic_rounding_reproducible_and_shape_independent(gpu, precision, walled):
    nx, ny, n = 300, 90, 31
    if walled:
        u0, v0 = inputs.top_pulse(ny, 0.01, nx=nx)
        v0 = v0 + inputs.filtered_random_velocity(nx, ny, 2.0, 23, 0.002)[1]
    else:
        u0, v0 = inputs.filtered_random_velocity(nx, ny, 3.0, 24, 0.03)
    base = _run(nx, ny, u0, v0, n, precision, "stochastic", 7, walled=walled)
    for kw in ({}, {"tiling": (64, 7)}, {"tiling": (256, 2)}, {"tiling": (512, 3)}, {"tiling": (128, 5)}):
        u, v = _run(nx, ny, u0, v0, n, precision, "stochastic", 7, walled=walled, **kw)
        assert np.array_equal(u, base[0]) and np.array_equal(v, base[1]), kw
    other = _run(nx, ny, u0, v0, n, precision, "stochastic", 8, walled=walled)
    nearest = _run(nx, ny, u0, v0, n, precision, "nearest", walled=walled)
    assert not np.array_equal(other[1], base[1])
    assert not np.array_equal(nearest[1], base[1])
    # all three are roundings of the same run
    scale = np.abs(nearest[1]).max()
    assert np.abs(base[1] - nearest[1]).max() < 0.05 * scale


def test_stochastic_rounding_in_batch_equals_alone(gpu):
    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    sizes = [(70, 40), (130, 96), (256, 64)]
    b = Batch(max_plates=4, arena_bytes=64 << 20, precision="fp16")
    slots, ins = [], []
    for k, (nx, ny) in enumerate(sizes):
        sp = PlateSpec(nx=nx, ny=ny, lam=0.08 + 0.01 * k, mu=0.05, rounding="stochastic", seed=100 + k)
        u0, v0 = inputs.filtered_random_velocity(nx, ny, 3.0, 60 + k, 0.03)
        ins.append((sp, u0, v0))
        slots.append(b.add(sp, u0, v0, 40))
    b.step(40)
    for slot, (sp, u0, v0) in zip(slots, ins):
        ub, vb, _, db, st = b.read(slot)
        us, vs = _run(sp.nx, sp.ny, u0, v0, 40, "fp16", "stochastic", sp.seed, lam=sp.lam, mu=sp.mu)
        assert st == 0 and np.array_equal(ub, us) and np.array_equal(vb, vs)
    b.close()


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_stochastic_rounding_unbiased(gpu, precision):
    """16-bit storage rounds the populations' deviation from the reference
    equilibrium. A plate at rest under a uniform body force stays uniform,
    and after one step its populations deviate from the reference by
    -(1/2) 3 w_i e_i . S (the reference takes the stored momentum, which
    carries half the source), the same at every site. The start state (all
    zero) is stored exactly, so step one gives the same v everywhere under
    either rounding; step two sees the deviations stored by step one through
    the BGK relaxation. Round to nearest stores the same value at every site:
    zero spread. Stochastic rounding stores independent unbiased roundings:
    a spread, and a site mean within a few standard errors of the FP64
    oracle (the float arithmetic's own error is far below that)."""
    from paper_2208_13769_amd import lbm
    from tests.helpers import oracle_run

    nx = ny = 256
    body = (3e-4, -2e-4)
    z0 = np.zeros((2, ny, nx))

    def run(rounding, n):
        s = lbm.Solver(nx, ny, 1.0, precision, "pc")
        s.set_material(1.0, 0.1, 0.05, 0.8)
        s.set_body_force(np.array(body))
        s.set_rounding(rounding, 3)
        s.set_fields(z0, z0)
        s.step(n)
        u, v, P, d, st = s.read()
        s.close()
        assert st == 0
        return v

    v1n, v1s = run("nearest", 1), run("stochastic", 1)
    assert np.all(v1n == v1n[:, :1, :1]) and np.array_equal(v1s, v1n)
    vn = run("nearest", 2)
    assert np.all(vn == vn[:, :1, :1])
    vs = run("stochastic", 2)
    _, vo, _, _ = oracle_run(8, 8, z0[:, :8, :8], z0[:, :8, :8], 2, body=body)
    for a in range(2):
        sd = vs[a].std()
        assert sd > 0
        z = (vs[a].mean() - vo[a, 0, 0]) / (sd / np.sqrt(nx * ny))
        print(f"{precision} v[{a}]: spread {sd:.3e}, site mean - oracle {vs[a].mean() - vo[a, 0, 0]:.3e} (z {z:.2f}); "
              f"nearest - oracle {vn[a, 0, 0] - vo[a, 0, 0]:.3e}", flush=True)
        assert abs(z) < 5.0


def test_stochastic_rounding_needs_16bit_storage(gpu):
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(64, 64, 1.0, "fp32", "pc")
    with pytest.raises(lbm.LbmError) as e:
        s.set_rounding("stochastic", 1)
    assert e.value.status == lbm.LBM_ERR_UNSUPPORTED
    s.set_rounding("nearest", 0)
    s.close()
