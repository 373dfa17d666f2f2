"""Read-outs beyond u, v and P: Cauchy stress, Green-Lagrange strain and
strain-energy density fields, and node samples, against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_13769_amd import inputs
from tests.helpers import BC_NAMES, rel_l2

pytestmark = pytest.mark.gpu


def _oracle(nx, ny, u0, v0, n, bc=None):
    kw = {}
    if bc:
        kw = dict(bc_ymin=BC_NAMES["dirichlet"], bc_ymax=BC_NAMES["neumann"], val_ymin=(0.0, 0.0),
                  val_ymax=(0.0, 0.002))
    p = O.Params(nx=nx, ny=ny, lam=0.1, mu=0.05, tau_over_dt=0.8, **kw)
    s = O.Solver(p, u0, v0)
    s.step(n)
    u, v, P = s.fields()
    return (u, v, P) + s.derived()


def _gpu(nx, ny, u0, v0, n, precision="fp64", bc=None):
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(nx, ny, 1.0, precision, "pc")
    s.set_material(1.0, 0.1, 0.05, 0.8)
    if bc:
        s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_DIRICHLET_J, (0.0, 0.0))
        s.set_boundary(lbm.LBM_EDGE_YMAX, lbm.LBM_BC_NEUMANN_T, (0.0, 0.002))
    s.set_fields(u0, v0)
    s.step(n)
    return s


@pytest.mark.parametrize("walled", [False, True])
def test_derived_fields_match_oracle(gpu, walled):
    nx, ny, n = 203, 67, 45
    if walled:
        u0, v0 = inputs.top_pulse(ny, 0.01, nx=nx)
        v0 = v0 + inputs.filtered_random_velocity(nx, ny, 2.0, 71, 0.003)[1]
    else:
        u0, v0 = inputs.filtered_random_velocity(nx, ny, 3.0, 70, 0.05)
    uo, vo, Po, so, Eo, Wo = _oracle(nx, ny, u0, v0, n, walled)
    s = _gpu(nx, ny, u0, v0, n, bc=walled)
    sg, Eg, Wg = s.read_derived()
    s.close()
    es, eE, eW = rel_l2(sg, so), rel_l2(Eg, Eo), rel_l2(Wg, Wo)
    print(f"rel-L2 sigma {es:.3e} E {eE:.3e} W {eW:.3e}", flush=True)
    assert es < 1e-12 and eE < 1e-12 and eW < 1e-11
    # the Cauchy stress is symmetric
    assert np.array_equal(sg[0, 1], sg[1, 0])


def test_samples_equal_the_fields(gpu):
    nx, ny, n = 130, 90, 30
    u0, v0 = inputs.filtered_random_velocity(nx, ny, 3.0, 72, 0.05)
    s = _gpu(nx, ny, u0, v0, n, precision="fp32")
    u, v, P, d, st = s.read()
    sg, E, W = s.read_derived()
    rng = np.random.Generator(np.random.PCG64(5))
    xs = np.concatenate([[0, nx - 1, 0, nx - 1], rng.integers(0, nx, 60)])
    ys = np.concatenate([[0, 0, ny - 1, ny - 1], rng.integers(0, ny, 60)])
    out = s.sample(xs, ys)
    s.close()
    want = np.stack([u[0], u[1], v[0], v[1], P[0, 0], P[0, 1], P[1, 0], P[1, 1], sg[0, 0], sg[0, 1], sg[1, 0],
                     sg[1, 1], E[0, 0], E[0, 1], E[1, 0], E[1, 1], W])[:, ys, xs].T
    assert np.array_equal(out, want)


def test_sample_rejects_nodes_outside(gpu):
    from paper_2208_13769_amd import lbm

    s = _gpu(64, 40, *inputs.filtered_random_velocity(64, 40, 3.0, 1, 0.01), 2)
    with pytest.raises(lbm.LbmError):
        s.sample([64], [0])
    with pytest.raises(lbm.LbmError):
        s.sample([0], [-1])
    s.close()


def test_probe_time_series_matches_oracle(gpu):
    """Displacement and Cauchy stress at three nodes every 10 steps of a
    loaded walled strip (the kind of series Sec. 7 plots)."""
    nx, ny = 96, 48
    u0 = np.zeros((2, ny, nx))
    v0 = np.zeros((2, ny, nx))
    xs, ys = np.array([48, 10, 80]), np.array([47, 24, 1])
    s = _gpu(nx, ny, u0, v0, 0, bc=True)
    steps, vals = s.sample_series(xs, ys, 60, 10)
    s.close()
    assert list(steps) == [0, 10, 20, 30, 40, 50, 60]
    p = O.Params(nx=nx, ny=ny, lam=0.1, mu=0.05, tau_over_dt=0.8, bc_ymin=BC_NAMES["dirichlet"],
                 bc_ymax=BC_NAMES["neumann"], val_ymin=(0.0, 0.0), val_ymax=(0.0, 0.002))
    o = O.Solver(p, u0, v0)
    for k, n in enumerate(steps):
        if n:
            o.step(10)
        u, v, P = o.fields()
        sig, E, W = o.derived()
        want = np.stack([u[0], u[1], sig[0, 1], sig[1, 1]])[:, ys, xs].T
        got = vals[k][:, [0, 1, 9, 11]]
        scale = max(np.abs(want).max(), 1e-30)
        assert np.abs(got - want).max() <= 1e-12 * scale + 1e-300, (n, got, want)
    # the traction on the top edge pulls the top row up
    assert vals[-1][0, 1] > 0


def test_batch_readouts_equal_single_plate(gpu):
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    nx, ny = 150, 70
    u0, v0 = inputs.filtered_random_velocity(nx, ny, 3.0, 73, 0.05)
    b = Batch(max_plates=2, arena_bytes=64 << 20, precision="fp32")
    slot = b.add(PlateSpec(nx=nx, ny=ny), u0, v0, 25)
    b.step(25)
    sb, Eb, Wb = b.read_derived(slot)
    smp = b.sample(slot, [3, 140], [5, 66])
    b.close()
    s = _gpu(nx, ny, u0, v0, 25, precision="fp32")
    ss, Es, Ws = s.read_derived()
    smp_s = s.sample([3, 140], [5, 66])
    s.close()
    assert np.array_equal(sb, ss) and np.array_equal(Eb, Es) and np.array_equal(Wb, Ws)
    assert np.array_equal(smp, smp_s)
