"""Call-order and argument errors of a live handle (LBM_ERR_STATE,
LBM_ERR_ARG), and the degenerate calls that must be no-ops."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _solver(n=24):
    from paper_2208_13769_amd import lbm

    return lbm, lbm.Solver(n, n, 1.0, "fp64", "pc")


def _status(fn, *a):
    from paper_2208_13769_amd import lbm

    with pytest.raises(lbm.LbmError) as e:
        fn(*a)
    return e.value.status


def test_call_order(gpu):
    lbm, s = _solver()
    z = np.zeros((2, 24, 24))
    assert _status(s.step, 1) == lbm.LBM_ERR_STATE            # no fields yet
    assert _status(s.set_fields, z, z) == lbm.LBM_ERR_STATE    # no material yet
    s.set_material(1.0, 0.1, 0.05, 0.8)
    s.set_fields(z, z)
    assert _status(s.set_material, 1.0, 0.1, 0.05, 0.8) == lbm.LBM_ERR_STATE  # after the fields
    s.close()


@pytest.mark.parametrize("args", [(0.0, 0.1, 0.05, 0.8), (1.0, 0.1, 0.0, 0.8), (1.0, -0.05, 0.05, 0.8),
                                  (1.0, 0.1, 0.05, 0.5), (1.0, float("inf"), 0.05, 0.8)])
def test_material_rejected(gpu, args):
    lbm, s = _solver()
    assert _status(s.set_material, *args) == lbm.LBM_ERR_ARG
    s.close()


def test_boundary_rejected(gpu):
    lbm, s = _solver()
    assert _status(s.set_boundary, 7, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0)) == lbm.LBM_ERR_ARG
    assert _status(s.set_boundary, lbm.LBM_EDGE_YMIN, 9, (0.0, 0.0)) == lbm.LBM_ERR_ARG
    assert _status(s.set_boundary, lbm.LBM_EDGE_YMIN, lbm.LBM_BC_NEUMANN_T, (float("nan"), 0.0)) == lbm.LBM_ERR_ARG
    s.close()


def test_zero_and_negative_steps(gpu):
    lbm, s = _solver()
    rng = np.random.Generator(np.random.PCG64(5))
    u0, v0 = 0.01 * rng.standard_normal((2, 2, 24, 24))
    s.set_material(1.0, 0.1, 0.05, 0.8)
    s.set_fields(u0, v0)
    a = s.read()
    s.step(0)  # no-op
    b = s.read()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and b[3].steps == 0
    assert _status(s.step, -1) == lbm.LBM_ERR_ARG
    s.close()


def test_nonfinite_start_fields_rejected(gpu):
    lbm, s = _solver()
    s.set_material(1.0, 0.1, 0.05, 0.8)
    u0 = np.zeros((2, 24, 24))
    u0[0, 3, 4] = np.nan
    assert _status(s.set_fields, u0, np.zeros((2, 24, 24))) == lbm.LBM_ERR_ARG
    s.close()


def test_binding_rejects_wrong_shapes_before_the_library(gpu):
    """Host arrays of the wrong shape never reach the library (it reads
    exactly the sizes the plate implies); a mask is material where nonzero."""
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    lbm, s = _solver()
    s.set_material(1.0, 0.1, 0.05, 0.8)
    z = np.zeros((2, 24, 24))
    with pytest.raises(ValueError):
        s.set_fields(np.zeros((2, 24, 23)), z)
    with pytest.raises(ValueError):
        s.set_fields(z, np.zeros((24, 24)))
    with pytest.raises(ValueError):
        s.set_body_force([0.0])
    with pytest.raises(ValueError):
        s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0, 0.0))
    s.set_fields(z, z)
    with pytest.raises(ValueError):
        s.sample([1, 2], [3])
    s.close()

    w = lbm.Solver(24, 24, 1.0, "fp64", "pc", walled=True)
    w.set_material(1.0, 0.1, 0.05, 0.8)
    for e in (lbm.LBM_EDGE_XMIN, lbm.LBM_EDGE_XMAX, lbm.LBM_EDGE_YMIN, lbm.LBM_EDGE_YMAX):
        w.set_boundary(e, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0))
    with pytest.raises(ValueError):
        w.set_mask(np.ones((24, 23)))
    m = np.full((24, 24), 0.5)  # fractional values are material, not truncated to holes
    m[8:16, 8:16] = 0.0
    w.set_mask(m)
    w.set_fields(z, z)
    w.step(2)
    u, v, P, d, st = w.read()
    assert st == 0 and np.all(u[:, 8:16, 8:16] == 0.0)
    w.close()

    b = Batch(max_plates=2, arena_bytes=16 << 20, precision="fp32")
    with pytest.raises(ValueError):
        b.add(PlateSpec(nx=32, ny=20), np.zeros((2, 32, 20)), np.zeros((2, 32, 20)), 4)
    b.close()
