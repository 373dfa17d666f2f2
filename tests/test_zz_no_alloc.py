"""The diagnostics entry point that allocates nothing
(lbm_read_diagnostics_noalloc: its scratch is a static device array) gives
the diagnostics of lbm_read_fields bit for bit, on two calls in a row, the
second on a smaller plate, and again on the first plate after that (the
shared array keeps the last call's contents)."""
import numpy as np
import pytest

from paper_2208_13769_amd import inputs

pytestmark = pytest.mark.gpu


def _plate(nx, ny, precision, seed, steps, walled):
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(nx, ny, 1.0, precision, "pc")
    s.set_material(1.0, 0.1, 0.05, 0.8)
    if walled:
        s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_DIRICHLET_J, (0.0, 0.0))
        s.set_boundary(lbm.LBM_EDGE_YMAX, lbm.LBM_BC_NEUMANN_T, (0.0, 0.001))
    u0, v0 = inputs.filtered_random_velocity(nx, ny, 3.0, seed, 0.02)
    s.set_fields(u0, v0)
    s.step(steps)
    return s


def _both(s):
    from paper_2208_13769_amd import lbm

    ref = lbm.lbm_diagnostics()
    st1 = lbm.lbm_read_fields(s.h, diag=ref)
    got = lbm.lbm_diagnostics()
    st2 = lbm.lbm_read_diagnostics_noalloc(s.h, got)
    assert st1 == st2 == lbm.LBM_OK
    return ref, got


def _same(a, b):
    assert list(a.momentum) == list(b.momentum)
    for f in ("mass_moment", "energy", "min_J", "max_strain", "unstable", "steps"):
        assert getattr(a, f) == getattr(b, f), f


def test_noalloc_diagnostics_equal_read_fields(gpu):
    big = _plate(700, 500, "fp64", 61, 30, True)      # 1368 blocks' worth of sites: the grid's cap
    small = _plate(90, 40, "fp32u64", 62, 20, False)  # 15 blocks
    r1, g1 = _both(big)
    r2, g2 = _both(small)
    r3, g3 = _both(big)
    for r, g in ((r1, g1), (r2, g2), (r3, g3)):
        _same(r, g)
        print(f"energy {g.energy:.6e} min J {g.min_J:.6f} max strain {g.max_strain:.4e} steps {g.steps}",
              flush=True)
    assert g1.energy != g2.energy and g1.steps == 30 and g2.steps == 20
    _same(g1, g3)
    big.close()
    small.close()
