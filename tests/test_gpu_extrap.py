"""The extrapolation variant (LBM_SCHEME_EXTRAP, end of Sec. 5) on the GPU
against the oracle: periodic plates and walled ones, FP64 and FP32."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_13769_amd import inputs
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

P_, D_, N_ = 0, 1, 2


def _pair(nx, ny, n, kinds=(P_, P_, P_, P_), precision="fp64", lam=0.025, mu=0.05, seed=90, body=(2e-5, 1e-5)):
    from paper_2208_13769_amd import lbm

    rng = np.random.Generator(np.random.PCG64(seed))
    u0 = 0.001 * rng.standard_normal((2, ny, nx))
    v0 = inputs.filtered_random_velocity(nx, ny, 2.0, seed, 0.01)[1]
    vals = {D_: (0.0001, -0.00005), N_: (0.0001, 0.0002), P_: (0.0, 0.0)}
    kw = {}
    for e, k in zip(("xmin", "xmax", "ymin", "ymax"), kinds):
        kw["bc_" + e] = k
        kw["val_" + e] = vals[k]
    p = O.Params(nx=nx, ny=ny, lam=lam, mu=mu, tau_over_dt=0.8, scheme=O.EXTRAP, body=body, **kw)
    s = O.Solver(p, u0, v0)
    s.step(n)
    uo, vo, Po = s.fields()
    g = lbm.Solver(nx, ny, 1.0, precision, "extrap")
    g.set_material(1.0, lam, mu, 0.8)
    if any(body):
        g.set_body_force(np.array(body))
    for e, k in enumerate(kinds):
        if k != P_:
            g.set_boundary(e, k, vals[k])
    g.set_fields(u0, v0)
    g.step(n)
    ug, vg, Pg, d, st = g.read()
    g.close()
    assert st == 0
    return (ug, vg, Pg), (uo, vo, Po)


@pytest.mark.parametrize("kinds", [(P_, P_, P_, P_), (P_, P_, D_, N_), (N_, D_, N_, N_)])
def test_extrap_matches_oracle_fp64(gpu, kinds):
    (ug, vg, Pg), (uo, vo, Po) = _pair(40, 33, 120, kinds)
    e = [rel_l2(ug, uo), rel_l2(vg, vo), rel_l2(Pg, Po)]
    print(f"extrap {kinds}: rel-L2 u {e[0]:.3e} v {e[1]:.3e} P {e[2]:.3e}", flush=True)
    assert max(e) < 1e-12


@pytest.mark.parametrize("precision,body", [("fp32", (0.0, 0.0)), ("fp32u64", (2e-5, 1e-5))])
def test_extrap_matches_oracle_fp32(gpu, precision, body):
    """A body force drifts the whole plate by a few spacings; a float
    displacement then loses P to cancellation, which the double
    displacement of FP32_U64 avoids."""
    (ug, vg, Pg), (uo, vo, Po) = _pair(64, 48, 200, precision=precision, body=body)
    e = [rel_l2(ug, uo), rel_l2(Pg, Po)]
    print(f"extrap {precision}: rel-L2 u {e[0]:.3e} P {e[1]:.3e}", flush=True)
    assert max(e) < 1e-5


def test_extrap_first_step_uses_j0(gpu):
    """One step from a state with j0 != 0: j(t - dt) is j(0)."""
    (ug, vg, Pg), (uo, vo, Po) = _pair(30, 30, 1)
    assert rel_l2(ug, uo) < 1e-13 and rel_l2(vg, vo) < 1e-13


def test_extrap_needs_the_walled_workspace(gpu):
    import ctypes
    import torch
    from paper_2208_13769_amd import lbm

    nb = lbm.lbm_workspace_bytes(32, 32, lbm.PRECISIONS["fp64"])
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(32, 32, 1.0, lbm.PRECISIONS["fp64"], lbm.LBM_SCHEME_EXTRAP, ctypes.c_void_p(ws.data_ptr()), nb,
                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert e.value.status == lbm.LBM_ERR_NOMEM
