"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the
same seeded inputs. Tolerances on the relative L2 error of u and P:
1e-12 for FP64, 1e-5 for FP32 (the accuracy bars of the method's contract);
16-bit population storage is checked against bounds stated per case."""
import numpy as np
import pytest

from paper_2208_13769_amd import inputs
from tests.helpers import MAX_NORM_FACTOR, gpu_run, max_rel, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

MAT = dict(lam=0.1, mu=0.05, tau=0.8)


def _compare(case, nsteps, tol_u, tol_P, tol_v=None, precision="fp64", general=False, **kw):
    u0, v0, nx, ny = case
    uo, vo, Po, do = oracle_run(nx, ny, u0, v0, nsteps, **kw)
    ug, vg, Pg, dg, st = gpu_run(nx, ny, u0, v0, nsteps, precision=precision, general=general, **kw)
    assert st == 0
    eu, eP, ev = rel_l2(ug, uo), rel_l2(Pg, Po), rel_l2(vg, vo)
    mu_, mP = max_rel(ug, uo), max_rel(Pg, Po)
    print(f"rel-L2 u {eu:.3e} P {eP:.3e} v {ev:.3e}; max-norm u {mu_:.3e} P {mP:.3e}", flush=True)
    assert eu <= tol_u and eP <= tol_P
    assert mu_ <= MAX_NORM_FACTOR * tol_u and mP <= MAX_NORM_FACTOR * tol_P
    if tol_v is not None:
        assert ev <= tol_v
    return (uo, vo, Po, do), (ug, vg, Pg, dg)


def shear_wave_64_case():
    u0, v0 = inputs.shear_wave(64, 64, 1e-4, 64)
    return u0, v0, 64, 64


def random_case(nx, ny, seed, peak, sigma=3.0):
    u0, v0 = inputs.filtered_random_velocity(nx, ny, sigma, seed, peak)
    u0 = inputs.random_field(nx, ny, seed + 1, 0.02)  # small start displacement as well
    return u0, v0, nx, ny


def test_shear_wave_64_fp64(gpu):
    """64 x 64 periodic shear wave, FP64, 1000 steps: u, v, P and momentum."""
    o, g = _compare(shear_wave_64_case(), 1000, 1e-12, 1e-12, 1e-12)
    assert np.allclose(g[3].momentum, o[3]["momentum"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("scheme", ["pc", "explicit"])
def test_ragged_nonlinear_fp64(gpu, scheme):
    """517 x 77: three column strips (the last ragged), several row segments,
    a large-strain random field; 60 steps."""
    _compare(random_case(517, 77, 7, 0.05), 60, 1e-12, 1e-12, 1e-12, scheme=scheme, lam=0.1, mu=0.05)


@pytest.mark.parametrize("precision", ["fp32", "fp32u64"])
def test_ragged_nonlinear_fp32(gpu, precision):
    _compare(random_case(517, 77, 8, 0.05), 60, 1e-5, 1e-5, precision=precision, lam=0.1, mu=0.05)


@pytest.mark.parametrize("scheme", ["pc", "explicit"])
def test_general_step_on_periodic_and_y_walled_plates(gpu, scheme):
    """The general step (2D tiles), which the autotuner picks for small
    plates, in the plain workspace: the 64 x 64 shear wave for 1000 steps
    (lam = mu for the explicit scheme, which grows for lam > mu) and a
    100 x 60 field with y walls (both small enough for two-row tiles), and
    the ragged 517 x 77 field with y walls (default tiles), against the
    oracle."""
    mat = dict(lam=0.05, mu=0.05) if scheme == "explicit" else {}
    o, g = _compare(shear_wave_64_case(), 1000, 1e-12, 1e-12, 1e-12, scheme=scheme, general=True, **mat)
    assert np.allclose(g[3].momentum, o[3]["momentum"], rtol=0, atol=1e-14)
    kw = dict(lam=0.1, mu=0.05, bc_lo=("dirichlet", (0.0, 0.0)), bc_hi=("neumann", (0.0, 2e-4)))
    _compare(random_case(100, 60, 11, 0.05), 60, 1e-12, 1e-12, 1e-12, scheme=scheme, general=True, **kw)
    _compare(random_case(517, 77, 7, 0.05), 60, 1e-12, 1e-12, 1e-12, scheme=scheme, general=True, **kw)
    _compare(random_case(517, 77, 8, 0.05), 60, 1e-5, 1e-5, precision="fp32u64", scheme=scheme, general=True,
             **kw)
    if scheme == "pc":  # 16-bit storage, two-row tiles
        _compare(random_case(96, 64, 13, 0.05), 60, 1e-3, 1e-3, precision="fp16", scheme=scheme, general=True,
                 **kw)


def test_small_block_widths(gpu):
    """Widths that select the 64- and 128-thread blocks."""
    _compare(random_case(40, 33, 9, 0.03), 40, 1e-12, 1e-12)
    _compare(random_case(100, 35, 10, 0.03), 40, 1e-12, 1e-12)


def test_body_force_fp64(gpu):
    _compare(random_case(130, 40, 11, 0.02), 30, 1e-12, 1e-12, body=(1e-3, -2e-3))


def test_walls_clamped_free_fp64(gpu):
    """Clamped bottom (bounce-back, j* = 0) and traction-free top (anti-bounce-back)."""
    n = 96
    u0, v0 = inputs.top_pulse(n, 0.01)
    v0 = v0 + inputs.filtered_random_velocity(n, n, 2.0, 12, 0.002)[1]
    _compare((u0, v0, n, n), 200, 1e-12, 1e-12, 1e-12,
             bc_lo=("dirichlet", (0.0, 0.0)), bc_hi=("neumann", (0.0, 0.0)))


@pytest.mark.parametrize("scheme", ["pc", "explicit"])
def test_walls_loaded_fp64(gpu, scheme):
    """Moving momentum wall below and a traction on the wall above; ragged strips."""
    nx, ny = 300, 53
    u0, v0, _, _ = random_case(nx, ny, 13, 0.01)
    _compare((u0, v0, nx, ny), 80, 1e-12, 1e-12, 1e-12, scheme=scheme,
             bc_lo=("dirichlet", (0.002, -0.001)), bc_hi=("neumann", (0.001, -0.003)))
    _compare((u0, v0, nx, ny), 80, 1e-12, 1e-12, 1e-12, scheme=scheme,
             bc_lo=("neumann", (0.0, 0.002)), bc_hi=("dirichlet", (-0.001, 0.0)))


@pytest.mark.parametrize("precision", ["fp32", "fp32u64"])
def test_walls_fp32(gpu, precision):
    n = 70
    u0, v0 = inputs.top_pulse(n, 0.01)
    _compare((u0, v0, n, n), 150, 1e-5, 1e-5, precision=precision,
             bc_lo=("dirichlet", (0.0, 0.0)), bc_hi=("neumann", (0.0, 0.0)))


def test_diagnostics_match_oracle(gpu):
    o, g = _compare(random_case(200, 60, 14, 0.05), 40, 1e-12, 1e-12)
    do, dg = o[3], g[3]
    scale = np.abs(o[1]).sum()  # sum |v| bounds the momentum sums' rounding
    assert np.allclose(dg.momentum, do["momentum"], rtol=0, atol=1e-13 * scale)
    assert abs(dg.energy - do["energy"]) <= 1e-11 * abs(do["energy"])
    assert abs(dg.min_J - do["min_J"]) <= 1e-12
    assert abs(dg.max_strain - do["max_strain"]) <= 1e-12 * do["max_strain"]
    assert abs(dg.mass_moment - do["mass_moment"]) <= 1e-12 * np.abs(o[0]).sum()
    assert not dg.unstable and dg.steps == 40


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32u64", "fp16", "bf16"])
def test_tiling_does_not_change_results(gpu, precision):
    """Bitwise identical results for different blocks and row segmentations
    (catches halo and barrier mistakes at tile seams)."""
    from paper_2208_13769_amd import lbm

    nx, ny = 260, 90
    u0, v0, _, _ = random_case(nx, ny, 15, 0.05)
    outs = []
    for block, segs in [(256, 1), (256, 5), (512, 2), (128, 3), (64, 9), (64, 90)]:
        s = lbm.Solver(nx, ny, 1.0, precision, "pc")
        s.set_material(1.0, 0.1, 0.05, 0.8)
        s.set_tiling(block, segs)
        s.set_fields(u0, v0)
        s.step(30)
        u, v, P, d, st = s.read()
        s.close()
        outs.append((u, v))
    for u, v in outs[1:]:
        assert np.array_equal(u, outs[0][0]) and np.array_equal(v, outs[0][1])


def test_deterministic(gpu):
    nx, ny = 300, 64
    u0, v0, _, _ = random_case(nx, ny, 16, 0.05)
    a = gpu_run(nx, ny, u0, v0, 50, precision="fp32")
    b = gpu_run(nx, ny, u0, v0, 50, precision="fp32")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_unstable_flag(gpu):
    """lam/mu = 10 lies beyond the predictor-corrector's stability range:
    the run blows up and the handle reports LBM_ERR_UNSTABLE."""
    from paper_2208_13769_amd import lbm

    nx = ny = 32
    u0, v0, _, _ = random_case(nx, ny, 17, 1e-6)
    *_, d, st = gpu_run(nx, ny, u0, v0, 300, lam=0.5, mu=0.05)
    assert st == lbm.LBM_ERR_UNSTABLE and d.unstable


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_16bit_storage_short_run(gpu, precision):
    """16-bit population storage (deviations from the reference equilibrium)
    against the FP64 oracle within the 1e-3 bound: 200 steps of the 64 x 64
    shear wave."""
    _compare(shear_wave_64_case(), 200, 1e-3, 1e-3, precision=precision)


@pytest.mark.parametrize("scheme", ["pc", "explicit"])
@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_16bit_storage_with_walls(gpu, precision, scheme):
    """Deviation storage next to y walls (its reference takes the ghost rows
    of the walls, with a moving momentum wall) and on a ragged plate: within
    1e-3 of the oracle after 120 steps. lambda = mu: the explicit source
    grows for lambda > mu."""
    nx, ny = 150, 41
    u0, v0 = inputs.top_pulse(ny, 0.01, nx=nx)
    v0 = v0 + inputs.filtered_random_velocity(nx, ny, 3.0, 24, 0.003)[1]
    _compare((u0, v0, nx, ny), 120, 1e-3, 1e-3, precision=precision, scheme=scheme, lam=0.05, mu=0.05,
             bc_lo=("dirichlet", (0.002, 0.0)), bc_hi=("neumann", (0.0, 0.0005)))


def test_16bit_storage_runs_one_step_per_launch(gpu):
    """16-bit storage has no two-step kernel: asking for one is refused."""
    from paper_2208_13769_amd import lbm

    for prec in ("fp16", "bf16"):
        s = lbm.Solver(300, 90, 1.0, prec, "pc")
        assert s.resident_blocks(256, 2) == 0 and s.resident_blocks(256, 1) > 0
        with pytest.raises(lbm.LbmError) as ei:
            s.set_steps_per_launch(2)
        assert ei.value.status == lbm.LBM_ERR_UNSUPPORTED
        assert s.steps_per_launch() == 1
        s.close()


@pytest.mark.parametrize("precision,walled", [("fp32", False), ("fp32", True),
                                              ("fp64", False), ("fp32u64", False), ("fp32u64", True)])
def test_two_steps_per_launch_bitwise(gpu, precision, walled):
    """Two fused steps per launch give the single-step results bitwise, for an
    odd step count (the remainder runs as one step) and several tilings."""
    from paper_2208_13769_amd import lbm

    nx, ny = 300, 90
    if walled:
        u0, v0 = inputs.top_pulse(ny, 0.01, nx=nx)
        v0 = v0 + inputs.filtered_random_velocity(nx, ny, 2.0, 22, 0.002)[1]
    else:
        u0, v0, _, _ = random_case(nx, ny, 21, 0.05)
    shapes = [(1, 256, 5), (2, 256, 5), (2, 128, 3), (2, 64, 7), (2, 256, 1), (2, 128, 90), (1, 64, 45)]
    # 512-thread two-step blocks fit the LDS with FP32, and with a double
    # displacement only on plates periodic in y
    if precision == "fp32" or (precision != "fp64" and not walled):
        shapes.append((2, 512, 2))
    outs = []
    for spl, block, segs in shapes:
        s = lbm.Solver(nx, ny, 1.0, precision, "pc")
        s.set_material(1.0, 0.1, 0.05, 0.8)
        if walled:
            s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_DIRICHLET_J, (0.0, 0.0))
            s.set_boundary(lbm.LBM_EDGE_YMAX, lbm.LBM_BC_NEUMANN_T, (0.0, 0.001))
        s.set_steps_per_launch(spl)
        s.set_tiling(block, segs)
        assert s.tiling() == (block, segs)
        s.set_fields(u0, v0)
        s.step(31)
        u, v, P, d, st = s.read()
        s.close()
        assert st == 0 and d.steps == 31
        outs.append((u, v, P))
    for u, v, P in outs[1:]:
        assert np.array_equal(u, outs[0][0]) and np.array_equal(v, outs[0][1]) and np.array_equal(P, outs[0][2])


def test_resident_blocks_and_default_tiling(gpu):
    """The occupancy query gives a whole number of blocks per compute unit for
    every launchable shape and 0 for the shapes that cannot be launched; the
    default tiling fills at most one wave of resident blocks."""
    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.autotune import strips

    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    s = lbm.Solver(1000, 700, 1.0, "fp32", "pc")
    for block in (64, 128, 256, 512):
        for spl in (1, 2):
            r = s.resident_blocks(block, spl)
            assert r > 0 and r % cus == 0, (block, spl, r)
    assert s.resident_blocks(96, 1) == 0
    block, segs = s.tiling()
    assert strips(1000, block, "fp32", "pc", 1) * segs <= s.resident_blocks(block, 1)
    s.close()
    e = lbm.Solver(300, 90, 1.0, "fp32", "explicit")
    assert e.resident_blocks(128, 1) > 0 and e.resident_blocks(128, 2) == 0
    e.close()
    # a small plate is latency-bound: the default plan marches one-row
    # segments; a large one keeps segments of at least 16 rows
    small = lbm.Solver(64, 64, 1.0, "fp64", "pc")
    assert small.tiling() == (128, 64)
    small.close()
    large = lbm.Solver(2048, 2048, 1.0, "fp32", "pc")
    block, segs = large.tiling()
    assert 2048 // segs >= 16
    large.close()


def test_two_step_block_must_fit_the_lds(gpu):
    """A 512-thread two-step block holds two pipelines in LDS: it does not fit
    with FP64 values, nor with a double displacement once the y edges are
    walls. The tiling call refuses it there, and a wall set later lowers a
    512-thread tiling to 256 threads."""
    from paper_2208_13769_amd import lbm

    d = lbm.Solver(300, 90, 1.0, "fp64", "pc")
    d.set_steps_per_launch(2)
    assert d.resident_blocks(512, 2) == 0
    with pytest.raises(lbm.LbmError) as ei:
        d.set_tiling(512, 2)
    assert ei.value.status == lbm.LBM_ERR_UNSUPPORTED
    d.close()

    s = lbm.Solver(300, 90, 1.0, "fp32u64", "pc")
    s.set_steps_per_launch(2)
    assert s.resident_blocks(512, 2) > 0
    s.set_tiling(512, 3)
    assert s.tiling() == (512, 3)
    s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_DIRICHLET_J, (0.0, 0.0))
    assert s.resident_blocks(512, 2) == 0
    assert s.tiling() == (256, 3)
    u0, v0, _, _ = random_case(300, 90, 23, 0.01)
    s.set_material(1.0, 0.1, 0.05, 0.8)
    s.set_fields(u0, v0)
    s.step(4)
    *_, dg, st = s.read()
    assert st == 0 and dg.steps == 4
    # the single-step kernel keeps 512 threads
    s.set_steps_per_launch(1)
    s.set_tiling(512, 3)
    assert s.tiling() == (512, 3)
    s.close()
