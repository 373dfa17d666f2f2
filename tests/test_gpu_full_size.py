"""Parity at full size: the 4096 x 4096 large-strain plate of the benchmark,
in the launch configuration the benchmark times (FP32 arithmetic with an
FP64 displacement, 256-thread blocks, 26 row segments, two steps per
launch), and in FP64, against the oracle on sampled regions.

A value after K steps depends only on the start fields within 5 K + 1
nodes (a predictor-corrector step reaches at most five nodes: the source of
u^p is a difference of differences of u^p, itself a step of u; the read-out
of P one more). The oracle therefore computes a sampled region exactly from
a periodic patch of the start fields around it, with that margin (on a
256 x 256 plate the patch reproduces the full run bitwise); the GPU result
at the region comes from node samples of the full plate."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_13769_amd import inputs
from tests.helpers import MAX_NORM_FACTOR, max_rel, rel_l2

pytestmark = pytest.mark.gpu

N, K = 4096, 8
MARGIN = 5 * K + 1
REGION = 12
PATCH = 2 * MARGIN + REGION
CENTRES = [(700, 1300), (2048, 2048), (3500, 400), (4000, 3900)]  # (x0, y0) of each region


@pytest.fixture(scope="module")
def start_fields():
    path = os.path.join(os.path.dirname(__file__), "golden", "large_strain_amplitude.json")
    with open(path) as fh:
        amp = float(json.load(fh)["peak_velocity"])
    return inputs.filtered_random_velocity(N, N, 32.0, 2, amp)


def _patch(a, x0, y0):
    ys = np.arange(y0 - MARGIN, y0 + REGION + MARGIN) % N
    xs = np.arange(x0 - MARGIN, x0 + REGION + MARGIN) % N
    return np.ascontiguousarray(a[:, ys][:, :, xs])


# The 16-bit forms (deviation storage, one step per launch) run on the same
# large-strain start in a 256-thread, 28-segment launch, against the 1e-3
# bound.
@pytest.mark.parametrize("precision,tiling,tol", [("fp32u64", (256, 26, 2), 1e-5), ("fp64", None, 1e-12),
                                                  ("fp16", (256, 28, 1), 1e-3), ("bf16", (256, 28, 1), 1e-3)])
def test_full_size_sampled_regions(gpu, start_fields, precision, tiling, tol):
    from paper_2208_13769_amd import lbm

    u0, v0 = start_fields
    s = lbm.Solver(N, N, 1.0, precision, "pc")
    s.set_material(1.0, 0.1, 0.05, 0.8)
    if tiling:
        s.set_steps_per_launch(tiling[2])
        s.set_tiling(tiling[0], tiling[1])
    s.set_fields(u0, v0)
    s.step(K)
    gx, gy = np.meshgrid(np.arange(REGION), np.arange(REGION))
    worst = worst_max = 0.0
    for x0, y0 in CENTRES:
        smp = s.sample((gx + x0).ravel(), (gy + y0).ravel())  # [n][17]: u (2), v (2), P (4), ...
        p = O.Params(nx=PATCH, ny=PATCH, lam=0.1, mu=0.05, tau_over_dt=0.8)
        o = O.Solver(p, _patch(u0, x0, y0), _patch(v0, x0, y0))
        o.step(K)
        uo, vo, Po = o.fields()
        sl = (slice(MARGIN, MARGIN + REGION), slice(MARGIN, MARGIN + REGION))
        ref_u = np.stack([uo[a][sl].ravel() for a in range(2)], axis=1)
        ref_P = np.stack([Po[a, b][sl].ravel() for a in range(2) for b in range(2)], axis=1)
        eu, eP = rel_l2(smp[:, 0:2], ref_u), rel_l2(smp[:, 4:8], ref_P)
        mu_, mP = max_rel(smp[:, 0:2], ref_u), max_rel(smp[:, 4:8], ref_P)
        print(f"{precision} region at ({x0}, {y0}): rel-L2 u {eu:.3e} P {eP:.3e}; "
              f"max-norm u {mu_:.3e} P {mP:.3e}", flush=True)
        worst = max(worst, eu, eP)
        worst_max = max(worst_max, mu_, mP)
    s.close()
    assert worst < tol
    assert worst_max < MAX_NORM_FACTOR * tol


def test_plates_256_fp64_batch_against_oracle_on_sampled_plates(gpu):
    """The batched workload at full size, in the benchmark's launch
    configuration: all 256 seeded plates (side log-uniform in 64..1024,
    clamped bottom, traction-free top, top pulse 0.01) in one FP64 batch,
    2000 steps in graph-captured chunks of 200. Whole plates are sampled:
    the three smallest within the interior's stability range (lam/mu <= 6)
    and one of about 200 nodes against the oracle. FP64 rounding differences
    between the two grow about in proportion to the step count, so the bound
    is the 1e-12 of the 1000-step FP64 workload scaled to 2000 steps."""
    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.batch import Batch, PlateSpec
    from tests.helpers import oracle_run

    plates = inputs.plate_batch(256, seed=4)
    steps, chunk = 2000, 200
    specs = [PlateSpec(nx=pl.n, ny=pl.n, lam=pl.lam, mu=pl.mu, tau_over_dt=0.8,
                       bc_ymin=lbm.LBM_BC_DIRICHLET_J, bc_ymax=lbm.LBM_BC_NEUMANN_T) for pl in plates]
    fields = [inputs.top_pulse(pl.n, 0.01) for pl in plates]
    arena = sum(Batch.plate_bytes_for(sp.nx, sp.ny, "fp64") for sp in specs) + (64 << 20)
    b = Batch(max_plates=len(specs), arena_bytes=arena, precision="fp64", walled=True)
    slots = [b.add(sp, u0, v0, steps) for sp, (u0, v0) in zip(specs, fields)]
    assert None not in slots
    for _ in range(steps // chunk):
        b.step(chunk)
    stable = [i for i, pl in enumerate(plates) if pl.lam / pl.mu <= 6.0]
    picks = sorted(stable, key=lambda i: plates[i].n)[:3]
    picks.append(min(stable, key=lambda i: abs(plates[i].n - 200)))
    for i in picks:
        sp, (u0, v0) = specs[i], fields[i]
        ub, vb, Pb, db, st = b.read(slots[i])
        assert st == 0 and db.steps == steps
        uo, vo, Po, _ = oracle_run(sp.nx, sp.ny, u0, v0, steps, lam=sp.lam, mu=sp.mu, tau=0.8,
                                   bc_lo=("dirichlet", (0.0, 0.0)), bc_hi=("neumann", (0.0, 0.0)))
        eu, ep = rel_l2(ub, uo), rel_l2(Pb, Po)
        print(f"plate {i}: n {sp.nx}, lam/mu {sp.lam / sp.mu:.2f}: rel-L2 u {eu:.2e} P {ep:.2e}", flush=True)
        assert eu < 2e-12 and ep < 2e-12, (i, eu, ep)
    b.close()


def _golden_500():
    path = os.path.join(os.path.dirname(__file__), "golden", "large_strain_4096_500.json")
    with open(path) as fh:
        return json.load(fh)


# The whole workload: the 4096 x 4096 large-strain plate for its 500 steps,
# against the FP64 oracle's values at 512 seeded nodes
# (golden/large_strain_4096_500.py, the oracle alone). FP32 with an FP64
# displacement runs in the benchmark's launch shape; plain FP32 misses 1e-5
# on P (it differences a float displacement of a few lattice units).
@pytest.mark.parametrize("precision,tiling,tol", [
    ("fp32u64", (256, 26, 2), 1e-5), ("fp64", None, 1e-11),
    pytest.param("fp32", (256, 26, 2), 1e-5, marks=pytest.mark.xfail(reason="plain FP32: P about 4e-5 after 500 "
                                                                            "steps", strict=False)),
    ("fp16", (256, 28, 1), 1e-3), ("bf16", (256, 28, 1), 1e-3)])
def test_full_size_500_steps_against_oracle(gpu, start_fields, precision, tiling, tol):
    from paper_2208_13769_amd import lbm

    g = _golden_500()
    u0, v0 = start_fields
    s = lbm.Solver(N, N, 1.0, precision, "pc")
    s.set_material(1.0, g["lam"], g["mu"], g["tau_over_dt"])
    if tiling:
        s.set_steps_per_launch(tiling[2])
        s.set_tiling(tiling[0], tiling[1])
    s.set_fields(u0, v0)
    s.step(g["steps"])
    smp = s.sample(np.array(g["x"]), np.array(g["y"]))
    *_, d, st = s.read(want_fields=False)
    s.close()
    assert st == 0 and d.steps == g["steps"]
    ref_u, ref_v, ref_P = np.array(g["u"]), np.array(g["v"]), np.array(g["P"])
    eu, ev, eP = rel_l2(smp[:, 0:2], ref_u), rel_l2(smp[:, 2:4], ref_v), rel_l2(smp[:, 4:8], ref_P)
    mu_, mP = max_rel(smp[:, 0:2], ref_u), max_rel(smp[:, 4:8], ref_P)
    print(f"{precision} 4096^2 after {g['steps']} steps, 512 nodes: rel-L2 u {eu:.3e} v {ev:.3e} P {eP:.3e}; "
          f"max-norm u {mu_:.3e} P {mP:.3e}; max strain {d.max_strain:.3f}", flush=True)
    assert d.max_strain > 0.15
    assert eu < tol and eP < tol
    assert mu_ < MAX_NORM_FACTOR * tol and mP < MAX_NORM_FACTOR * tol
