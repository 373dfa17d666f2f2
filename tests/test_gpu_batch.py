"""Batched plates (one persistent launch per step, graph-captured chunks)
against the same plates run alone, and against the oracle."""
import numpy as np
import pytest

from paper_2208_13769_amd import inputs
from tests.helpers import oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _plate_inputs(n, ny, seed, walled):
    if walled:
        u0, v0 = inputs.top_pulse(ny, 0.01, nx=n)
        v0 = v0 + inputs.filtered_random_velocity(n, ny, 2.0, seed, 0.002)[1]
    else:
        u0, v0 = inputs.filtered_random_velocity(n, ny, 3.0, seed, 0.03)
    return np.ascontiguousarray(u0), np.ascontiguousarray(v0)


def _single(spec, u0, v0, nsteps, precision, scheme="pc"):
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(spec.nx, spec.ny, spec.dx, precision, scheme)
    s.set_material(spec.rho0, spec.lam, spec.mu, spec.tau_over_dt)
    if spec.bc_ymin != lbm.LBM_BC_PERIODIC:
        s.set_boundary(lbm.LBM_EDGE_YMIN, spec.bc_ymin, spec.val_ymin)
        s.set_boundary(lbm.LBM_EDGE_YMAX, spec.bc_ymax, spec.val_ymax)
    s.set_fields(u0, v0)
    s.step(nsteps)
    out = s.read()
    s.close()
    return out


def _specs(walled):
    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.batch import PlateSpec

    sizes = [(40, 33), (64, 64), (100, 71), (260, 90), (300, 150), (517, 40)]
    specs = []
    for k, (nx, ny) in enumerate(sizes):
        sp = PlateSpec(nx=nx, ny=ny, lam=0.05 + 0.02 * k, mu=0.03 + 0.01 * k, tau_over_dt=0.7 + 0.05 * k)
        if walled:
            sp.bc_ymin, sp.bc_ymax = lbm.LBM_BC_DIRICHLET_J, lbm.LBM_BC_NEUMANN_T
            sp.val_ymin = (0.0, 0.0)
            sp.val_ymax = (0.0, 0.001 * (k % 2))
        specs.append(sp)
    return specs


@pytest.mark.parametrize("precision,walled,spl", [("fp16", False, 1), ("fp32", False, 2), ("fp64", True, 2),
                                                  ("fp16", True, 1), ("fp32", False, 1), ("fp32u64", False, 2),
                                                  ("fp32u64", True, 1), ("bf16", True, 1), ("bf16", False, 1)])
def test_batch_equals_plates_alone(gpu, precision, walled, spl):
    """Every plate of a mixed batch equals the same plate run alone, bitwise,
    after each of several graph-replayed chunks (eager reads in between);
    plates with fewer steps stop at their own count. Chunks of odd length and
    odd step counts exercise the single last step of the two-step kernel."""
    from paper_2208_13769_amd.batch import Batch

    specs = _specs(walled)
    targets = [60, 60, 35, 60, 51, 60]
    b = Batch(max_plates=8, arena_bytes=256 << 20, precision=precision, walled=walled)
    b.set_steps_per_launch(spl)
    assert b.steps_per_launch() == spl
    slots, ins = [], []
    for k, sp in enumerate(specs):
        u0, v0 = _plate_inputs(sp.nx, sp.ny, 30 + k, walled)
        ins.append((u0, v0))
        slots.append(b.add(sp, u0, v0, targets[k]))
    assert None not in slots
    done = 0
    for chunk in (20, 13, 27):
        b.step(chunk)
        done += chunk
        for k, sp in enumerate(specs):
            n = min(done, targets[k])
            ub, vb, Pb, db, st = b.read(slots[k])
            us, vs, Ps, ds, st2 = _single(sp, *ins[k], n, precision)
            assert st == 0 and st2 == 0 and db.steps == n
            assert np.array_equal(ub, us) and np.array_equal(vb, vs), (k, n)
    b.close()


def test_batch_fp64_matches_oracle(gpu):
    from paper_2208_13769_amd.batch import Batch

    specs = _specs(True)[:3]
    b = Batch(max_plates=4, arena_bytes=64 << 20, precision="fp64", walled=True)
    for k, sp in enumerate(specs):
        u0, v0 = _plate_inputs(sp.nx, sp.ny, 40 + k, True)
        slot = b.add(sp, u0, v0, 40)
        b.step(40)
        ub, vb, Pb, db, st = b.read(slot)
        uo, vo, Po, do = oracle_run(sp.nx, sp.ny, u0, v0, 40, lam=sp.lam, mu=sp.mu, tau=sp.tau_over_dt,
                                    bc_lo=("dirichlet", sp.val_ymin), bc_hi=("neumann", sp.val_ymax))
        assert rel_l2(ub, uo) < 1e-12 and rel_l2(Pb, Po) < 1e-12
        b.retire(slot)
    b.close()


def test_batch_admission_and_reuse(gpu):
    """Admission by arena footprint: a plate that does not fit is refused;
    retiring frees the space for the next one, which then runs correctly."""
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    sp_big = PlateSpec(nx=256, ny=256)
    b0 = Batch(max_plates=4, arena_bytes=1, precision="fp32")
    need = b0.plate_bytes(256, 256)
    b0.close()
    b = Batch(max_plates=4, arena_bytes=need + need // 2, precision="fp32")
    u0, v0 = _plate_inputs(256, 256, 50, False)
    s1 = b.add(sp_big, u0, v0, 10)
    assert s1 is not None
    assert b.add(sp_big, u0, v0, 10) is None  # no room for a second one
    b.step(10)
    b.retire(s1)
    sp2 = PlateSpec(nx=200, ny=180, lam=0.08, mu=0.04)
    u2, v2 = _plate_inputs(200, 180, 51, False)
    s2 = b.add(sp2, u2, v2, 25)
    assert s2 is not None
    b.step(25)
    ub, vb, *_ = b.read(s2)
    us, vs, *_ = _single(sp2, u2, v2, 25, "fp32")
    assert np.array_equal(ub, us) and np.array_equal(vb, vs)
    n, free, big = b.info()
    assert n == 1 and free > 0
    b.close()


def test_batch_unstable_plate_is_isolated(gpu):
    """A plate that blows up (lam/mu = 10) raises its own flag; the other
    plate's result is unchanged."""
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    good = PlateSpec(nx=96, ny=64)
    bad = PlateSpec(nx=64, ny=64, lam=0.5, mu=0.05)
    ug, vg = _plate_inputs(96, 64, 60, False)
    ub_, vb_ = inputs.random_field(64, 64, 61, 0.0), inputs.random_field(64, 64, 62, 1e-6)
    b = Batch(max_plates=2, arena_bytes=64 << 20, precision="fp32")
    sg = b.add(good, ug, vg, 300)
    sb = b.add(bad, ub_, vb_, 300)
    b.step(300)
    assert b.query(sb)[2] is True
    assert b.query(sg)[2] is False
    u1, v1, *_ = b.read(sg)
    u2, v2, *_ = _single(good, ug, vg, 300, "fp32")
    assert np.array_equal(u1, u2) and np.array_equal(v1, v2)
    b.close()


def test_packed_tile_table_with_many_tiles_per_block(gpu):
    """A batch with several tiles per block of the persistent grid (the
    packed table then has empty entries and blocks with different tile
    counts): sampled plates still equal the same plates run alone, bitwise."""
    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    rng = np.random.default_rng(11)
    sizes = [int(s) for s in rng.integers(300, 700, size=48)]
    specs = [PlateSpec(nx=n, ny=n + 7 * (k % 5), lam=0.1, mu=0.05, tau_over_dt=0.8,
                       bc_ymin=lbm.LBM_BC_DIRICHLET_J, bc_ymax=lbm.LBM_BC_NEUMANN_T)
             for k, n in enumerate(sizes)]
    arena = sum(Batch.plate_bytes_for(sp.nx, sp.ny, "fp16") for sp in specs) + (64 << 20)
    b = Batch(max_plates=len(specs), arena_bytes=arena, precision="fp16", walled=True)
    ins = [_plate_inputs(sp.nx, sp.ny, 60 + k, True) for k, sp in enumerate(specs)]
    steps = [5 if k % 3 else 4 for k in range(len(specs))]
    slots = [b.add(sp, u0, v0, steps[k]) for k, (sp, (u0, v0)) in enumerate(zip(specs, ins))]
    assert None not in slots
    b.step(5)
    for k in (0, 7, 19, 30, 47):
        ub, vb, Pb, db, st = b.read(slots[k])
        us, vs, Ps, ds, st2 = _single(specs[k], *ins[k], steps[k], "fp16")
        assert st == 0 and st2 == 0 and db.steps == steps[k]
        assert np.array_equal(ub, us) and np.array_equal(vb, vs) and np.array_equal(Pb, Ps), k
    b.close()


def test_batch_16bit_storage_runs_one_step_per_launch(gpu):
    """16-bit storage has no two-step batch kernel: the batch defaults to one
    step per launch and refuses two."""
    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.batch import Batch

    for prec in ("fp16", "bf16"):
        b = Batch(max_plates=2, arena_bytes=16 << 20, precision=prec)
        assert b.steps_per_launch() == 1
        with pytest.raises(lbm.LbmError) as ei:
            b.set_steps_per_launch(2)
        assert ei.value.status == lbm.LBM_ERR_UNSUPPORTED
        b.close()
