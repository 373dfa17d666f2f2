"""The autotuner on the GPU: it times every candidate launch shape, re-times
the fastest few, caches its choice, and the choice changes nothing but the
speed."""
import json

import numpy as np
import pytest

from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


def test_tuner_choice_is_a_candidate_and_changes_no_result(gpu, tmp_path, monkeypatch):
    from paper_2208_13769_amd import inputs, lbm
    from paper_2208_13769_amd.autotune import GENERAL, apply_tiling, best_tiling, candidates

    cache = tmp_path / "autotune.json"
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(cache))
    n, steps = 256, 24
    u0, v0 = inputs.filtered_random_velocity(n, n, 8.0, 3, 0.01)

    def run(tiling):
        s = lbm.Solver(n, n, 1.0, "fp64", "pc")
        s.set_material(1.0, 0.1, 0.05, 0.8)
        s.set_fields(u0, v0)
        if tiling is not None:
            apply_tiling(s, tiling)
        s.step(steps)
        u, v, P, d, st = s.read()
        s.close()
        assert st == 0
        return u, P

    s = lbm.Solver(n, n, 1.0, "fp64", "pc")
    s.set_material(1.0, 0.1, 0.05, 0.8)
    s.set_fields(u0, v0)
    cands = [tuple(c) for c in candidates(s, n, n, "fp64", "pc")]
    best = tuple(best_tiling(s, n, n, "fp64", "pc"))
    s.close()
    assert best in cands
    entry = next(iter(json.loads(cache.read_text()).values()))
    assert entry["tiling"] == list(best)
    table = entry["table"]
    assert sorted(tuple(r[:3]) for r in table) == sorted(cands)
    assert sum(1 for r in table if len(r) == 5) == min(3, len(cands))  # the re-timed finalists
    assert all(r[3] > 0 for r in table)
    print(f"tuned 256^2 fp64: {best}, {entry['ms_per_step'] * 1e3:.1f} us per step", flush=True)

    # a second call takes the cached choice
    s = lbm.Solver(n, n, 1.0, "fp64", "pc")
    assert tuple(best_tiling(s, n, n, "fp64", "pc")) == best
    s.close()

    u_def, P_def = run(None)
    u_best, P_best = run(best)
    if best == GENERAL:  # the general step: the same results up to rounding
        assert rel_l2(u_best, u_def) < 1e-12 and rel_l2(P_best, P_def) < 1e-12
    else:  # fused-kernel shapes: bitwise
        assert np.array_equal(u_best, u_def) and np.array_equal(P_best, P_def)
