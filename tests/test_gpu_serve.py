"""Continuous-batching server: each result is the same alone and in the mix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone(gpu):
    from paper_2208_13769_amd import serve

    reqs = serve.make_requests(8, seed=11, n_median=64, sigma_ln=0.6, n_min=32, n_max=200,
                               steps_min=50, steps_max=400, peak=1e-4)
    serve.set_arrivals(reqs, rate=200.0, seed=11)
    srv = serve.BatchServer(arena_bytes=256 << 20, precision="fp16", chunk=64, max_plates=8)
    keep = {r.rid for r in reqs}
    summ, finish, got = srv.run(reqs, keep=keep)
    srv.close()
    assert summ["max_resident"] >= 2  # requests really overlapped on the GPU
    alone16 = serve.SerialServer("fp16")
    alone32 = serve.SerialServer("fp32")
    for r in reqs:
        u, v, P, d, st = got[r.rid]
        ua, va, Pa, da, sta = alone16.serve_one(r)
        assert st == 0 and sta == 0 and d.steps == r.steps
        assert np.array_equal(u, ua) and np.array_equal(v, va) and np.array_equal(P, Pa)
        # and the FP16-storage answer is close to the FP32 one
        u32, *_ = alone32.serve_one(r)
        assert np.linalg.norm(u - u32) <= 2e-2 * np.linalg.norm(u32)
