"""Calibrate the velocity amplitude of the 4096 x 4096 large-strain workload.

The workload asks for a seeded Gaussian-filtered velocity field (sigma = 32
cells, seed 2) scaled so that the peak Green-Lagrange strain reaches about
0.2 within 200 steps. This script runs the FP64 oracle once at a small,
linear-regime peak velocity (1e-3), records the largest spectral norm of
E = (F^T F - I)/2 over all sites at every 10th step up to step 200, and
scales the amplitude linearly to a target strain of 0.2. The result is
written to large_strain_amplitude.json next to this file.

Runs only the oracle (about 10-15 minutes on 8 cores).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2208_13769_amd import inputs  # noqa: E402

N, SIGMA, SEED, PILOT, TARGET, STEPS = 4096, 32.0, 2, 1e-3, 0.2, 200


def main():
    t0 = time.time()
    u0, v0 = inputs.filtered_random_velocity(N, N, SIGMA, SEED, PILOT)
    s = O.Solver(O.Params(nx=N, ny=N, lam=0.1, mu=0.05, tau_over_dt=0.8), u0, v0)
    peak = 0.0
    history = []
    for k in range(STEPS // 10):
        s.step(10)
        e = s.diagnostics()["max_strain"]
        history.append([s.step_index, e])
        peak = max(peak, e)
        print(f"step {s.step_index}: max strain {e:.6e} ({time.time() - t0:.0f}s)", flush=True)
    amp = PILOT * TARGET / peak
    out = {"grid": N, "sigma": SIGMA, "seed": SEED, "pilot_peak_velocity": PILOT,
           "pilot_peak_strain": peak, "target_strain": TARGET, "peak_velocity": amp,
           "history": history}
    with open(os.path.join(HERE, "large_strain_amplitude.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "history"}))


if __name__ == "__main__":
    main()
