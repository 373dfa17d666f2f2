"""Reference values of the 4096 x 4096 large-strain workload after 500 steps.

The workload: a periodic 4096 x 4096 lattice, dX = rho0 = 1, neo-Hooke
lam = 0.1, mu = 0.05, tau/dt = 0.8, predictor-corrector source; u0 = 0 and
the seeded Gaussian-filtered velocity field (sigma = 32 cells, seed 2) scaled
to the calibrated peak velocity (large_strain_amplitude.json). This script
runs the FP64 oracle over the whole lattice for 500 steps (the workload's
length; peak strain about 0.2) and keeps u, v and P at 512 nodes drawn from
a seeded PCG64 stream (seed 500), plus every field's rel-L2 norm over the
whole lattice, in large_strain_4096_500.json next to this file.

Runs only the oracle: about 40 minutes on 8 cores, 6 GB of memory.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2208_13769_amd import inputs  # noqa: E402

N, SIGMA, SEED, STEPS, NODES, NODE_SEED = 4096, 32.0, 2, 500, 512, 500


def sample_nodes():
    rng = np.random.Generator(np.random.PCG64(NODE_SEED))
    return rng.integers(0, N, NODES).tolist(), rng.integers(0, N, NODES).tolist()


def main():
    with open(os.path.join(HERE, "large_strain_amplitude.json")) as fh:
        peak = float(json.load(fh)["peak_velocity"])
    t0 = time.time()
    u0, v0 = inputs.filtered_random_velocity(N, N, SIGMA, SEED, peak)
    s = O.Solver(O.Params(nx=N, ny=N, lam=0.1, mu=0.05, tau_over_dt=0.8), u0, v0)
    del u0, v0
    strain = []
    for k in range(STEPS // 25):
        s.step(25)
        e = s.diagnostics()["max_strain"]
        strain.append([s.step_index, e])
        print(f"step {s.step_index}: max strain {e:.4f} ({time.time() - t0:.0f} s)", flush=True)
    u, v, P = s.fields()
    xs, ys = sample_nodes()
    out = {"grid": N, "sigma": SIGMA, "seed": SEED, "peak_velocity": peak, "steps": STEPS,
           "lam": 0.1, "mu": 0.05, "tau_over_dt": 0.8, "scheme": "pc", "node_seed": NODE_SEED,
           "x": xs, "y": ys,
           "u": [[float(u[a, y, x]) for a in range(2)] for x, y in zip(xs, ys)],
           "v": [[float(v[a, y, x]) for a in range(2)] for x, y in zip(xs, ys)],
           "P": [[float(P[a, b, y, x]) for a in range(2) for b in range(2)] for x, y in zip(xs, ys)],
           "norm_u": float(np.linalg.norm(u)), "norm_v": float(np.linalg.norm(v)), "norm_P": float(np.linalg.norm(P)),
           "max_strain_history": strain, "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "large_strain_4096_500.json"), "w") as fh:
        json.dump(out, fh)
    print(json.dumps({k: out[k] for k in ("grid", "steps", "norm_u", "norm_P", "oracle_seconds")}), flush=True)


if __name__ == "__main__":
    main()
