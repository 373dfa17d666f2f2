"""Shared helpers of the test suite: run a case on the oracle and on the GPU
path with the same seeded inputs and compare them."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

BC_NAMES = {"periodic": 0, "dirichlet": 1, "neumann": 2}


def rel_l2(x, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))


def max_rel(x, ref):
    """Largest element-wise error over the largest |reference| value: a
    pointwise check beside rel-L2, which an error confined to one row, column
    or tile seam can pass."""
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / den) if den > 0 else float(np.abs(x).max())


# Pointwise bound as a multiple of a case's rel-L2 bound: smooth errors sit
# within a small factor of their L2 norm, while an error confined to a row
# of an N-row plate is about sqrt(N) times its share of the norm.
MAX_NORM_FACTOR = 10.0


def oracle_run(nx, ny, u0, v0, nsteps, *, dx=1.0, rho0=1.0, lam=0.1, mu=0.05, tau=0.8, scheme="pc",
               body=(0.0, 0.0), bc_lo=("periodic", (0.0, 0.0)), bc_hi=("periodic", (0.0, 0.0))):
    p = O.Params(nx=nx, ny=ny, dx=dx, rho0=rho0, lam=lam, mu=mu, tau_over_dt=tau,
                 scheme=O.PC if scheme == "pc" else O.EXPLICIT, body=tuple(body),
                 bc_ymin=BC_NAMES[bc_lo[0]], bc_ymax=BC_NAMES[bc_hi[0]],
                 val_ymin=tuple(bc_lo[1]), val_ymax=tuple(bc_hi[1]))
    s = O.Solver(p, u0, v0)
    s.step(nsteps)
    u, v, P = s.fields()
    return u, v, P, s.diagnostics()


def gpu_run(nx, ny, u0, v0, nsteps, *, precision="fp64", dx=1.0, rho0=1.0, lam=0.1, mu=0.05, tau=0.8,
            scheme="pc", body=(0.0, 0.0), bc_lo=("periodic", (0.0, 0.0)), bc_hi=("periodic", (0.0, 0.0)),
            general=False):
    """general: run the general step (2D tiles) in place of the fused kernel."""
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(nx, ny, dx, precision, scheme)
    if general:
        s.set_general_path(True)
    s.set_material(rho0, lam, mu, tau)
    if any(body):
        s.set_body_force(np.array(body, dtype=np.float64))
    if bc_lo[0] != "periodic":
        s.set_boundary(lbm.LBM_EDGE_YMIN, BC_NAMES[bc_lo[0]], bc_lo[1])
        s.set_boundary(lbm.LBM_EDGE_YMAX, BC_NAMES[bc_hi[0]], bc_hi[1])
    s.set_fields(u0, v0)
    s.step(nsteps)
    u, v, P, d, st = s.read()
    s.close()
    return u, v, P, d, st
