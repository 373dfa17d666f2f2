#!/usr/bin/env python3
"""Throughput of the per-time-step lattice update on one MI355X.

Default workload (the large-strain periodic plate): a 4096 x 4096 D2Q9 grid,
dX = rho0 = 1, neo-Hooke lam = 0.1, mu = 0.05, tau/dt = 0.8, predictor-
corrector source, FP32 storage and arithmetic with the displacement stored
and accumulated in FP64 (plain FP32 misses the 1e-5 bound on P after 500
steps; --precision fp32 runs it); u0 = 0 and a seeded
Gaussian-filtered velocity field (sigma = 32 cells, seed 2) scaled to the
calibrated peak velocity (tests/golden/large_strain_amplitude.json). A "step" is
one time step of the whole grid; the fused step kernel advances one or two
steps per launch (the autotuner picks).

Prints one JSON line with MLUPS, the HBM roofline fraction of the step kernel,
the FP64 oracle timed on the host cores on a bounded sample, and the rel-L2
error of the GPU against that oracle sample.

Timing: after the warm-up steps, --repeats windows of --steps time steps
each are timed with HIP events on the plate's stream; ms_per_step and the
roofline use the median window (every window's time is listed).

Roofline accounting (per lattice update): a lattice update reads the 13-value
state (f, u, j) of a site and writes it once, so its algorithmic bytes are
BYTES_PER_UPDATE of the storage form (208 B in FP64, 104 B in FP32, 120 B in
FP32 with an FP64 displacement, 84 B with 16-bit populations). A launch of
the step kernel processes sites x steps-per-launch updates, so
``achieved`` = BYTES_PER_UPDATE x sites x steps-per-launch / launch time, and
``frac`` is that over the HBM peak: the fraction of the ceiling of a scheme
that streams the state once per time step (MLUPS / (8 TB/s / BYTES_PER_UPDATE)).
With two steps per launch the kernel streams the state once per two updates,
so this figure can exceed what the HBM moves; the rate of the launch's own
minimum traffic (the state read and written once per launch) is reported
beside it as ``per_launch_state_GBps``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (fp64/fp32/fp16-storage) at stated error vs FP64 oracle; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one lattice update: the state f (9), u (2), j (2) of
# a site read once and written once
BYTES_PER_UPDATE = {"fp64": 2 * 13 * 8, "fp32": 2 * 13 * 4, "fp32u64": 2 * (9 * 4 + 2 * 8 + 2 * 4),
                    "fp16": 2 * (9 * 2 + 2 * 8 + 2 * 4),
                    "bf16": 2 * (9 * 2 + 2 * 8 + 2 * 4)}
# one pass of a launch over the state moves the same bytes per site
BYTES_PER_SITE_PASS = BYTES_PER_UPDATE
DTYPE = {"fp64": "f64", "fp32": "f32", "fp32u64": "f32 (f64 displacement)", "fp16": "f16-storage/f32",
         "bf16": "bf16-storage/f32"}


def _code_hash(files) -> str:
    """Hash of the sources' code: comments and blank space do not count, so
    an edit of comments keeps a counter record valid."""
    import re

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2208_13769_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    return _code_hash(["step_kernel.hpp", "lattice.hpp"])


def large_strain_amplitude() -> float:
    path = os.path.join(ROOT, "tests", "golden", "large_strain_amplitude.json")
    with open(path) as fh:
        return float(json.load(fh)["peak_velocity"])


def workload(name: str):
    from paper_2208_13769_amd import inputs

    if name == "large-strain-4096":
        n = 4096
        u0, v0 = inputs.filtered_random_velocity(n, n, 32.0, 2, large_strain_amplitude())
        return dict(nx=n, ny=n, precision="fp32u64", u0=u0, v0=v0, lam=0.1, mu=0.05, tau=0.8,
                    desc="periodic 4096x4096 D2Q9, neo-Hooke lam=0.1 mu=0.05, tau/dt=0.8, "
                         "predictor-corrector, FP32 arithmetic and storage with the displacement "
                         "accumulated in FP64; v0 Gaussian-filtered (sigma 32 cells, seed 2), "
                         "peak strain ~0.2 within 200 steps")
    if name == "shear-wave-64":
        n = 64
        u0, v0 = inputs.shear_wave(n, n, 1e-4, n)
        return dict(nx=n, ny=n, precision="fp64", u0=u0, v0=v0, lam=0.1, mu=0.05, tau=0.8,
                    desc="periodic 64x64, FP64, standing shear wave v_y = 1e-4 sin(2 pi x / 64); a plate this "
                         "small is latency-bound: read ms_per_step")
    if name == "fp16-4096":
        n = 4096
        u0, v0 = inputs.shear_wave(n, n, 1e-4, n)
        return dict(nx=n, ny=n, precision="fp16", u0=u0, v0=v0, lam=0.1, mu=0.05, tau=0.8,
                    desc="periodic 4096x4096, FP16 populations / FP64 u / FP32 j, shear wave")
    raise SystemExit(f"unknown workload {name}")


def traffic_for(precision: str, sites: int, block: int, segs: int, spl: int):
    """HBM bytes per launch from the committed rocprofv3 counter record, if it
    was taken on the current kernel source with the same launch shape."""
    path = os.path.join(ROOT, "profiles", f"step_{precision}_4096_counters.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("kernel_hash") != kernel_source_hash() or rec.get("sites") != sites
            or rec.get("tiling") != {"block": block, "n_segs": segs, "steps_per_launch": spl}):
        return None
    return rec.get("hbm_bytes_per_launch")


def timed_windows(solver, stream, steps: int, repeats: int):
    """Time `repeats` windows of `steps` time steps each with HIP events on
    the solver's stream (a device synchronisation on both sides of each).
    Returns the window times in ms and the host wall time of all windows."""
    import torch

    out = []
    wall0 = time.perf_counter()
    for _ in range(repeats):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        solver.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        out.append(ev0.elapsed_time(ev1))
    return out, time.perf_counter() - wall0


def step_roofline(prec: str, sites: int, spl: int, ms_step: float, traffic, kernel=None):
    """Roofline object of the step kernel: algorithmic bytes per launch are
    BYTES_PER_UPDATE x the updates one launch processes (sites x spl), over
    the launch's duration (spl time steps)."""
    ms_launch = spl * ms_step
    updates_launch = sites * spl
    bytes_launch = BYTES_PER_UPDATE[prec] * updates_launch
    achieved = bytes_launch / (ms_launch / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel or ("step2_kernel" if spl == 2 else "step_kernel"), "steps_per_launch": spl,
            "launch_us": round(ms_launch * 1e3, 2), "bytes_per_update": BYTES_PER_UPDATE[prec],
            "updates_per_launch": updates_launch, "algorithmic_bytes_per_launch": bytes_launch,
            # the launch's own minimum traffic: the state read and written once
            "per_launch_state_GBps": round(BYTES_PER_SITE_PASS[prec] * sites / (ms_launch / 1e3) / 1e9, 1),
            "mlups_ceiling_at_peak": round(HBM_PEAK_GBS * 1e3 / BYTES_PER_UPDATE[prec], 1)}


def cpu_baseline(wl, steps: int):
    """FP64 oracle on the same input: `steps` time steps of the full grid."""
    from oracle import oracle as O

    p = O.Params(nx=wl["nx"], ny=wl["ny"], lam=wl["lam"], mu=wl["mu"], tau_over_dt=wl["tau"])
    s = O.Solver(p, wl["u0"], wl["v0"])
    t0 = time.perf_counter()
    s.step(steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    mlups = wl["nx"] * wl["ny"] * steps / el / 1e6
    u, v, P = s.fields()
    return dict(value=mlups, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"{steps} time steps of the full {wl['nx']}x{wl['ny']} grid from the same seeded input, "
                       f"FP64, {el:.1f} s"), (u, v, P)


# Element sizes (f, u, j, compute) of each storage form.
ELEM = {"fp64": (8, 8, 8, 8), "fp32": (4, 4, 4, 4), "fp32u64": (4, 8, 4, 4), "fp16": (2, 8, 4, 4),
        "bf16": (2, 8, 4, 4)}


def general_bytes_per_site(precision: str) -> int:
    """Algorithmic bytes per material site and step of the general step: the
    state read and written once, plus the mask byte."""
    return BYTES_PER_UPDATE[precision] + 1


def copy_probe(mib: int, device):
    """A plain elementwise copy of `mib` MiB (float32 read + write), three
    times: its HBM counter readings calibrate the kernels' (profiling runs)."""
    import torch

    if mib <= 0:
        return
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def general_source_hash() -> str:
    # the host code that splits the plate between the fused kernel and the
    # 2D tiles decides the traffic too
    return _code_hash(["general_kernels.hpp", "step_kernel.hpp", "lattice.hpp", "lbm_solid.hip"])


def general_traffic_for(precision: str, n: int):
    """HBM bytes per step of the hole workload from the committed rocprofv3
    counter record, if it was taken on the current source at this size."""
    path = os.path.join(ROOT, "profiles", f"tile_step_{precision}_{n}_hole_counters.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_hash") != general_source_hash() or rec.get("n") != n:
        return None
    return rec.get("hbm_bytes_per_step")


TAU_HOLE = 0.55


def bench_hole(args):
    """The plate with a square hole of Sec. 7.2 at a size that fills the GPU:
    side l = 1 on n x n nodes (default 4096), a centred hole of 0.4 l, all four
    edges and the hole traction-free except for a normal traction of 0.02 mu
    on the top and bottom edges, lam = mu = rho0 = 1, starting
    at rest; tau/dt = 0.55, as the paper runs its Sec. 7 examples (reading
    Q24): at 0.8 the scheme itself diverges on this plate within a few
    hundred steps. It runs on the general step: the fused kernel for the
    strips and rows clear of the walls and the hole, beside 2D tiles for the
    rest."""
    import torch

    from oracle import oracle as O
    from paper_2208_13769_amd import lbm

    n = args.hole_n
    prec = args.precision or "fp32u64"
    h = int(round(0.4 * n))
    a = (n - h) // 2
    solid = np.ones((n, n), np.uint8)
    solid[a:a + h, a:a + h] = 0
    material = int(solid.sum())
    T = 0.02
    z = np.zeros((2, n, n))
    s = lbm.Solver(n, n, 1.0 / n, prec, "pc", walled=True)
    s.set_material(1.0, 1.0, 1.0, TAU_HOLE)
    s.set_boundary(lbm.LBM_EDGE_XMIN, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0))
    s.set_boundary(lbm.LBM_EDGE_XMAX, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0))
    s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_NEUMANN_T, (0.0, -T))
    s.set_boundary(lbm.LBM_EDGE_YMAX, lbm.LBM_BC_NEUMANN_T, (0.0, T))
    s.set_mask(solid)
    s.set_fields(z, z)
    copy_probe(args.copy_probe_mib, s.device)
    s.step(args.warmup)
    torch.cuda.synchronize()
    windows_ms, _ = timed_windows(s, s.stream, args.steps, args.repeats)
    ms_step = float(np.median(windows_ms)) / args.steps
    u, v, P, d, st = s.read()
    s.close()
    per_site = general_bytes_per_site(prec)
    # hole nodes move no state: the bytes count material nodes, as MLUPS does
    step_bytes = per_site * material
    achieved = step_bytes / (ms_step / 1e3) / 1e9
    traffic = general_traffic_for(prec, n)
    out = {
        "metric": METRIC, "value": round(material / (ms_step / 1e3) / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": f"plate with a centred square hole (Sec. 7.2 geometry) on {n}x{n} nodes, hole "
                               f"{h}x{h}, all edges and the hole traction-free except 0.02 mu normal traction on "
                               "top and bottom, lam = mu = 1, tau/dt = 0.55, predictor-corrector; general step (fused "
                               "kernel clear of walls and hole, 2D tiles for the rest); MLUPS counts material nodes",
                   "grid": [n, n], "material_sites": material, "precision": prec, "scheme": "pc",
                   "repeats": args.repeats, "window_ms": [round(w, 4) for w in windows_ms]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "general step: the fused kernel over the share clear of walls and the hole "
                               "(step2_list_kernel, two steps per launch, with 32/64-bit populations; else "
                               "step_list_kernel) beside tile_step_kernel on a second stream (traffic: HBM bytes "
                               "per step)",
                     "bytes_per_material_site": per_site},
        "run": {"status": int(st), "min_J": d.min_J, "max_strain": d.max_strain},
    }
    if not args.no_cpu_baseline:
        steps = args.cpu_steps
        p = O.Params(nx=n, ny=n, dx=1.0 / n, lam=1.0, mu=1.0, tau_over_dt=TAU_HOLE, bc_xmin=O.NEUMANN_T,
                     bc_xmax=O.NEUMANN_T, bc_ymin=O.NEUMANN_T, bc_ymax=O.NEUMANN_T, val_ymin=(0.0, -T),
                     val_ymax=(0.0, T), solid=solid)
        ref = O.Solver(p, z, z)
        t0 = time.perf_counter()
        ref.step(steps)
        el = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": material * steps / el / 1e6, "unit": "MLUPS", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{steps} time steps of the full grid from rest, FP64, {el:.1f} s"}
        g = lbm.Solver(n, n, 1.0 / n, prec, "pc", walled=True)
        g.set_material(1.0, 1.0, 1.0, TAU_HOLE)
        for e, val in ((lbm.LBM_EDGE_XMIN, (0.0, 0.0)), (lbm.LBM_EDGE_XMAX, (0.0, 0.0)),
                       (lbm.LBM_EDGE_YMIN, (0.0, -T)), (lbm.LBM_EDGE_YMAX, (0.0, T))):
            g.set_boundary(e, lbm.LBM_BC_NEUMANN_T, val)
        g.set_mask(solid)
        g.set_fields(z, z)
        g.step(steps)
        ug, _, Pg, _, _ = g.read()
        g.close()
        uo, _, Po = ref.fields()
        out["error_vs_oracle"] = {"steps": steps, "rel_l2_u": float(np.linalg.norm(ug - uo) / np.linalg.norm(uo)),
                                  "rel_l2_P": float(np.linalg.norm(Pg - Po) / np.linalg.norm(Po))}
    print(json.dumps(out), flush=True)
    if st != 0:
        sys.exit(f"the hole plate diverged (status {st}): its timing is not a valid measurement")


def bench_plates(args):
    """256 plates of uneven sizes in one batch (one persistent launch per one
    or two steps, graph-captured chunks), FP16 populations, 2000 steps each."""
    import torch

    from paper_2208_13769_amd import inputs, lbm
    from paper_2208_13769_amd.batch import Batch, PlateSpec

    plates = inputs.plate_batch(256, seed=4)
    steps = args.plate_steps
    specs, fields = [], []
    for pl in plates:
        specs.append(PlateSpec(nx=pl.n, ny=pl.n, lam=pl.lam, mu=pl.mu, tau_over_dt=0.8,
                               bc_ymin=lbm.LBM_BC_DIRICHLET_J, bc_ymax=lbm.LBM_BC_NEUMANN_T))
        fields.append(inputs.top_pulse(pl.n, 0.01))
    sites = sum(sp.nx * sp.ny for sp in specs)

    def run_batch(precision, keep=None):
        keep = range(len(specs)) if keep is None else keep
        sel = [(specs[i], fields[i]) for i in keep]
        arena = sum(Batch.plate_bytes_for(sp.nx, sp.ny, precision) for sp, _ in sel) + (64 << 20)
        b = Batch(max_plates=len(sel), arena_bytes=arena, precision=precision, walled=True)
        if args.batch_spl:
            b.set_steps_per_launch(args.batch_spl)
        slots = [b.add(sp, u0, v0, steps) for sp, (u0, v0) in sel]
        b.step(args.chunk)  # warm-up chunk: graph capture, first touch
        torch.cuda.synchronize()
        # restart from the start fields for the timed run
        for s_ in slots:
            b.retire(s_)
        slots = [b.add(sp, u0, v0, steps) for sp, (u0, v0) in sel]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        left = steps
        while left > 0:
            b.step(min(args.chunk, left))
            left -= args.chunk
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        return b, slots, ms

    copy_probe(args.copy_probe_mib, torch.device("cuda:0"))
    b16, s16, ms16 = run_batch("fp16")
    b16_spl = b16.steps_per_launch()
    flagged = [i for i, s_ in enumerate(s16) if b16.query(s_)[2]]
    b64, s64, ms64 = run_batch("fp64")
    # every plate's error against the same plate in the FP64 batch; a plate
    # counts as completed only if it ran without the unstable flag AND within
    # the 1e-3 bound of 16-bit storage on u and P
    per_plate = []
    for i in range(len(specs)):
        u2, _, p2, d2, st2 = b64.read(s64[i])
        fp64_bad = bool(b64.query(s64[i])[2])
        if i in flagged:
            per_plate.append((i, float("inf"), float("inf"), fp64_bad))
            continue
        u1, _, p1, _, _ = b16.read(s16[i])
        per_plate.append((i, float(np.linalg.norm(u1 - u2) / np.linalg.norm(u2)),
                          float(np.linalg.norm(p1 - p2) / np.linalg.norm(p2)), fp64_bad))
    b16.close()
    b64.close()
    tol = 1e-3
    bad = [i for i, eu, ep, _ in per_plate if not (eu <= tol and ep <= tol)]
    done = [i for i in range(len(specs)) if i not in bad]
    done_sites = sum(specs[i].nx * specs[i].ny for i in done)
    mlups16 = done_sites * steps / (ms16 / 1e3) / 1e6
    errs_u = [eu for i, eu, ep, _ in per_plate if i in done]
    errs_p = [ep for i, eu, ep, _ in per_plate if i in done]
    worst = max((x for x in per_plate if x[0] in done), key=lambda x: max(x[1], x[2]))
    # second run without the plates beyond the interior's stability limit
    # (the predictor-corrector grows for lam/mu above 7.0 at tau/dt = 0.8,
    # mode model), so that every plate completes
    clean = [i for i in range(len(specs)) if specs[i].lam / specs[i].mu <= 7.0]
    bc, sc, msc = run_batch("fp16", clean)
    bad_c = sum(1 for s_ in sc if bc.query(s_)[2])
    clean_sites = sum(specs[i].nx * specs[i].ny for i in clean)
    bc.close()
    # plain FP32, one plate at a time, on every 16th plate
    sample = list(range(0, len(specs), 16))
    t_fp32, ups_fp32 = 0.0, 0
    for i in sample:
        sp, (u0, v0) = specs[i], fields[i]
        s = lbm.Solver(sp.nx, sp.ny, 1.0, "fp32", "pc")
        s.set_material(1.0, sp.lam, sp.mu, sp.tau_over_dt)
        s.set_boundary(lbm.LBM_EDGE_YMIN, sp.bc_ymin, (0.0, 0.0))
        s.set_boundary(lbm.LBM_EDGE_YMAX, sp.bc_ymax, (0.0, 0.0))
        s.set_fields(u0, v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        t_fp32 += time.perf_counter() - t0
        ups_fp32 += sp.nx * sp.ny * steps
        s.close()
    out = {
        "metric": METRIC, "value": round(mlups16, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": args.chunk, "ms_per_step": round(ms16 / steps, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE["fp16"], "data": "synthetic",
        "config": {"workload": "256 plates, side log-uniform 64..1024 (seed 4), lam U[0.05,0.2], mu U[0.02,0.1], "
                               "tau/dt=0.8, periodic in x, clamped bottom, traction-free top, initial top "
                               "velocity pulse 0.01; FP16 populations; one batch, one persistent launch per "
                               "one or two steps",
                   "plates": len(specs), "sites": sites, "chunk": args.chunk,
                   "steps_per_launch": b16_spl},
        "completed_plates": len(done),
        "failed_plates": [{"plate": i, "n": specs[i].nx, "lam_over_mu": round(specs[i].lam / specs[i].mu, 3),
                           "flagged_unstable": i in flagged, "rel_l2_u": eu, "rel_l2_P": ep,
                           "fp64_flagged_unstable": f64}
                          for i, eu, ep, f64 in per_plate if i in bad],
        "error_vs_fp64": {"median_rel_l2_u": float(np.median(errs_u)), "max_rel_l2_u": float(np.max(errs_u)),
                          "median_rel_l2_P": float(np.median(errs_p)), "max_rel_l2_P": float(np.max(errs_p)),
                          "worst_plate": {"plate": worst[0], "n": specs[worst[0]].nx,
                                          "lam_over_mu": round(specs[worst[0]].lam / specs[worst[0]].mu, 3),
                                          "rel_l2_u": worst[1], "rel_l2_P": worst[2]},
                          "bound": tol, "over": "completed plates (MLUPS counts these only)",
                          "reference": "the same batch in FP64 (bitwise equal to single-plate FP64)"},
        "clean_run": {"rejected": "lam/mu > 7 (the interior's stability limit at tau/dt 0.8)", "plates": len(clean),
                      "sites": clean_sites,
                      "diverged_plates": bad_c, "ms_per_step": round(msc / steps, 5),
                      "MLUPS": round(clean_sites * steps / (msc / 1e3) / 1e6, 1)},
        "fp64_batch_MLUPS": round(sites * steps / (ms64 / 1e3) / 1e6, 1),
        "plain_fp32_one_at_a_time_MLUPS": round(ups_fp32 / t_fp32 / 1e6, 1),
        "plain_fp32_sample": f"every 16th plate ({len(sample)} plates), {steps} steps each",
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5, help="timed windows of --steps steps; the median is reported")
    ap.add_argument("--workload", default="large-strain-4096",
                    help="large-strain-4096 (default) | fp16-4096 | shear-wave-64 | plates-256 | hole")
    ap.add_argument("--precision", default=None,
                    help="override the workload's precision (fp64, fp32, fp32u64, fp16, bf16)")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiling", default="auto",
                    help="auto | default | BLOCK,NSEGS,STEPS_PER_LAUNCH (0,0,1: the general step)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run a plain elementwise copy of this many MiB (float32 read + "
                         "write) three times: its HBM counter readings calibrate the step kernel's")
    ap.add_argument("--plate-steps", type=int, default=2000, help="plates-256: steps per plate")
    ap.add_argument("--chunk", type=int, default=200, help="plates-256: steps per graph-captured chunk")
    ap.add_argument("--batch-spl", type=int, default=0,
                    help="plates-256: time steps per batch launch (1 or 2; 0 = the batch's default)")
    ap.add_argument("--hole-n", type=int, default=4096, help="hole: nodes per side")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the single-plate path has no multi-GPU decomposition).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_13769_amd import lbm
    from paper_2208_13769_amd.autotune import GENERAL, apply_tiling, best_tiling

    if args.workload == "hole":
        bench_hole(args)
        return
    if args.workload == "plates-256":
        bench_plates(args)
        return
    wl = workload(args.workload)
    if args.precision:
        wl["precision"] = args.precision
        wl["desc"] += f" (storage form {args.precision})"
    nx, ny, prec = wl["nx"], wl["ny"], wl["precision"]
    s = lbm.Solver(nx, ny, 1.0, prec, "pc")
    s.set_material(1.0, wl["lam"], wl["mu"], wl["tau"])
    s.set_fields(wl["u0"], wl["v0"])
    tiling_source, general = "default", False
    if args.tiling == "auto":
        t = best_tiling(s, nx, ny, prec, "pc")
        apply_tiling(s, t)
        s.set_fields(wl["u0"], wl["v0"])
        tiling_source, general = "autotuned", tuple(t) == GENERAL
    elif args.tiling != "default":
        t = tuple(map(int, args.tiling.split(",")))
        apply_tiling(s, t)
        tiling_source, general = "given", t == GENERAL
    block, segs = s.tiling()
    spl = 1 if general else s.steps_per_launch()

    stream = s.stream
    copy_probe(args.copy_probe_mib, s.device)
    s.step(args.warmup)
    torch.cuda.synchronize()
    windows_ms, wall = timed_windows(s, stream, args.steps, args.repeats)
    ms = float(np.median(windows_ms))
    _, _, _, diag, status = s.read(want_fields=False)

    sites = nx * ny
    ms_step = ms / args.steps
    mlups = sites * args.steps / (ms / 1e3) / 1e6
    roofline = step_roofline(prec, sites, spl, ms_step,
                             None if general else traffic_for(prec, sites, block, segs, spl),
                             "tile_step_kernel" if general else None)

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": wl["desc"], "grid": [nx, ny], "sites": sites, "precision": prec, "scheme": "pc",
                   "tiling": ({"path": "general step (2D tiles, 512 threads)", "source": tiling_source} if general else
                              {"block": block, "n_segs": segs, "steps_per_launch": spl, "source": tiling_source}),
                   "repeats": args.repeats, "window_ms": [round(w, 4) for w in windows_ms],
                   "wall_s": round(wall, 4)},
        "roofline": roofline,
        "run": {"status": int(status), "max_strain": diag.max_strain, "min_J": diag.min_J},
    }

    if not args.no_cpu_baseline:
        base, (uo, vo, Po) = cpu_baseline(wl, args.cpu_steps)
        out["cpu_baseline"] = base
        # the GPU on the same sample, for the error statement
        g = lbm.Solver(nx, ny, 1.0, prec, "pc")
        g.set_material(1.0, wl["lam"], wl["mu"], wl["tau"])
        g.set_fields(wl["u0"], wl["v0"])
        g.step(args.cpu_steps)
        ug, vg, Pg, _, _ = g.read()
        g.close()
        out["error_vs_oracle"] = {
            "steps": args.cpu_steps,
            "rel_l2_u": float(np.linalg.norm(ug - uo) / np.linalg.norm(uo)),
            "rel_l2_P": float(np.linalg.norm(Pg - Po) / np.linalg.norm(Po)),
        }
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
