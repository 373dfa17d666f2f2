"""Launch-shape autotuner of a plate's time step.

The step's results do not depend on how it is launched, only its speed does:
the fused step kernel's shape (threads per block = columns per strip + halo,
row segments per strip, one or two steps per launch), or the general step
(2D tiles whose stages run in parallel, the faster one on small plates). For
a plate size, precision and scheme the tuner times a short run of each
candidate with HIP events on the solver's stream, times the fastest few
again over longer runs, and keeps the fastest of those.
Results are cached in a JSON file (``$LBM_AUTOTUNE_CACHE``, default
``~/.cache/lbm_solid/autotune.json``) keyed by device name and problem.

Tuning advances the solver's state: call ``set_fields`` again afterwards.
``best_tiling`` returns (block, segments, steps per launch), with
``GENERAL`` = (0, 0, 1) standing for the general step; ``apply_tiling`` sets
either on a solver.
"""
from __future__ import annotations

import json
import os

HALO = {"pc": 5, "explicit": 3}
GENERAL = (0, 0, 1)  # the general step in place of a fused-kernel shape


def _cache_path() -> str:
    return os.environ.get("LBM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbm_solid", "autotune.json"))


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def halo(precision: str, scheme: str, spl: int) -> int:
    """Halo columns of a launch: the stencil reach of its steps, one more per
    step with 16-bit (deviation) storage, whose store needs the gradient of
    the new displacement."""
    return (HALO[scheme] + (1 if precision in ("fp16", "bf16") else 0)) * spl


def strips(nx: int, block: int, precision: str, scheme: str, spl: int) -> int:
    """Column strips of a launch shape (the library's own rule: strips as wide
    as the block minus both halos, rounded down to a multiple of 32 columns)."""
    halo_ = halo(precision, scheme, spl)
    wmax = block - 2 * halo_
    if nx <= wmax:
        return 1
    align = 32
    w = wmax // align * align if wmax >= align else wmax
    return -(-nx // w)


def candidates(solver, nx: int, ny: int, precision: str, scheme: str):
    """(block, segments, steps per launch): block widths that fit the plate,
    one or two time steps per launch (two only with the predictor-corrector
    and where the library can launch the shape), and segment counts that fill
    1/2, 1, 2, 3 or 4 waves of the blocks the device holds at once (each
    segment at least 8 rows). A plate whose grid fits one wave also tries
    segments of ny, ny/2 and ny/4 rows: a block marches its rows one after
    another, so on a small plate shorter segments cut the time of a step."""
    out = []
    for spl in ((1, 2) if scheme == "pc" else (1,)):
        for block in (64, 128, 256, 512):
            resident = solver.resident_blocks(block, spl)
            if resident <= 0:
                continue
            h = halo(precision, scheme, spl)
            n_str = strips(nx, block, precision, scheme, spl)
            if block > 64 and n_str == 1 and nx <= (block // 2) - 2 * h:
                continue  # a narrower block already covers the width
            seen = set()
            for waves in (0.5, 1, 2, 3, 4):
                segs = max(1, min(max(1, ny // 8), int(waves * resident) // n_str))
                if segs not in seen:
                    seen.add(segs)
                    out.append((block, segs, spl))
            for rows in (1, 2, 4):
                segs = max(1, ny // rows)
                if n_str * segs <= resident and segs not in seen:
                    seen.add(segs)
                    out.append((block, segs, spl))
    out.append(GENERAL)
    return out


def apply_tiling(solver, tiling) -> None:
    """Run the solver's steps with a candidate of ``candidates``."""
    block, segs, spl = tiling
    if tuple(tiling) == GENERAL:
        solver.set_general_path(True)
        return
    solver.set_general_path(False)
    solver.set_steps_per_launch(spl)
    solver.set_tiling(block, segs)


def _time(solver, stream, steps: int) -> float:
    """ms per step of `steps` steps with HIP events on the solver's stream."""
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(solver, nx: int, ny: int, precision: str, scheme: str, window_ms: float = 2.0, finalists: int = 3):
    """Time every candidate; returns ((block, segs, steps per launch), ms per
    step, table). The device is first kept busy for a while on the first
    candidate (its clocks ramp up over the first milliseconds of work), each
    candidate then runs a window of about `window_ms` (at least 6 steps),
    and the `finalists` fastest run again over four such windows: the
    fastest of those wins. Short single windows ranked shapes within a few
    per cent of each other by noise."""
    stream = solver.stream
    cands = candidates(solver, nx, ny, precision, scheme)
    apply_tiling(solver, cands[0])
    solver.step(2)
    t0 = _time(solver, stream, 4)
    steps = max(6, min(400, int(window_ms / max(t0, 1e-4)) + 1))
    _time(solver, stream, max(1, int(20.0 / max(t0, 1e-4))))  # about 20 ms of work
    table = []
    for c in cands:
        apply_tiling(solver, c)
        solver.step(2)
        table.append([*c, _time(solver, stream, steps)])
    table.sort(key=lambda r: r[3])
    best, best_ms = None, float("inf")
    for r in table[:finalists]:
        c = tuple(r[:3])
        apply_tiling(solver, c)
        solver.step(2)
        ms = _time(solver, stream, 4 * steps)
        r.append(ms)
        if ms < best_ms:
            best, best_ms = c, ms
    return best, best_ms, table


def best_tiling(solver, nx: int, ny: int, precision: str, scheme: str):
    import torch

    key = f"{torch.cuda.get_device_name(solver.device)}|{nx}x{ny}|{precision}|{scheme}|v7"
    cache = _load_cache()
    if key in cache:
        return tuple(cache[key]["tiling"])
    best, ms, table = tune(solver, nx, ny, precision, scheme)
    cache[key] = {"tiling": list(best), "ms_per_step": ms, "table": table}
    _store_cache(cache)
    return best
