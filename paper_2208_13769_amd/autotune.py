"""Launch-shape autotuner for the fused step kernel.

The step kernel's results do not depend on its launch shape (threads per
block = columns per strip + halo, and row segments per strip), only its speed
does. For a plate size, precision and scheme the tuner times a short run of
each candidate shape with HIP events on the solver's stream and keeps the
fastest. Results are cached in a JSON file (``$LBM_AUTOTUNE_CACHE``, default
``~/.cache/lbm_solid/autotune.json``) keyed by device name and problem.

Tuning advances the solver's state: call ``set_fields`` again afterwards.
"""
from __future__ import annotations

import json
import os

HALO = {"pc": 5, "explicit": 3}


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


def candidates(nx: int, ny: int, scheme: str):
    """Block widths that fit the plate and segment counts spanning 1/4 to 16
    blocks per CU of a 256-CU device, each segment at least 8 rows."""
    out = []
    for block in (64, 128, 256, 512):
        w = block - 2 * HALO[scheme]
        strips = -(-nx // w)
        if block > 64 and strips == 1 and nx <= (block // 2) - 2 * HALO[scheme]:
            continue  # a narrower block already covers the width
        seen = set()
        for target in (64, 128, 256, 512, 1024, 2048, 4096):
            segs = max(1, min(ny // 8 if ny >= 8 else 1, -(-target // strips)))
            if segs not in seen:
                seen.add(segs)
                out.append((block, segs))
    return out


def tune(solver, nx: int, ny: int, precision: str, scheme: str, steps: int = 6):
    import torch

    stream = solver.stream
    best, best_ms, table = None, float("inf"), []
    for block, segs in candidates(nx, ny, scheme):
        solver.set_tiling(block, segs)
        solver.step(2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        table.append([block, segs, ms])
        if ms < best_ms:
            best, best_ms = (block, segs), ms
    return best, best_ms, table


def best_tiling(solver, nx: int, ny: int, precision: str, scheme: str):
    import torch

    key = f"{torch.cuda.get_device_name(solver.device)}|{nx}x{ny}|{precision}|{scheme}"
    cache = _load_cache()
    if key in cache:
        return tuple(cache[key]["tiling"])
    best, ms, table = tune(solver, nx, ny, precision, scheme)
    cache[key] = {"tiling": list(best), "ms_per_step": ms, "table": table}
    _store_cache(cache)
    return best
