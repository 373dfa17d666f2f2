"""Request server for plate solves: continuous batching on one GPU.

Requests arrive over time (Poisson process). Each asks for a periodic plate
of side N to be advanced a number of steps from a seeded start field; the
answer is the final displacement, velocity and stress fields.

``BatchServer`` keeps every admitted plate resident in one batch and
advances all of them together in chunks of ``chunk`` steps (one persistent
launch per step, graph-captured). At each chunk boundary it returns the
finished plates, frees their memory and admits waiting requests in arrival
order while the batch arena has room (admission by device-memory
footprint). Requests that arrive while others run therefore join the work
already on the GPU.

``SerialServer`` is the reference: one request at a time, FIFO, each on
its own single-plate solver.

Latency of a request = time its fields are back on the host - its arrival.
Throughput = lattice updates of all requests / (last finish - first arrival).
"""
from __future__ import annotations

import argparse
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import inputs, lbm
from .batch import Batch, PlateSpec


@dataclass
class Request:
    rid: int
    n: int
    steps: int
    seed: int
    arrival: float = 0.0
    lam: float = 0.1
    mu: float = 0.05
    tau: float = 0.8
    u0: np.ndarray = field(default=None, repr=False)
    v0: np.ndarray = field(default=None, repr=False)

    @property
    def updates(self) -> int:
        return self.n * self.n * self.steps


def make_requests(count: int, seed: int, n_median: float = 256.0, sigma_ln: float = 0.83, n_min: int = 32,
                  n_max: int = 2048, steps_min: int = 500, steps_max: int = 20000, peak: float = 1e-4):
    """Seeded request mix: side N lognormal (median, log-sd) clipped to
    [n_min, n_max]; steps uniform in [steps_min, steps_max]; start field u0 = 0
    and a Gaussian-filtered random velocity (sigma = max(2, N/16) cells, a
    seed per request) with peak |v| = peak. Arrival times are set later."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(count):
        n = int(np.clip(round(n_median * math.exp(sigma_ln * rng.standard_normal())), n_min, n_max))
        steps = int(rng.integers(steps_min, steps_max + 1))
        r = Request(rid=k, n=n, steps=steps, seed=seed * 100003 + k)
        r.u0, r.v0 = inputs.filtered_random_velocity(n, n, max(2.0, n / 16.0), r.seed, peak)
        reqs.append(r)
    return reqs


def set_arrivals(reqs, rate: float, seed: int):
    """Poisson arrivals at `rate` requests per second, starting at t = 0."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    t = 0.0
    for r in reqs:
        r.arrival = t
        t += rng.exponential(1.0 / rate)


def _summary(name, reqs, finish, rejected=()):
    """Latency percentiles and MLUPS over the requests that were served;
    rejected requests (too large for the server) are counted apart."""
    done = [r for r in reqs if r.rid in finish]
    out = {"server": name, "requests": len(reqs), "rejected": len(rejected)}
    if not done:
        return out
    lat = np.array([finish[r.rid] - r.arrival for r in done])
    span = max(finish.values()) - min(r.arrival for r in done)
    ups = sum(r.updates for r in done)
    out.update({"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "makespan_s": span, "MLUPS": ups / span / 1e6})
    return out


def _progress(name, done, total, every):
    """One line per `every` finished requests (0: silent)."""
    if every and done % every == 0:
        print(json.dumps({"server": name, "finished": done, "of": total}), flush=True)


def _wait_until(start, t):
    while True:
        d = t - (time.perf_counter() - start)
        if d <= 0:
            return
        time.sleep(min(d, 0.002))


class SerialServer:
    """One request at a time on a single-plate solver (FIFO)."""

    def __init__(self, precision: str = "fp32", progress: int = 0):
        self.precision = precision
        self.progress = progress

    def serve_one(self, r: Request):
        s = lbm.Solver(r.n, r.n, 1.0, self.precision, "pc")
        s.set_material(1.0, r.lam, r.mu, r.tau)
        s.set_fields(r.u0, r.v0)
        s.step(r.steps)
        u, v, P, d, st = s.read()
        s.close()
        return u, v, P, d, st

    def run(self, reqs, keep=None):
        start = time.perf_counter()
        finish, results = {}, {}
        for r in sorted(reqs, key=lambda q: q.arrival):
            _wait_until(start, r.arrival)
            out = self.serve_one(r)
            finish[r.rid] = time.perf_counter() - start
            if keep is not None and r.rid in keep:
                results[r.rid] = out
            _progress(f"serial-{self.precision}", len(finish), len(reqs), self.progress)
        return _summary(f"serial-{self.precision}", reqs, finish), finish, results


class BatchServer:
    """Continuous batching: resident plates advanced together in chunks."""

    def __init__(self, arena_bytes: int, precision: str = "fp16", chunk: int = 200, max_plates: int = 512,
                 progress: int = 0, batch=None):
        self.batch = batch if batch is not None else Batch(max_plates=max_plates, arena_bytes=arena_bytes,
                                                           precision=precision, walled=False)
        self.precision = precision
        self.chunk = chunk
        self.progress = progress

    def close(self):
        self.batch.close()

    def run(self, reqs, keep=None):
        b = self.batch
        pending = deque(sorted(reqs, key=lambda q: q.arrival))
        waiting = deque()
        live = {}
        finish, results, rejected = {}, {}, []
        max_live = 0
        start = time.perf_counter()
        while pending or waiting or live:
            now = time.perf_counter() - start
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                r = waiting[0]
                if not b.fits_empty(r.n, r.n):
                    # larger than the whole batch: it would wait forever and
                    # hold up every request behind it
                    rejected.append(waiting.popleft().rid)
                    continue
                slot = b.add(PlateSpec(nx=r.n, ny=r.n, lam=r.lam, mu=r.mu, tau_over_dt=r.tau), r.u0, r.v0, r.steps)
                if slot is None:
                    if not live:  # no room even in an empty batch (e.g. no free slot)
                        rejected.append(waiting.popleft().rid)
                        continue
                    break  # no room: wait for plates to finish
                waiting.popleft()
                live[slot] = r
            max_live = max(max_live, len(live))
            if not live:
                if pending:
                    _wait_until(start, pending[0].arrival)
                continue
            b.step(self.chunk)
            b.synchronize()
            for slot, r in list(live.items()):
                done, left, bad = b.query(slot)
                if left == 0 or bad:
                    out = b.read(slot)
                    finish[r.rid] = time.perf_counter() - start
                    if keep is not None and r.rid in keep:
                        results[r.rid] = out
                    b.retire(slot)
                    del live[slot]
                    _progress(f"batched-{self.precision}", len(finish), len(reqs), self.progress)
        summ = _summary(f"batched-{self.precision}", reqs, finish, rejected)
        summ["rejected_ids"] = rejected
        summ["max_resident"] = max_live
        summ["chunk"] = self.chunk
        return summ, finish, results


def capacity(reqs, precision="fp32"):
    """Requests per second of the serial server on back-to-back requests."""
    srv = SerialServer(precision)
    t0 = time.perf_counter()
    for r in reqs:
        srv.serve_one(r)
    return len(reqs) / (time.perf_counter() - t0)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--rates", default="0.5,0.8,0.95", help="fractions of the serial FP32 capacity")
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--arena-gib", type=float, default=16.0)
    ap.add_argument("--steps-max", type=int, default=20000)
    ap.add_argument("--progress", type=int, default=0, help="print a line every N finished requests")
    ap.add_argument("--capacity", type=float, default=0.0,
                    help="serial FP32 capacity in requests/s to set the rates from (0: measure it)")
    args = ap.parse_args()
    import torch

    reqs = make_requests(args.requests, args.seed, steps_max=args.steps_max)
    # warm both paths (kernels, graphs, allocator) on a few small requests
    warm = make_requests(3, args.seed + 1, n_median=64, steps_max=600)
    capacity(warm)
    srv = BatchServer(int(args.arena_gib * (1 << 30)), chunk=args.chunk, progress=args.progress)
    set_arrivals(warm, 1e6, 0)
    srv.run(warm)
    cap = args.capacity if args.capacity > 0 else capacity(reqs[: max(4, len(reqs) // 6)])
    out = {"capacity_serial_fp32_req_per_s": cap, "requests": args.requests,
           "mix": "N lognormal(median 256, sd_ln 0.83) in [32, 2048], steps U[500, %d], periodic, "
                  "lam=0.1 mu=0.05 tau/dt=0.8, Gaussian-filtered start velocity" % args.steps_max,
           "runs": []}
    for frac in [float(x) for x in args.rates.split(",")]:
        set_arrivals(reqs, frac * cap, args.seed)
        s_b, *_ = srv.run(reqs)
        print(json.dumps({"load": frac, "batched_fp16": s_b}), flush=True)
        s_s, *_ = SerialServer("fp32", progress=args.progress).run(reqs)
        out["runs"].append({"load": frac, "rate_req_per_s": frac * cap, "batched_fp16": s_b, "serial_fp32": s_s})
        print(json.dumps(out["runs"][-1]), flush=True)
    srv.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
