"""Request loops over the batched solver (aq_batch_* in include/aqlbm.h).

* `sweep`: a parameter sweep of independent steady-state solves (uneven lattice sizes,
  per-request relaxation time, permeability, inflow, chamber angle, Rayleigh number and
  orientation), all submitted at time zero and admitted as memory, slots and the
  active-node cap allow (continuous batching: a finished solve frees its slot for the next).
* `serve`: the same solves arriving as a Poisson stream; latency = finish - arrival.

Both only schedule: admission, stepping, convergence checks and retirement run in the
library.  Tile shapes come from `autotune_shape`, which times the candidate 256-thread tiles
on one instance of each (size, storage) class with aq_autotune_tile and caches the winner.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

import aqinputs as A

from . import Batch, Solver, F16S, F32, F64, AQ_OK


class ShapeCache:
    """(gfx arch, storage, nx, ny) -> tile shape, optionally persisted as JSON."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.d = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.d = json.load(f)

    def key(self, storage, nx, ny):
        return f"gfx950/{storage}/{nx}x{ny}"

    def get(self, storage, nx, ny):
        v = self.d.get(self.key(storage, nx, ny))
        return tuple(v) if v else None

    def put(self, storage, nx, ny, shape):
        self.d[self.key(storage, nx, ny)] = list(shape)
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.d, f, indent=1)


def autotune_shape(cache: ShapeCache, p, mask, walls, n_launch=20):
    shape = cache.get(p.storage, p.nx, p.ny)
    if shape is None:
        s = Solver(p, mask, walls)
        tx, ty, _ = s.autotune(n_launch, only_256=True)
        s.close()
        shape = (tx, ty)
        cache.put(p.storage, p.nx, p.ny, shape)
    return shape


def sweep_request(seed: int, storage: int, large_every: int = 0, check_interval: int = 100):
    """One request of the sweep distribution (seeded): size uniform over the four classes,
    or 2048x1024 for every `large_every`-th seed when set."""
    nx, ny = A.batch_size_of(seed)
    if large_every and seed % large_every == large_every - 1:
        nx, ny = 2048, 1024
    p, mask, walls, geo = A.sweep_instance(seed, nx, ny, tau_f="draw", phi_deg="draw", storage=storage,
                                           check_interval=check_interval)
    return p, mask, walls


def _percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def run_requests(make, arrivals, *, budget_bytes, max_slots=512, max_active_nodes=0, tol=1e-6,
                 drift_tol=1e-3, max_steps=200000, intervals_per_call=1, cache=None, time_limit=None,
                 check_interval=100, log=None):
    """Admit request i (built by make(i) -> (params, mask, walls) when it is first
    considered) at its arrival time (seconds after start) into one batch and run until all
    finish or `time_limit`.  Returns summary statistics and per-request records."""
    cache = cache or ShapeCache()
    b = Batch(budget_bytes=budget_bytes, max_slots=max_slots, max_active_nodes=max_active_nodes,
              max_tiles=1 << 21, check_interval=check_interval)
    n_req = len(arrivals)
    built = {}
    order = sorted(range(n_req), key=lambda i: arrivals[i])
    queue = []                 # arrived, not yet admitted (FIFO)
    nxt = 0
    admitted_at, finished = {}, {}
    active_of = {}
    t0 = time.perf_counter()
    node_updates = 0.0
    while len(finished) < n_req:
        now = time.perf_counter() - t0
        if time_limit is not None and now > time_limit:
            break
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            queue.append(order[nxt])
            nxt += 1
        while queue:
            i = queue[0]
            if i not in built:
                built[i] = make(i)
            p, mask, walls = built[i]
            shape = autotune_shape(cache, p, mask, walls)
            slot = b.admit(p, mask, walls, tile=shape, tol=tol, drift_tol=drift_tol, max_steps=max_steps,
                           request_id=i)
            if slot is None:
                break
            queue.pop(0)
            admitted_at[i] = time.perf_counter() - t0
            active_of[i] = int(A.active(mask).sum())
            del built[i]
        info = b.info()
        if info["running"] == 0:
            if nxt < len(order) and not queue:
                time.sleep(max(0.0, min(0.01, arrivals[order[nxt]] - (time.perf_counter() - t0))))
                continue
            if not queue:
                break
        if info["running"]:
            b.run(intervals_per_call)
            node_updates += info["active_nodes"] * intervals_per_call * check_interval
        for r in b.poll():
            i = r["request_id"]
            r["t_done"] = time.perf_counter() - t0
            r["t_arrival"] = arrivals[i]
            r["t_admit"] = admitted_at[i]
            finished[i] = r
            if log:
                log(r)
    wall = time.perf_counter() - t0
    b.close()
    lat = [r["t_done"] - r["t_arrival"] for r in finished.values()]
    ok = [r for r in finished.values() if r["status"] == AQ_OK]
    return {
        "requests": n_req, "finished": len(finished), "converged": len(ok),
        "not_converged": sum(r["status"] == -5 for r in finished.values()),
        "diverged": sum(r["status"] == -4 for r in finished.values()),
        "fallbacks": sum(r["fallback"] for r in finished.values()),
        "wall_s": wall, "solves_per_s": len(finished) / wall if wall > 0 else 0.0,
        "latency_p50_s": _percentile(lat, 50), "latency_p99_s": _percentile(lat, 99),
        "aggregate_active_mlups": node_updates / wall / 1e6 if wall > 0 else 0.0,
        "records": finished,
    }


def sweep(n=512, storage=F32, tol=1e-6, budget_bytes=64 << 30, max_steps=200000, **kw):
    return run_requests(lambda i: sweep_request(i, storage), [0.0] * n, budget_bytes=budget_bytes, tol=tol,
                        max_steps=max_steps, **kw)


def poisson_arrivals(n, rate, seed0=1000):
    """Arrival times of requests seed0, seed0+1, ...: cumulative exponential gaps drawn from
    the 'arrival' counter of each request's seed."""
    t, out = 0.0, []
    for i in range(n):
        t += A.interarrival(seed0 + i, rate)
        out.append(t)
    return out


def serve(rate=50.0, duration=60.0, storage=F16S, tol=1e-6, budget_bytes=64 << 30, max_steps=200000,
          seed0=1000, large_every=10, **kw):
    n = int(rate * duration * 1.5) + 10
    arr = [t for t in poisson_arrivals(n, rate, seed0) if t <= duration]
    return run_requests(lambda i: sweep_request(seed0 + i, storage, large_every=large_every), arr,
                        budget_bytes=budget_bytes, tol=tol, max_steps=max_steps, **kw)
