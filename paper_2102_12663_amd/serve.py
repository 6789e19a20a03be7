"""Request loops over the batched solver (aq_batch_* in include/aqlbm.h).

* `sweep`: a parameter sweep of independent steady-state solves (uneven lattice sizes,
  per-request relaxation time, permeability, inflow, chamber angle, Rayleigh number and
  orientation), all submitted at time zero and admitted as memory, slots and the
  active-node cap allow (continuous batching: a finished solve frees its slot for the next).
* `serve`: the same solves arriving as a Poisson stream; latency = finish - arrival.
* `calibrate`: the healthy-eye procedure of section 3.1 as dependent requests: for each
  eye (lumped meshwork outlet), adjust the meshwork thickness until the steady IOP is the
  target one.  Each round runs the resident solve to its steady residual, reads the IOP,
  sets the new thickness and resumes from the current state (warm start).

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

from . import Batch, Solver, F16S, F32, F64, AQ_OK, AQ_RESULT_FLOOR

# statuses of a finished request that count as a solve: residual below tol, or (F16S) the
# state accepted at binary16's rounding floor by the IOP drift check
SOLVED = (AQ_OK, AQ_RESULT_FLOOR)


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


def default_budget(reserve_bytes=12 << 30, cap_bytes=288 * 10 ** 9):
    """Serving arena: the device's free HBM (at most 288 GB) minus a reserve for the
    runtime and everything else the process holds."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    return max(1 << 30, min(free, cap_bytes) - reserve_bytes)


def latency_summary(finished, arrivals, t_stop):
    """p50 / p99 latency over every request that arrived before t_stop: finished ones
    with finish - arrival, unfinished ones censored at t_stop - arrival (so the percentiles
    are lower bounds whenever any request is censored)."""
    lat = [r["t_done"] - r["t_arrival"] for r in finished.values()]
    cens = [t_stop - a for i, a in enumerate(arrivals) if a <= t_stop and i not in finished]
    allv = lat + cens
    return {"latency_p50_s": _percentile(allv, 50), "latency_p99_s": _percentile(allv, 99),
            "latency_censored": len(cens), "latency_is_lower_bound": bool(cens),
            "finished_latency_p50_s": _percentile(lat, 50), "finished_latency_p99_s": _percentile(lat, 99)}


def run_requests(make, arrivals, *, budget_bytes, max_slots=512, max_active_nodes=0, tol=1e-6,
                 drift_tol=1e-5, max_steps=200000, intervals_per_call=1, cache=None, time_limit=None,
                 check_interval=100, log=None, on_start=None):
    """Admit request i (built by make(i) -> (params, mask, walls) when it is first
    considered) at its arrival time (seconds after start) into one batch and run until all
    finish or `time_limit`.  Admission is first come, first served, as the arena, the slots
    and the active-node cap (max_active_nodes, 0 = none) allow.  on_start(batch) is called
    once, after the first admissions and before the first interval (timing hooks).
    Returns summary statistics and per-request records."""
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
    started = False
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
            if not started and on_start is not None:
                extra = on_start(b)
                node_updates += extra
            started = True
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
    solved = [r for r in finished.values() if r["status"] in SOLVED]
    arrived = sum(1 for a in arrivals if a <= wall)
    out = {
        "requests": n_req, "arrived": arrived, "finished": len(finished), "unfinished": arrived - len(finished),
        "converged": sum(r["status"] == AQ_OK for r in finished.values()),
        "accepted_at_floor": sum(r["status"] == AQ_RESULT_FLOOR for r in finished.values()),
        "not_converged": sum(r["status"] == -5 for r in finished.values()),
        "diverged": sum(r["status"] == -4 for r in finished.values()),
        "fallbacks": sum(r["fallback"] for r in finished.values()),
        "wall_s": wall, "solves_per_s": len(solved) / wall if wall > 0 else 0.0,
        "finished_per_s": len(finished) / wall if wall > 0 else 0.0,
        "aggregate_active_mlups": node_updates / wall / 1e6 if wall > 0 else 0.0,
        "records": finished,
    }
    out.update(latency_summary(finished, arrivals, wall))
    return out


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


def stream_arrivals(rate=50.0, duration=60.0, seed0=1000):
    n = int(rate * duration * 1.5) + 10
    return [t for t in poisson_arrivals(n, rate, seed0) if t <= duration]


def serve(rate=50.0, duration=60.0, storage=F16S, tol=1e-6, budget_bytes=None, max_steps=200000,
          seed0=1000, large_every=10, **kw):
    """The Poisson serving stream: request i (sweep draw seed0 + i, every large_every-th a
    2048x1024 eye) arrives at the i-th arrival time.  budget_bytes None: default_budget()."""
    arr = stream_arrivals(rate, duration, seed0)
    if budget_bytes is None:
        budget_bytes = default_budget()
    return run_requests(lambda i: sweep_request(seed0 + i, storage, large_every=large_every), arr,
                        budget_bytes=budget_bytes, tol=tol, max_steps=max_steps, **kw)


def one_at_a_time(make, arrivals, sample, *, tol=1e-6, max_steps=200000, storage=F64, t_stop=None):
    """The plain one-instance path on a stream: each sampled request (indices `sample`)
    solved alone, one after another, in `storage` (the single-lattice solver).  Returns the
    measured service times and the first-come-first-served latencies of the whole stream
    with the sampled service times taken in turn (request i gets sample i mod n), censored
    at t_stop like the batched loop's."""
    svc, solved = [], 0
    for i in sample:
        p, mask, walls = make(i)
        p = A.Params(**{**p.asdict(), "storage": storage})
        t0 = time.perf_counter()
        s = Solver(p, mask, walls)
        ok, _ = s.run_to_steady(tol, max_steps)
        s.close()
        svc.append(time.perf_counter() - t0)
        solved += int(ok)
    finished, t_free = {}, 0.0
    for i, a in enumerate(arrivals):
        start = max(a, t_free)
        t_free = start + svc[i % len(svc)]
        if t_stop is None or t_free <= t_stop:
            finished[i] = {"t_done": t_free, "t_arrival": a}
    stop = t_stop if t_stop is not None else t_free
    out = {"sampled": len(sample), "sampled_solved": solved, "service_s_mean": float(np.mean(svc)),
           "service_s": [round(v, 3) for v in svc], "solves_per_s": len(svc) / float(np.sum(svc)),
           "finished_by_stop": len(finished)}
    out.update(latency_summary(finished, arrivals, stop))
    return out


def thickness_update(h, rise, target, history):
    """Next meshwork thickness: a secant step on (h, rise) pairs; the first step is
    proportional (the steady rise IOP - p_sc of the lumped meshwork scales with h)."""
    history.append((h, rise))
    if len(history) >= 2:
        (h0, r0), (h1, r1) = history[-2], history[-1]
        if r1 != r0:
            return h1 + (target - r1) * (h1 - h0) / (r1 - r0)
    return h * target / rise


def calibrate(eyes, targets, *, tol=1e-9, iop_rtol=1e-6, max_rounds=8, max_steps=400000,
              budget_bytes=8 << 30, max_slots=64, intervals_per_call=5, check_interval=100, warm=True):
    """Calibrate the meshwork thickness of every eye (params, mask, walls with the lumped
    outlet) so that its steady IOP - p_sc is targets[i].  All eyes share one batch.  With
    warm=False every round starts a fresh solve from the initial state instead (the cold
    baseline).  Returns per-eye records (thickness per round, steps, rounds) and
    throughput figures."""
    b = Batch(budget_bytes=budget_bytes, max_slots=max_slots, max_tiles=1 << 21, check_interval=check_interval)
    n = len(eyes)
    pending = list(range(n))
    slot_of, rec = {}, {}
    t0 = time.perf_counter()
    done = 0
    while done < n:
        while pending:
            i = pending[0]
            p, mask, walls = eyes[i]
            sl = b.admit(p, mask, walls, tile=(64, 4), tol=tol, max_steps=max_steps, request_id=i, keep=True)
            if sl is None:
                break
            pending.pop(0)
            slot_of[i] = sl
            rec[i] = {"h": [p.h_tm], "rise": [], "steps": 0, "rounds": 0, "status": AQ_OK,
                      "t_admit": time.perf_counter() - t0, "history": []}
        if b.info()["running"] == 0 and not pending:
            break
        b.run(intervals_per_call)
        for r in b.poll():
            i = r["request_id"]
            p = eyes[i][0]
            e = rec[i]
            e["rounds"] += 1
            e["steps"] = r["steps"] + e.get("steps_before", 0)
            rise = r["obs"]["p_mean_fluid"] - p.p_sc
            e["rise"].append(rise)
            ok = r["status"] == AQ_OK and abs(rise / targets[i] - 1.0) <= iop_rtol
            if ok or r["status"] != AQ_OK or e["rounds"] >= max_rounds:
                e["status"] = r["status"] if r["status"] != AQ_OK else (AQ_OK if ok else -5)
                e["t_done"] = time.perf_counter() - t0
                b.release(slot_of[i])
                done += 1
                continue
            h_new = thickness_update(e["h"][-1], rise, targets[i], e["history"])
            e["h"].append(h_new)
            if warm:
                b.set_outlet(slot_of[i], p.K_tm, h_new, p.p_sc)
                if not b.resume(slot_of[i], tol, max_steps):
                    raise RuntimeError("no room to resume a resident instance")
            else:
                b.release(slot_of[i])
                e["steps_before"] = e.get("steps_before", 0) + r["steps"]
                p2 = A.Params(**{**p.asdict(), "h_tm": h_new})
                sl = b.admit(p2, eyes[i][1], eyes[i][2], tile=(64, 4), tol=tol, max_steps=max_steps,
                             request_id=i, keep=True)
                if sl is None:
                    raise RuntimeError("no room to restart the instance")
                slot_of[i] = sl
    wall = time.perf_counter() - t0
    b.close()
    for e in rec.values():
        e.pop("history")
        e.pop("steps_before", None)
    lat = [e["t_done"] - e["t_admit"] for e in rec.values() if "t_done" in e]
    return {"eyes": n, "calibrated": sum(e["status"] == AQ_OK for e in rec.values()),
            "wall_s": wall, "calibrations_per_s": n / wall if wall > 0 else 0.0,
            "rounds_mean": float(np.mean([e["rounds"] for e in rec.values()])),
            "steps_mean": float(np.mean([e["steps"] for e in rec.values()])),
            "latency_p50_s": _percentile(lat, 50), "latency_p99_s": _percentile(lat, 99), "records": rec}
