"""Benchmark of the fused collide-and-stream hot path on one MI355X.

Headline workload: the batched parameter sweep of 512 eye sections (lattices 256x128 to
1024x512, per-instance relaxation time, permeability, inflow, chamber angle, Rayleigh
number and gravity orientation, all seeded), FP32 populations, resident in one batch.  One
benchmark step = one check interval of every instance: 96 time steps as 48 two-step
launches (an even number: the batch keeps every instance's buffer parity), three single
steps and the reducing step (IOP, fluxes, wall shear stress, residuals).  The timed steps are taken inside the full sweep, which then continues until
every instance has reached its steady residual of 1e-6 (solves/s, p50/p99 latency).

Further fields: the 8192x4096 eye in FP64 (active and lattice MLUPS), a plain device copy's
bandwidth, the dense 8192x4096 box (every interior node active) in FP64, FP32 and F16S, the
8192x4096 precision sweep, the 2048x1024 eye per storage, the Poisson serving stream with the
one-at-a-time FP64 path beside it, and the oracle on the host cores.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (flow+thermal) & HBM-roofline %; batched solves/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
STORAGES = {"f64": 0, "f32": 1, "f16s": 2, "f32x": 3}
# algorithmic HBM bytes per active node and launch: one read and one write of the 13 live
# populations plus the type byte, whether the launch advances one time step or two (the
# two-step kernel keeps the intermediate step in LDS)
BYTES_PER_NODE_LAUNCH = {"f64": 209, "f32": 105, "f16s": 53, "f32x": 105}
DTYPE = {"f64": "f64", "f32": "f32", "f16s": "f16 storage / f32 compute", "f32x": "f32 storage / f64 compute"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("aq_kernels.hip", "aq_device.h"):
        with open(os.path.join(ROOT, "paper_2102_12663_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_entry(key, kernel):
    """The committed rocprofv3 summary of a kernel (HBM bytes per launch, VALU figures), if
    it was taken on the current kernel source and the same kernel; else None."""
    path = os.path.join(ROOT, "profiles", "kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(key)
    if not e or e.get("kernel_hash") != kernel_source_hash() or not kernel.startswith(e.get("kernel", "?")):
        return None
    return e


def measured_traffic(key, kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source and the same kernel; else None."""
    e = measured_entry(key, kernel)
    return e.get("bytes_per_launch") if e else None


def roofline(key, kernel, storage, active_nodes, launch_ms):
    """Roofline of a launch that moves every population of `active_nodes` nodes once in and
    once out (single step or two steps): algorithmic bytes over the live launch time, and
    beside it the bytes the HBM counters saw (when committed for this kernel source)."""
    bpl = BYTES_PER_NODE_LAUNCH[storage] * active_nodes
    achieved = bpl / (launch_ms * 1e-3) / 1e9
    e = measured_entry(key, kernel)
    traffic = e.get("bytes_per_launch") if e else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "kernel_ms": round(launch_ms, 5), "bytes_per_launch": bpl,
            "bytes_per_active_node_launch": BYTES_PER_NODE_LAUNCH[storage],
            "counter_GBs": round(traffic / (launch_ms * 1e-3) / 1e9, 1) if traffic else None,
            # from the same committed profile: VALU wave instructions per busy CU cycle (1.0 =
            # the four 16-lane SIMDs' issue limit) and per wave
            "valu_issue": e.get("valu_issue") if e else None,
            "valu_per_wave": e.get("valu_per_wave") if e else None}


# ---------------------------------------------------------------------------------- oracle
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_inst=8, budget_s=2.5):
    """The oracle, as it stands, on the host cores, on a bounded sample of the headline
    workload: the first n_inst requests of the sweep (two per lattice size), each stepped
    for the same number of time steps, at all OpenMP threads and at one thread, median of
    three timed runs after one warm-up step.  Active-node MLUPS."""
    import numpy as np
    import aqinputs as A
    import oracle as O
    from paper_2102_12663_amd import serve as S
    reqs = [S.sweep_request(i, 0) for i in range(n_inst)]
    act = sum(int(A.active(m).sum()) for _, m, _ in reqs)
    all_threads = O.max_threads()
    out = {}
    for threads in (all_threads, 1):
        O.set_threads(threads)
        orcs = [O.Oracle(p, m, w) for p, m, w in reqs]
        for o in orcs:
            o.step(1)                                  # first touch
        t0 = time.perf_counter()
        for o in orcs:
            o.step(1)
        per_step = time.perf_counter() - t0
        n = max(1, int(budget_s / max(per_step, 1e-6)))
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            for o in orcs:
                o.step(n)
            runs.append(act * n / (time.perf_counter() - t0) / 1e6)
        out[threads] = (float(np.median(runs)), n)
        del orcs
    O.set_threads(all_threads)
    v_all, n_all = out[all_threads]
    v_one, n_one = out[1]
    sizes = sorted({f"{p.nx}x{p.ny}" for p, _, _ in reqs})
    return {"value": round(v_all, 2), "unit": "MLUPS", "cores": all_threads, "kind": "oracle",
            "sample": f"the first {n_inst} requests of the 512-instance sweep ({', '.join(sizes)}; {act} active "
                      f"nodes), {n_all} time steps each at {all_threads} threads and {n_one} at 1 thread; "
                      f"median of 3 runs",
            "single_thread": round(v_one, 2), "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "other_samples": other_oracle_samples()}


def other_oracle_samples():
    """The oracle at all threads on the two single-lattice FP64 workloads: the 192x96 eye
    (all 5,000 time steps of its run) and the 8192x4096 eye (sweep draw seed 0; 5 time
    steps of it).  Active-node MLUPS, median of 3 runs after one warm-up step."""
    import numpy as np
    import aqinputs as A
    import oracle as O
    out = {}
    for name, make, steps in (("eye192x96_f64", A.config0, 5000),
                              ("eye8192x4096_f64", lambda: A.sweep_instance(0, 8192, 4096), 5)):
        p, mask, walls, _ = make()
        act = int(A.active(mask).sum())
        o = O.Oracle(p, mask, walls)
        o.step(1)
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            o.step(steps)
            runs.append(act * steps / (time.perf_counter() - t0) / 1e6)
        del o
        out[name] = {"mlups": round(float(np.median(runs)), 2), "active_nodes": act, "time_steps": steps,
                     "threads": O.max_threads()}
    return out


# ------------------------------------------------------------------------- headline: sweep
def sweep512(steps, warmup, n=512, tol=1e-6, max_steps=200000, time_limit=240.0, storage="f32"):
    """The batched sweep (all n requests submitted at t = 0, FP32, residual tol, at most
    max_steps time steps each, tile shapes of the single steps from the autotuner): the
    first `warmup` intervals untimed, then `steps` intervals timed with HIP events around
    their two-step launches (the headline throughput and roofline), then the run continues
    until every solve has finished (or time_limit).  The clock of the latencies starts
    when the batch is complete, after the synthetic inputs have been built."""
    import torch
    import aqinputs as A
    import paper_2102_12663_amd as aq
    from paper_2102_12663_amd import serve as S
    t_build = time.perf_counter()
    reqs = [S.sweep_request(i, STORAGES[storage]) for i in range(n)]
    act_all = sum(int(A.active(m).sum()) for _, m, _ in reqs)
    log(f"sweep: {n} requests built in {time.perf_counter() - t_build:.1f} s, {act_all} active nodes")
    timed = {}

    def on_start(b):
        b.run(warmup)
        torch.cuda.synchronize()
        info = b.info()
        t0 = time.perf_counter()
        total_ms, fused_ms, n_fused = b.run_timed(steps)
        wall = time.perf_counter() - t0
        timed.update(info=info, wall=wall, total_ms=total_ms, fused_ms=fused_ms, n_fused=n_fused)
        log(f"sweep: timed {steps} intervals, {info['active_nodes']} active nodes, {wall:.3f} s")
        return info["active_nodes"] * (warmup + steps) * 100

    shapes = {}
    cache = S.ShapeCache()

    def make(i):
        p, m, w = reqs[i]
        shapes[(p.nx, p.ny)] = None
        return p, m, w

    r = S.run_requests(make, [0.0] * n, budget_bytes=S.default_budget(), max_slots=n, tol=tol,
                       max_steps=max_steps, intervals_per_call=5, cache=cache, time_limit=time_limit,
                       on_start=on_start)
    r.pop("records")
    info = timed["info"]
    act = info["active_nodes"]
    mlups = act * steps * 100 / timed["wall"] / 1e6
    launch_ms = timed["fused_ms"] / timed["n_fused"]
    kernel = (f"batch_step2_kernel<{STORAGES[storage]}, {'true' if info['active_nodes'] * 105 > 192 * 2 ** 20 else 'false'}, "
              f"false, {info['fused_tile_rows'][STORAGES[storage]]}>")
    tiles = {k[len("gfx950/1/"):]: "x".join(map(str, v)) for k, v in cache.d.items()}
    return {"mlups": mlups, "wall": timed["wall"], "active_nodes": act, "running": info["running"],
            "roofline": roofline(f"sweep512/{storage}", kernel, storage, act, launch_ms),
            "tiles": tiles, "solve": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()},
            "active_nodes_all": act_all}


# ------------------------------------------------------------------------- other workloads
def eye_run(storage, nx, ny, seed, steps, warmup, tm="resolved", bc=0, tile=(64, 4)):
    """One eye lattice: `steps` check intervals timed after `warmup`, with HIP events around
    the graph part of each interval (two-step launches when fusion is on)."""
    import torch
    import aqinputs as A
    import paper_2102_12663_amd as aq
    p, mask, walls, geo = A.sweep_instance(seed, nx, ny, storage=STORAGES[storage], tm=tm)
    p.bc_scheme = bc
    s = aq.Solver(p, mask, walls)
    s.set_tile(*tile)
    info = s.info()
    D = info["check_interval"]
    if warmup:
        s.run_intervals_timed(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_ms, plain_ms = s.run_intervals_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ob = s.observe()
    s.close()
    act = info["active_nodes"]
    launch_ms = plain_ms / (steps * info["graph_launches"])
    nt = "true" if info["nt_store"] else "false"
    bcs = "true" if bc else "false"
    kernel = (f"step2_kernel<{STORAGES[storage]}, {nt}, {bcs}, {info['fused_tile_rows']}>" if info["fusion"]
              else f"step_kernel<{STORAGES[storage]}, false, {nt}, {bcs}>")
    return {"mlups": act * steps * D / wall / 1e6, "wall": wall, "active_nodes": act, "launch_ms": launch_ms,
            "kernel": kernel, "steps_per_launch": 2 if info["fusion"] else 1, "obs": ob, "geo": geo, "p": p}


def brief(e, storage, key):
    r = roofline(key, e["kernel"], storage, e["active_nodes"], e["launch_ms"])
    return {"mlups": round(e["mlups"], 1), "kernel": e["kernel"], "time_steps_per_launch": e["steps_per_launch"],
            "kernel_ms": r["kernel_ms"], "achieved_GBs": r["achieved"], "frac": r["frac"], "traffic": r["traffic"]}


def precision_sweep(steps=20000, nx=8192, ny=4096, seed=0):
    """The 8192x4096 eye (sweep draw seed 0) for `steps` time steps in each storage, from
    the same initial state: active MLUPS, and the IOP and velocity errors of FP32, F16S and
    F32X storage against the FP64 run on the GPU (velocity: L2 over active nodes, relative).
    A transient: the slowest mode of this chamber needs ~1e7 steps."""
    import numpy as np
    import aqinputs as A
    import paper_2102_12663_amd as aq
    out = {"workload": f"{nx}x{ny} eye section (sweep draw seed {seed}), {steps} time steps per storage"}
    ref = None
    p0, mask, walls, geo = A.sweep_instance(seed, nx, ny)
    on = A.active(mask)
    for st in ("f64", "f32", "f16s", "f32x"):
        p = A.Params(**{**p0.asdict(), "storage": STORAGES[st]})
        s = aq.Solver(p, mask, walls)
        D = s.info()["check_interval"]
        t0 = time.perf_counter()
        s.run_intervals_timed(steps // D)
        wall = time.perf_counter() - t0
        act = s.info()["active_nodes"]
        ob = s.observe()
        ux, uy = s.read_field("ux"), s.read_field("uy")
        s.close()
        e = {"mlups": round(act * steps / wall / 1e6, 1), "iop_gauge": ob["iop_gauge"]}
        if ref is None:
            ref = (ob["iop_gauge"], ux[on], uy[on])
        else:
            du = np.sqrt(np.sum((ux[on] - ref[1]) ** 2 + (uy[on] - ref[2]) ** 2))
            e["velocity_l2_rel"] = float(du / np.sqrt(np.sum(ref[1] ** 2 + ref[2] ** 2)))
            e["iop_rel"] = abs(ob["iop_gauge"] - ref[0]) / abs(ref[0])
        out[st] = e
    return out


def precision_steady(cases=((512, 256, 3), (512, 256, 5), (1024, 512, 6), (2048, 1024, 3)), tol=1e-9):
    """The reduced-precision forms against FP64 at steady states: each sweep draw runs in FP64
    to a residual of `tol`; FP32, F16S and F32X storage then run the same number of steps from the
    same initial state.  Velocity L2 error relative to FP64 over active nodes, IOP relative
    error, max |T| error and the reduced form's own final residual."""
    import numpy as np
    import aqinputs as A
    import paper_2102_12663_amd as aq
    out = []
    for nx, ny, seed in cases:
        p0, mask, walls, geo = A.sweep_instance(seed, nx, ny)
        act = A.active(mask)
        s = aq.Solver(p0, mask, walls)
        ok, ob64 = s.run_to_steady(tol, 4_000_000)
        f64 = s.fields()
        s.close()
        den = np.sqrt(np.sum(f64[1][act] ** 2 + f64[2][act] ** 2))
        row = {"case": f"{nx}x{ny} seed {seed}", "fp64_steps": ob64["step"], "fp64_converged": bool(ok)}
        for st in ("f32", "f16s", "f32x"):
            s = aq.Solver(A.Params(**{**p0.asdict(), "storage": STORAGES[st]}), mask, walls)
            s.step(ob64["step"])
            ob, f = s.observe(), s.fields()
            s.close()
            du = np.sqrt(np.sum((f[1][act] - f64[1][act]) ** 2 + (f[2][act] - f64[2][act]) ** 2))
            row[st] = {"velocity_l2_rel": float(du / den),
                       "iop_rel": abs(ob["iop_gauge"] - ob64["iop_gauge"]) / abs(ob64["iop_gauge"]),
                       "t_max_err": float(np.max(np.abs(f[3][act] - f64[3][act]))), "resid_u": ob["resid_u"]}
        out.append(row)
    return out


def config1_steady(seed=0, nx=2048, ny=1024):
    """The 2048x1024 eye run to its steady state as the workload states it: FP64 to a
    residual of 1e-8 and FP32 to 1e-6, each on its own; IOP, cornea and iris mean / max wall
    shear stress (section 3.6), and the velocity L2 of the FP32 state against FP64."""
    import numpy as np
    import aqinputs as A
    import paper_2102_12663_amd as aq
    p0, mask, walls, geo = A.sweep_instance(seed, nx, ny)
    act = A.active(mask)
    out = {"workload": f"{nx}x{ny} eye (sweep draw seed {seed}), FP64 to 1e-8, FP32 to 1e-6"}
    f64 = None
    keys = ("iop_gauge", "wss_cornea_mean", "wss_cornea_max", "wss_iris_mean", "wss_iris_max", "u_max")
    for st, tol in (("f64", 1e-8), ("f32", 1e-6)):
        s = aq.Solver(A.Params(**{**p0.asdict(), "storage": STORAGES[st]}), mask, walls)
        t0 = time.perf_counter()
        ok, ob = s.run_to_steady(tol, 6_000_000)
        wall = time.perf_counter() - t0
        f = s.fields()
        s.close()
        e = {"converged": bool(ok), "steps": ob["step"], "seconds": round(wall, 2), **{k: ob[k] for k in keys}}
        if f64 is None:
            f64 = (f, ob)
        else:
            den = np.sqrt(np.sum(f64[0][1][act] ** 2 + f64[0][2][act] ** 2))
            e["velocity_l2_rel"] = float(np.sqrt(np.sum((f[1][act] - f64[0][1][act]) ** 2 +
                                                       (f[2][act] - f64[0][2][act]) ** 2)) / den)
            for k in keys:
                e[k + "_rel"] = abs(ob[k] - f64[1][k]) / abs(f64[1][k])
        out[st] = e
    return out


def serve_stream(rate=50.0, duration=60.0, time_limit=150.0, storage="f16s", max_active_nodes=16_000_000,
                 n_sample=20, sample_steps=200000):
    """The serving stream (Poisson arrivals, every 10th request a 2048x1024 eye, residual
    1e-6, F16S with the IOP drift check and the F32 hand-off), the arena sized to the free
    HBM, admission capped at max_active_nodes running active nodes, stopped at time_limit
    seconds; beside it the one-at-a-time FP64 path on the same stream from n_sample
    requests solved alone (spread over the stream and over its mix: request i is a
    2048x1024 eye when i % 10 == 9, and the sample walks the residues 0..9)."""
    from paper_2102_12663_amd import serve as S
    import paper_2102_12663_amd as aq
    done = [0]

    def progress(r):
        done[0] += 1
        if done[0] % 50 == 1:
            log(f"serve: {done[0]} finished, {r['t_done']:.0f} s")

    r = S.serve(rate=rate, duration=duration, storage=STORAGES[storage], tol=1e-6, max_steps=sample_steps,
                intervals_per_call=5, time_limit=time_limit, max_active_nodes=max_active_nodes, log=progress)
    r.pop("records")
    arr = S.stream_arrivals(rate, duration)
    stride = max(10, len(arr) // n_sample // 10 * 10)
    sample = [min(len(arr) - 1, j * stride + j % 10) for j in range(n_sample)]
    log(f"serve: one-at-a-time FP64 on {len(sample)} sampled requests")
    base = S.one_at_a_time(lambda i: S.sweep_request(1000 + i, aq.F64, large_every=10), arr, sample,
                           tol=1e-6, max_steps=sample_steps, storage=aq.F64, t_stop=time_limit)
    form = "F16S with the FP32 hand-off" if storage == "f16s" else storage.upper()
    out = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}
    out["workload"] = (f"Poisson stream of sweep requests, {rate:g}/s for {duration:g} s (every 10th 2048x1024), "
                       f"{form}, residual 1e-6, cap {sample_steps} steps, at most {max_active_nodes} active nodes "
                       f"running, stopped at {time_limit:g} s")
    out["one_at_a_time_f64"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in base.items()}
    return out


def aq_copy_GBs():
    import paper_2102_12663_amd as aq
    return aq.copy_bandwidth(1 << 30, 5)


def dense_box(storages, intervals=10, nx=8192, ny=4096):
    """An 8192x4096 closed box, every interior node active (heated floor, cooled lid,
    buoyancy on), per storage: active MLUPS and the roofline of the graph-part launches."""
    import aqinputs as A
    import paper_2102_12663_amd as aq
    mask = A.box_mask(nx, ny, wall_ids=(A.WALL_IRIS, A.WALL_CORNEA, A.WALL_BOX, A.WALL_BOX))
    out = {"workload": f"{nx}x{ny} closed box, {(nx - 2) * (ny - 2)} active nodes, heated floor, "
                       f"{intervals} check intervals of 100 time steps"}
    for st in storages:
        p = A.Params(nx=nx, ny=ny, gbeta=1e-6, storage=STORAGES[st], check_interval=100)
        s = aq.Solver(p, mask, A.no_walls())
        s.run_intervals_timed(1)
        t0 = time.perf_counter()
        total_ms, plain_ms = s.run_intervals_timed(intervals)
        wall = time.perf_counter() - t0
        info = s.info()
        s.close()
        act = info["active_nodes"]
        launch_ms = plain_ms / (intervals * info["graph_launches"])
        r = roofline(f"box{nx}x{ny}/{st}", "?", st, act, launch_ms)
        out[st] = {"mlups": round(act * intervals * 100 / wall / 1e6, 1), "kernel_ms": r["kernel_ms"],
                   "time_steps_per_launch": 2 if info["fusion"] else 1, "achieved_GBs": r["achieved"],
                   "frac": r["frac"]}
    return out


def outflow_area(mask):
    """Outflow area of a lumped-meshwork mask: sum over links from active nodes into OUTLET
    nodes of 6 w_i (e_i . n), n the node's outward direction (mask bits 3-4)."""
    import numpy as np
    import aqinputs as A
    e = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    act = A.active(mask)
    cls, d = mask & 7, (mask >> 3) & 3
    area = 0.0
    for i in range(1, 9):
        ex, ey = e[i]
        nb_cls = np.roll(np.roll(cls, -ey, axis=0), -ex, axis=1)
        nb_d = np.roll(np.roll(d, -ey, axis=0), -ex, axis=1)
        hit = act & (nb_cls == A.OUTLET)
        for k in range(4):
            nx_, ny_ = e[k + 1]
            area += 6 * w[i] * (ex * nx_ + ey * ny_) * np.count_nonzero(hit & (nb_d == k))
    return area


def calibration_workload(n=12, cap=400000):
    """Section 3.1's thickness calibration for n lumped-outlet eyes (sweep draws 256x128 and
    512x256, meshwork permeability set so the coupling contracts by 0.6 per interval):
    target IOP rise 1.25x that of the initial thickness; warm restarts of the resident
    solves against fresh restarts every round."""
    import aqinputs as A
    from paper_2102_12663_amd import serve as S
    eyes, targets = [], []
    for i in range(n):
        nx, ny = ((256, 128), (512, 256))[i % 2]
        p, mask, walls, geo = A.sweep_instance(100 + i, nx, ny, tm="lumped")
        p.gbeta = 0.0                      # Ra = 0: the secretion-driven steady state
        nu = (2 * p.tau_f - 1) / 6
        area = outflow_area(mask)
        p.K_tm = 0.4 * 5 * int(A.active(mask).sum()) * nu * p.h_tm / (3 * area * p.check_interval)
        q_in = p.u_in_y * (geo.inlet_cols[1] - geo.inlet_cols[0] + 1)
        targets.append(1.25 * nu * p.h_tm * q_in / (p.K_tm * area))
        eyes.append((p, mask, walls))
    out = {"workload": f"{n} lumped-outlet eyes (sweep draws 100..{99 + n}, 256x128 and 512x256, Ra = 0), "
                       f"target IOP rise 1.25x the initial thickness's, residual 1e-9, IOP to 1e-6"}
    for warm in (True, False):
        r = S.calibrate(eyes, targets, tol=1e-9, iop_rtol=1e-6, max_steps=cap, warm=warm)
        out["warm" if warm else "cold"] = {
            "calibrated": r["calibrated"], "calibrations_per_s": round(r["calibrations_per_s"], 3),
            "rounds_mean": round(r["rounds_mean"], 2), "steps_mean": round(r["steps_mean"]),
            "p50_s": round(r["latency_p50_s"], 3), "p99_s": round(r["latency_p99_s"], 3)}
    return out


def probe(kind, storage):
    """Short program for hardware-counter runs: a few launches of one workload's dominant
    kernel, then three device copies of 256 MiB (a copy kernel of known size, the
    calibration of the byte counters)."""
    import torch
    import aqinputs as A
    import paper_2102_12663_amd as aq
    from paper_2102_12663_amd import serve as S
    if kind == "sweep512":
        reqs = [S.sweep_request(i, STORAGES[storage]) for i in range(512)]
        b = aq.Batch(budget_bytes=S.default_budget(), max_slots=512, max_tiles=1 << 21)
        cache = S.ShapeCache()
        for p, m, w in reqs:
            b.admit(p, m, w, tile=S.autotune_shape(cache, p, m, w), tol=1e-30, max_steps=10 ** 9)
        b.run(1)
        act = b.info()["active_nodes"]
        b.close()
    else:
        nx, ny = (int(v) for v in kind[3:].split("x"))
        p, mask, walls, geo = A.sweep_instance(0, nx, ny, storage=STORAGES[storage])
        s = aq.Solver(p, mask, walls)
        if s.info()["fusion"]:
            s.time_fused_kernel(10)
        else:
            s.time_step_kernel(10)
        act = s.info()["active_nodes"]
        s.close()
    x = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"probe": f"{kind}/{storage}", "active_nodes": act, "kernel_hash": kernel_source_hash(),
                      "copy_bytes": 256 << 20}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed check intervals of the 512-instance batch")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="only the headline (the batch throughput)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--extra", action="store_true",
                    help="also the dense 8192x4096 box in F32X, the lumped-outlet and paper-boundary variants "
                         "of the 2048x1024 eye and the thickness calibration")
    ap.add_argument("--precision-steady", action="store_true",
                    help="only the steady-state precision comparison of FP32, F16S and F32X against FP64")
    ap.add_argument("--config1-steady", action="store_true",
                    help="only the 2048x1024 steady state (FP64 to 1e-8, FP32 to 1e-6) with IOP and WSS")
    ap.add_argument("--serve", action="store_true", help="only the serving stream")
    ap.add_argument("--probe", default=None, metavar="KIND",
                    help="hardware-counter program: 'sweep512' or 'eyeNXxNY' (with --storage)")
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGES))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): every workload here fits one "
              "MI355X, and the multi-GPU decomposition is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.probe:
        probe(args.probe, args.storage)
        return
    if args.precision_steady:
        print(json.dumps({"precision_steady": precision_steady()}), flush=True)
        return
    if args.config1_steady:
        print(json.dumps({"config1_steady": config1_steady()}), flush=True)
        return
    if args.serve:
        print(json.dumps({"serve": serve_stream()}), flush=True)
        return

    t_start = time.perf_counter()
    sw = sweep512(args.steps, args.warmup, time_limit=20.0 if args.quick else 240.0)
    log(f"sweep done at {time.perf_counter() - t_start:.0f} s")
    solve = sw["solve"]
    out = {
        "metric": METRIC,
        "value": round(sw["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sw["wall"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched parameter sweep: 512 synthetic eye sections (seeds 0..511, lattices "
                               f"256x128 to 1024x512, per-instance tau, Da, inflow, chamber angle, Ra and gravity "
                               f"orientation) resident in one batch, f32 populations; one step = one check interval "
                               f"(100 time steps incl. the reducing step) of every instance",
                   "instances": sw["running"], "active_nodes": sw["active_nodes"], "time_steps_per_step": 100,
                   "storage": "f32", "single_step_tiles": sw["tiles"], "parallelism": "single GPU"},
        "roofline": sw["roofline"],
        "sweep512": {"workload": "the same 512 requests, each to a steady residual of 1e-6 (cap 200000 steps), "
                                 "all submitted at t = 0, continuously batched",
                     "solves_per_s": solve["solves_per_s"], "finished_per_s": solve["finished_per_s"],
                     "p50_s": solve["latency_p50_s"], "p99_s": solve["latency_p99_s"],
                     "latency_is_lower_bound": solve["latency_is_lower_bound"],
                     "converged": solve["converged"], "not_converged": solve["not_converged"],
                     "diverged": solve["diverged"], "unfinished": solve["unfinished"], "wall_s": solve["wall_s"],
                     "aggregate_active_mlups": solve["aggregate_active_mlups"]},
    }
    if not args.quick:
        log("fp64 8192x4096")
        e = eye_run("f64", 8192, 4096, 0, 10, 2)
        r = roofline("eye8192x4096s0/f64", e["kernel"], "f64", e["active_nodes"], e["launch_ms"])
        out["fp64_8192x4096"] = {"workload": "8192x4096 eye section (sweep draw seed 0), f64, 10 check intervals",
                                 "mlups": round(e["mlups"], 1), "active_nodes": e["active_nodes"],
                                 "lattice_mlups": round(e["mlups"] * 8192 * 4096 / e["active_nodes"], 1),
                                 "roofline": r}
        log("copy bandwidth")
        out["copy_kernel"] = {"GBs": round(aq_copy_GBs(), 1), "bytes": 1 << 30,
                              "kernel": "copy_kernel: 16-byte words, non-temporal stores, grid-stride, 2048 blocks of 256; "
                                        "(read + written bytes) / time, best of 5 after one warm-up"}
        log("dense box")
        out["dense_box"] = dense_box(("f64", "f32", "f16s"))
        log("2048x1024 per storage")
        out["eye2048x1024"] = {st: brief(eye_run(st, 2048, 1024, 0, 20, 2), st, f"eye2048x1024s0/{st}")
                               for st in ("f64", "f32", "f16s", "f32x")}
        log("precision sweep")
        out["precision_sweep"] = precision_sweep()
        if not args.no_serve:
            log("serving stream")
            out["serve"] = serve_stream()
        if args.extra:
            out["dense_box_f32x"] = dense_box(("f32x",))
            e = eye_run("f64", 2048, 1024, 0, 20, 2, tm="lumped")
            out["lumped_outlet"] = {**brief(e, "f64", "eye2048x1024s0/f64-lumped"), "iop_gauge": e["obs"]["iop_gauge"],
                                    "u_seep": e["obs"]["u_seep"]}
            e = eye_run("f64", 2048, 1024, 0, 20, 2, bc=1)
            out["paper_boundaries"] = {**brief(e, "f64", "eye2048x1024s0/f64-paper"), "iop_gauge": e["obs"]["iop_gauge"]}
            out["calibration"] = calibration_workload()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline()
    out["bench_seconds"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
