"""Batched serving form: continuous batching of uneven solves in one multi-instance kernel.

Each instance must compute exactly what it computes alone (fields and observables bitwise
equal for the same tile shape); admission respects memory, slots and the active-node cap;
a failing instance is retired without disturbing the others."""
import numpy as np
import pytest

import aqinputs as A
import oracle as O
from gpu_util import announce, field_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    return aq


def _instances():
    """Uneven sizes, storages, angles, orientations (the batched sweep's draws)."""
    out = []
    for seed, (nx, ny), st in ((3, (256, 128), A.F32), (5, (512, 256), A.F64), (6, (256, 128), A.F16S),
                                (7, (384, 192), A.F32), (9, (320, 160), A.F64), (11, (320, 160), A.F32X)):
        p, mask, walls, geo = A.sweep_instance(seed, nx, ny, tau_f="draw", phi_deg="draw", storage=st)
        out.append((p, mask, walls))
    return out


def _fields_equal(a, b):
    return all(np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0)) for x, y in zip(a, b))


def test_alone_vs_in_the_mix_bitwise(aq):
    insts = _instances()
    b = aq.Batch(budget_bytes=1 << 30, max_slots=16)
    slots = [b.admit(p, m, w, tile=(64, 4), tol=1e-12, max_steps=10 ** 6, request_id=i, keep=True)
             for i, (p, m, w) in enumerate(insts)]
    assert all(s is not None for s in slots)
    b.run(7)
    for i, (p, m, w) in enumerate(insts):
        announce(f"[batch] instance {i} {p.nx}x{p.ny} storage {p.storage}")
        alone = aq.Solver(p, m, w)
        alone.set_tile(64, 4)
        alone.step(700)
        mixed = [b.read_field(slots[i], f) for f in ("p", "ux", "uy", "T")]
        solo = [alone.read_field(f) for f in ("p", "ux", "uy", "T")]
        assert _fields_equal(mixed, solo), f"instance {i}"
        assert b.observe(slots[i]) == alone.observe()
        alone.close()
    b.close()


def test_fused_tile_rows_bitwise(aq):
    """The batch's two-step tiles: a small batch takes 64 x 4 in its F32 and F16S classes
    (FP64 and F32X keep 64 x 8), and the fields are bitwise the same as with 64 x 8
    throughout, or with the height switched between intervals."""
    insts = _instances()
    runs = {}
    for name, plan in (("auto", (0, 0)), ("eight", (8, 8)), ("switch", (4, 8))):
        b = aq.Batch(budget_bytes=1 << 30, max_slots=16)
        slots = [b.admit(p, m, w, tile=(64, 4), tol=1e-12, max_steps=10 ** 6, request_id=i, keep=True)
                 for i, (p, m, w) in enumerate(insts)]
        b.set_fused_tile_rows(plan[0])
        rows_first = b.info()["fused_tile_rows"]
        b.run(3)
        b.set_fused_tile_rows(plan[1])
        b.run(4)
        announce(f"[batch] fused rows {name}: {rows_first} then {b.info()['fused_tile_rows']}")
        runs[name] = (rows_first, [[b.read_field(sl, f) for f in ("p", "ux", "uy", "T")] for sl in slots])
        b.close()
    assert runs["auto"][0] == [8, 4, 4, 8]
    assert runs["eight"][0] == [8, 8, 8, 8]
    assert runs["switch"][0] == [8, 4, 4, 8]
    for i in range(len(insts)):
        assert _fields_equal(runs["auto"][1][i], runs["eight"][1][i]), f"instance {i}"
        assert _fields_equal(runs["switch"][1][i], runs["eight"][1][i]), f"instance {i}"


def test_staggered_admission_and_retirement_bitwise(aq):
    """Work lists that grow and shrink between runs (each change re-sizes the launches):
    an instance admitted late and one that keeps running after another retires both match
    their solo runs bitwise."""
    insts = _instances()
    b = aq.Batch(budget_bytes=1 << 30, max_slots=16)
    first = b.admit(*insts[0], tile=(64, 4), tol=1e-12, max_steps=10 ** 6, keep=True)
    short = b.admit(*insts[3], tile=(64, 4), tol=1e-12, max_steps=200, request_id=7)
    b.run(3)                                      # `short` retires at its step cap
    assert [r["request_id"] for r in b.poll()] == [7]
    late = b.admit(*insts[2], tile=(64, 4), tol=1e-12, max_steps=10 ** 6, keep=True)
    late2 = b.admit(*insts[1], tile=(64, 4), tol=1e-12, max_steps=10 ** 6, keep=True)
    b.run(4)
    for sl, (p, m, w), steps in ((first, insts[0], 700), (late, insts[2], 400), (late2, insts[1], 400)):
        announce(f"[batch] staggered {p.nx}x{p.ny} storage {p.storage} after {steps} steps")
        alone = aq.Solver(p, m, w)
        alone.set_tile(64, 4)
        alone.step(steps)
        assert _fields_equal([b.read_field(sl, f) for f in ("p", "ux", "uy", "T")],
                             [alone.read_field(f) for f in ("p", "ux", "uy", "T")])
        assert b.observe(sl) == alone.observe()
        alone.close()
    b.close()


def test_batch_fp64_matches_oracle(aq):
    p, mask, walls, geo = A.config0()
    b = aq.Batch(budget_bytes=256 << 20, max_slots=4)
    s = b.admit(p, mask, walls, tol=1e-14, max_steps=10 ** 6, keep=True)
    b.run(10)
    o = O.Oracle(p, mask, walls).step(1000)
    g = [b.read_field(s, f) for f in ("p", "ux", "uy", "T")]
    g[0] = g[0] - p.p_ref
    err = field_errors(g, o.fields(), mask, p.T_ref)
    assert all(v <= 1e-12 for v in err.values()), err
    assert b.observe(s)["iop_gauge"] == pytest.approx(o.observables()["iop_gauge"], rel=1e-12)
    b.close()


def test_admission_limits(aq):
    p, mask, walls = _instances()[1]           # 512x256 F64
    need = aq.required_bytes(p, mask)
    b = aq.Batch(budget_bytes=need + need // 2, max_slots=2)
    assert b.admit(p, mask, walls) is not None
    assert b.admit(p, mask, walls) is None      # out of arena
    p2, m2, w2 = _instances()[0]                # 256x128 F32 fits
    s2 = b.admit(p2, m2, w2)
    assert s2 is not None
    assert b.admit(p2, m2, w2) is None          # out of slots
    b.release(s2)
    assert b.admit(p2, m2, w2) is not None
    b.close()
    act = int(A.active(m2).sum())
    c = aq.Batch(budget_bytes=1 << 30, max_slots=8, max_active_nodes=act + act // 2)
    assert c.admit(p2, m2, w2) is not None
    assert c.admit(p2, m2, w2) is None          # active-node cap
    c.close()


def test_failure_isolated(aq):
    """An instance whose state is non-finite is retired as diverged; the others continue
    exactly as they would alone."""
    insts = _instances()[:2]
    b = aq.Batch(budget_bytes=1 << 30, max_slots=8)
    good = [b.admit(p, m, w, tol=1e-12, max_steps=10 ** 6, keep=True) for p, m, w in insts]
    p, m, w = insts[0]
    bad_p = A.Params(**{**p.asdict(), "p_init": float("nan")})
    bad = b.admit(bad_p, m, w, tol=1e-12, request_id=99)
    b.run(3)
    res = b.poll()
    assert [r["request_id"] for r in res] == [99]
    assert res[0]["status"] == aq.AQ_EDIVERGED
    assert b.info()["running"] == 2
    for sl, (pp, mm, ww) in zip(good, insts):
        alone = aq.Solver(pp, mm, ww)
        alone.set_tile(64, 4)
        alone.step(300)
        assert _fields_equal([b.read_field(sl, f) for f in ("ux", "T")], [alone.read_field(f) for f in ("ux", "T")])
        alone.close()
    b.close()


def test_run_to_steady_and_f16_fallback(aq):
    """Small Ra = 0 eyes run to a steady residual in the batch; the IOP matches a single
    FP64 solve.  The F16S residual stops at binary16's floor above tol: with an impossible
    IOP drift tolerance the solve falls back to F32 and converges to tol (AQ_OK); with a
    loose one it is accepted at the floor (AQ_RESULT_FLOOR, no fallback), its IOP within
    0.1% of FP64."""
    mask, walls, geo = A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2)
    base = A.eye_params(96, 48, geo, Ra=0.0, Da=1e-3, check_interval=100)
    ref = aq.Solver(base, mask, walls)
    ok, ro = ref.run_to_steady(1e-7, 400000)
    assert ok
    b = aq.Batch(budget_bytes=512 << 20, max_slots=8)
    s64 = b.admit(base, mask, walls, tol=1e-7, max_steps=400000, request_id=1)
    p16 = A.Params(**{**base.asdict(), "storage": A.F16S})
    b.admit(p16, mask, walls, tol=1e-7, drift_tol=1e-15, max_steps=600000, request_id=2)
    b.admit(p16, mask, walls, tol=1e-7, drift_tol=10.0, max_steps=600000, request_id=3)
    results = {}
    for _ in range(5000):
        b.run(5)
        for r in b.poll():
            results[r["request_id"]] = r
        if len(results) == 3:
            break
    announce(f"[batch] results {results}")
    assert set(results) == {1, 2, 3}
    r1 = results[1]
    assert r1["status"] == aq.AQ_OK
    assert r1["obs"]["iop_gauge"] == pytest.approx(ro["iop_gauge"], rel=1e-6)
    assert results[2]["fallback"] == 1 and results[2]["storage"] == aq.F32 and results[2]["status"] == aq.AQ_OK
    assert results[3]["fallback"] == 0 and results[3]["storage"] == aq.F16S
    assert results[3]["status"] == aq.AQ_RESULT_FLOOR
    assert max(results[3]["obs"]["resid_u"], results[3]["obs"]["resid_T"]) >= 1e-7
    assert results[3]["obs"]["iop_gauge"] == pytest.approx(ro["iop_gauge"], rel=1e-3)
    announce(f"[batch] iop f64 {r1['obs']['iop_gauge']:.6e} f16->f32 {results[2]['obs']['iop_gauge']:.6e} "
             f"f16 {results[3]['obs']['iop_gauge']:.6e}")
    assert results[2]["obs"]["iop_gauge"] == pytest.approx(ro["iop_gauge"], rel=1e-3)
    b.close()
    ref.close()


def test_autotune_picks_a_valid_shape(aq):
    p, mask, walls = _instances()[1]
    s = aq.Solver(p, mask, walls)
    tx, ty, ms = s.autotune(10, only_256=True)
    assert tx * ty == 256 and ms > 0
    assert (s.info()["tile_x"], s.info()["tile_y"]) == (tx, ty)
    s.close()


def test_full_sweep_batch_sampled_oracle_parity(aq):
    """The 512-instance sweep (every size class, per-instance tau, angle, Ra, Da, gravity
    orientation) resident in one FP64 batch with the benchmark's launch configuration
    (autotuned single-step tiles, 64x8 two-step tiles): after two check intervals one sampled
    instance of each size class matches the oracle to 1e-12."""
    from paper_2102_12663_amd import serve as S
    reqs = [S.sweep_request(i, aq.F64) for i in range(512)]
    cache = S.ShapeCache()
    b = aq.Batch(budget_bytes=96 << 30, max_slots=512, max_tiles=1 << 21)
    slots = []
    for i, (p, m, w) in enumerate(reqs):
        tile = S.autotune_shape(cache, p, m, w)
        slots.append(b.admit(p, m, w, tile=tile, tol=1e-30, max_steps=10 ** 9, request_id=i, keep=True))
    assert all(s is not None for s in slots)
    b.run(2)
    for seed in (3, 16, 13, 4):            # 256x128, 512x256, 768x384, 1024x512
        p, m, w = reqs[seed]
        announce(f"[batch] sweep instance {seed} {p.nx}x{p.ny} vs the oracle")
        o = O.Oracle(p, m, w).step(200)
        g = [b.read_field(slots[seed], f) for f in ("p", "ux", "uy", "T")]
        g[0] = g[0] - p.p_ref
        err = field_errors(g, o.fields(), m, p.T_ref)
        assert all(v <= 1e-12 for v in err.values()), (seed, err)
    b.close()


@pytest.mark.parametrize("storage,tol", [(A.F32, 1e-4), (A.F16S, 2.5e-2)])
def test_full_sweep_batch_against_the_oracle(aq, storage, tol):
    """The benchmark's workload in its launch configuration: the 512-instance sweep in one
    FP32 (or F16S) batch (autotuned single-step tiles, 64x8 two-step tiles, non-temporal
    stores).  After two check intervals, one sampled instance of each size class hands its
    populations to the oracle; one more interval of the batch (48 two-step launches, three
    single steps and the reducing step) is compared with 100 FP64 oracle steps from that
    state.  FP32 must agree to 1e-4 of each field's largest value, the linear-growth bound
    of its arithmetic (about 16 roundings of 2^-24 per value and step over 100 steps); F16S
    to 2.5e-2, the same bound for its binary16 stores (50 roundings of 2^-11, one every
    other step; measured 6.3e-3).  A wrong pull, halo or rule is off by a good part of the
    field."""
    from paper_2102_12663_amd import serve as S
    reqs = [S.sweep_request(i, storage) for i in range(512)]
    cache = S.ShapeCache()
    b = aq.Batch(budget_bytes=64 << 30, max_slots=512, max_tiles=1 << 21)
    slots = [b.admit(p, m, w, tile=S.autotune_shape(cache, p, m, w), tol=1e-30, max_steps=10 ** 9,
                     request_id=i, keep=True) for i, (p, m, w) in enumerate(reqs)]
    assert all(s is not None for s in slots)
    assert b.info()["fused_tile_rows"][storage] == 8
    b.run(2)
    oracles = {}
    for seed in (3, 16, 13, 4):            # 256x128, 512x256, 768x384, 1024x512
        p, m, w = reqs[seed]
        h = np.stack([b.read_field(slots[seed], "pop_flow", q) for q in range(1, 9)])
        g = np.stack([b.read_field(slots[seed], "pop_heat", q) for q in range(5)])
        o = O.Oracle(p, m, w)
        o.set_populations(h, g)
        oracles[seed] = o
    b.run(1)
    for seed, o in oracles.items():
        p, m, w = reqs[seed]
        o.step(100)
        gf = [b.read_field(slots[seed], f) for f in ("p", "ux", "uy", "T")]
        gf[0] = gf[0] - p.p_ref
        err = field_errors(gf, o.fields(), m, p.T_ref)
        announce(f"[batch] storage {storage} sweep instance {seed} {p.nx}x{p.ny}, one interval vs the oracle: "
                 + ", ".join(f"{k} {v:.2e}" for k, v in err.items()))
        assert all(v <= tol for v in err.values()), (seed, err)
    b.close()
