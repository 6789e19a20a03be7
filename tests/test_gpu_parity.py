"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

FP64 storage must match the oracle to 1e-12 normwise per field after 1000 steps; the
observables of the check steps to 1e-12 relative (sums in a different order).
"""
import math
import os
import tempfile

import numpy as np
import pytest

import aqinputs as A
import oracle as O
from gpu_util import announce, field_errors, obs_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    return aq


FIELD_TOL = 1e-12
OBS_TOL = 1e-12


def _run_pair(aq, p, mask, walls, steps):
    announce(f"[parity] {p.nx}x{p.ny} storage={p.storage} steps={steps}")
    s = aq.Solver(p, mask, walls)
    s.step(steps)
    gf = s.fields()
    gobs = s.observe()
    o = O.Oracle(p, mask, walls)
    o.step(steps)
    return s, o, gf, o.fields(), gobs, o.observables()


def test_config0_fp64_fields_and_observables(aq):
    """192x96 eye, FP64, 1000 steps: fields and check-step observables vs the oracle."""
    p, mask, walls, geo = A.config0()
    s, o, gf, of, gobs, oobs = _run_pair(aq, p, mask, walls, 1000)
    err = field_errors(gf, of, mask, p.T_ref)
    announce(f"[parity] config0 field errors {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err
    assert gobs["step"] == oobs["step"] == 1000
    bad = obs_close(gobs, oobs, OBS_TOL,
                    keys=["iop_gauge", "p_mean_fluid", "q_in", "q_out", "wss_cornea_mean",
                          "wss_cornea_max", "wss_iris_mean", "wss_iris_max", "resid_u", "resid_T",
                          "u_max"])
    assert not bad, bad
    # masses are sums with cancellation: compare against the sum of magnitudes
    h, g = o.populations()
    act = A.active(mask)
    assert abs(gobs["mass_flow"] - oobs["mass_flow"]) <= 1e-13 * np.sum(np.abs(h[:, act]))
    assert abs(gobs["mass_thermal"] - oobs["mass_thermal"]) <= 1e-13 * np.sum(np.abs(g[:, act]))
    assert gobs["n_nonfinite"] == 0


def test_config0_fp64_populations(aq):
    """Pre-collision populations (deviation form) after 1000 steps."""
    p, mask, walls, geo = A.config0()
    s = aq.Solver(p, mask, walls)
    s.step(1000)
    h, g = s.populations()
    o = O.Oracle(p, mask, walls).step(1000)
    ho, go = o.populations()
    act = A.active(mask)
    for q in range(8):
        sc = np.max(np.abs(ho[q][act]))
        assert np.max(np.abs(h[q][act] - ho[q][act])) <= FIELD_TOL * sc
    for q in range(5):
        sc = np.max(np.abs(go[q][act]))
        assert np.max(np.abs(g[q][act] - go[q][act])) <= FIELD_TOL * max(sc, 1e-300)
    assert np.all(np.isnan(h[:, ~act]))


@pytest.mark.parametrize("nx,ny,alpha", [(131, 70, 37.0), (200, 101, 30.0)])
def test_ragged_random_state_every_boundary(aq, nx, ny, alpha):
    """Ragged lattice (nx not a multiple of the tile width), random pre-collision state
    (so every link rule sees non-trivial values), buoyancy at an angle, strong drag."""
    mask, walls, geo = A.eye_mask(nx, ny, alpha)
    p = A.eye_params(nx, ny, geo, u_in=3e-4, Da=3e-4, Ra=5e3, phi_deg=30.0, check_interval=20)
    p.p_out = p.p_ref + 1e-4
    p.T_inlet = 0.8
    rng = np.random.default_rng(11)
    h = rng.normal(0, 1e-4, (8, ny, nx))
    g = rng.normal(0, 1e-2, (5, ny, nx))
    s = aq.Solver(p, mask, walls)
    s.write_populations(h, g)
    o = O.Oracle(p, mask, walls)
    o.set_populations(h, g)
    s.step(200)
    o.step(200)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    announce(f"[parity] ragged {nx}x{ny} errors {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err
    bad = obs_close(s.observe(), o.observables(), 1e-11,
                    keys=["iop_gauge", "q_in", "q_out", "wss_cornea_mean", "wss_iris_max", "resid_u", "u_max"])
    assert not bad, bad


def _apart(p):
    """The eye's parameters with every reference level apart: the deviation form's T_ref and
    p_ref, the Boussinesq T0 (eq. 16), the initial, wall and inlet temperatures, the initial
    and outlet pressures."""
    return A.Params(**{**p.asdict(), "T_ref": 0.2, "T0": 0.6, "T_init": 0.45, "T_cornea": 0.05,
                       "T_iris": 0.95, "T_inlet": 0.8, "p_init": p.p_ref + 2e-5, "p_out": p.p_ref + 1e-4,
                       "u_in_x": 0.5 * p.u_in_y})


@pytest.mark.parametrize("storage,tol", [(A.F64, FIELD_TOL), (A.F32, 1e-4), (A.F32X, 1e-4), (A.F16S, 1e-2)])
def test_reference_levels_apart(aq, storage, tol):
    """192x96 eye with every reference level apart (T_ref, T0, the wall, inlet and initial
    temperatures, p_ref, p_init, p_out), an oblique inlet velocity and strong buoyancy (Ra 2e4), 500 steps: fields
    against the oracle: FP64 to 1e-12 of each field's largest value, FP32 and F32X to
    1e-4 (measured 1.2e-6 and 2.6e-7), F16S (binary16 storage, 11 significant bits) to 1e-2
    (measured 1.9e-3).  A level taken for another
    (say the buoyancy measured from T_ref, off by 0.4 g beta against forces of at most
    0.55 g beta) moves the fields by far more than any of these."""
    p0, mask, walls, geo = A.config0()
    p = _apart(A.Params(**{**p0.asdict(), "gbeta": 20 * p0.gbeta, "storage": storage}))
    s, o, gf, of, gobs, oobs = _run_pair(aq, p, mask, walls, 500)
    err = field_errors(gf, of, mask, p.T_ref)
    announce(f"[parity] reference levels apart, storage={storage}: {err}")
    assert all(v <= tol for v in err.values()), err
    if storage == A.F64:
        bad = obs_close(gobs, oobs, 1e-11, keys=["iop_gauge", "q_in", "q_out", "wss_cornea_mean", "wss_iris_mean",
                                                  "resid_u", "resid_T", "u_max"])
        assert not bad, bad


def test_reference_levels_apart_paper_scheme(aq):
    """The same case under the paper's boundary schemes (interpolated bounce-back on the
    cornea and iris, extrapolated inlet, outlet and Dirichlet walls), FP64, to 1e-12."""
    p0, mask, walls, geo = A.config0()
    p = _apart(A.Params(**{**p0.asdict(), "gbeta": 20 * p0.gbeta, "bc_scheme": A.BC_PAPER}))
    s, o, gf, of, gobs, oobs = _run_pair(aq, p, mask, walls, 500)
    err = field_errors(gf, of, mask, p.T_ref)
    announce(f"[parity] reference levels apart, paper scheme: {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err


def test_reference_levels_apart_in_a_batch(aq):
    """The same case as an FP64 instance of a batch, beside an instance at the default
    levels: the batch's per-instance constants carry every level."""
    p0, mask, walls, geo = A.config0()
    p = _apart(A.Params(**{**p0.asdict(), "gbeta": 20 * p0.gbeta}))
    b = aq.Batch(budget_bytes=1 << 30, max_slots=4)
    sa = b.admit(p, mask, walls, tile=(64, 4), tol=1e-30, max_steps=10 ** 6, keep=True)
    sb = b.admit(p0, mask, walls, tile=(64, 4), tol=1e-30, max_steps=10 ** 6, keep=True)
    b.run(5)
    for sl, q in ((sa, p), (sb, p0)):
        o = O.Oracle(q, mask, walls).step(500)
        g = [b.read_field(sl, f) for f in ("p", "ux", "uy", "T")]
        g[0] = g[0] - q.p_ref
        err = field_errors(g, o.fields(), mask, q.T_ref)
        assert all(v <= FIELD_TOL for v in err.values()), err
    b.close()


@pytest.mark.parametrize("tile", [(64, 1), (64, 2), (128, 2), (256, 1)])
def test_tile_shapes_bitwise(aq, tile):
    """The per-node arithmetic does not depend on the tile shape: fields bitwise equal."""
    p, mask, walls, geo = A.config0()
    ref = aq.Solver(p, mask, walls)
    ref.step(300)
    s = aq.Solver(p, mask, walls)
    s.set_tile(*tile)
    s.step(300)
    for a, b in zip(ref.fields(), s.fields()):
        assert np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))
    bad = obs_close(ref.observe(), s.observe(), 1e-13, keys=["iop_gauge", "q_out", "resid_u", "u_max"])
    assert not bad


def test_determinism_and_partial_steps(aq):
    """Two runs are bitwise identical, including the (fixed-order) reductions; stepping
    in irregular pieces equals stepping in whole intervals."""
    p, mask, walls, geo = A.config0()
    a = aq.Solver(p, mask, walls)
    a.step(1000)
    b = aq.Solver(p, mask, walls)
    for n in (7, 93, 1, 299, 600):
        b.step(n)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0))
    assert a.observe() == b.observe()


def test_checkpoint_resume_bitwise(aq):
    p, mask, walls, geo = A.config0()
    a = aq.Solver(p, mask, walls)
    a.step(600)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(400)
        b = aq.Solver(p, mask, walls)
        b.load(path)
        b.step(400)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0))
    assert a.observe() == b.observe()


def test_closed_box_conservation_gpu(aq):
    """Closed box with buoyancy and a porous patch: sum h and sum g stay fixed on the GPU."""
    nx, ny = 150, 70
    mask = A.box_mask(nx, ny, porous_rect=(20, 40, 10, 30))
    p = A.Params(nx=nx, ny=ny, tau_f=0.7, tau_t=0.8, gbeta=1e-3, check_interval=10, K=0.05)
    rng = np.random.default_rng(2)
    s = aq.Solver(p, mask, A.no_walls())
    h = rng.normal(0, 1e-4, (8, ny, nx))
    g = rng.normal(0, 1e-2, (5, ny, nx))
    s.write_populations(h, g)
    s.step(10)
    m0 = s.observe()
    s.step(2000)
    m1 = s.observe()
    act = A.active(mask)
    assert abs(m1["mass_flow"] - m0["mass_flow"]) < 1e-12 * np.sum(np.abs(h[:, act]))
    assert abs(m1["mass_thermal"] - m0["mass_thermal"]) < 1e-12 * np.sum(np.abs(g[:, act]))


def test_run_to_steady_matches_oracle_iop(aq):
    """Small eye at Ra = 0 run to a steady residual: IOP and outflow = inflow."""
    mask, walls, geo = A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2)
    p = A.eye_params(96, 48, geo, Ra=0.0, Da=1e-3, check_interval=100)
    s = aq.Solver(p, mask, walls)
    ok, ob = s.run_to_steady(1e-7, 200000)
    assert ok, ob
    o = O.Oracle(p, mask, walls).step(ob["step"])
    oo = o.observables()
    assert ob["iop_gauge"] == pytest.approx(oo["iop_gauge"], rel=1e-10)
    assert abs(ob["q_out"] / ob["q_in"] - 1) < 1e-6


@pytest.mark.parametrize("storage,tol_u,tol_iop", [(A.F32, 1e-4, 1e-3), (A.F16S, 5e-2, 5e-2), (A.F32X, 1e-6, 1e-6)])
def test_reduced_precision_close_to_fp64(aq, storage, tol_u, tol_iop):
    """FP32, F16S and F32X storage after 1000 steps of the 192x96 case stay near FP64."""
    p, mask, walls, geo = A.config0()
    ref = aq.Solver(p, mask, walls)
    ref.step(1000)
    p2 = A.Params(**{**p.asdict(), "storage": storage})
    s = aq.Solver(p2, mask, walls)
    s.step(1000)
    act = A.active(mask)
    ur = np.hypot(*ref.fields()[1:3])[act]
    u2 = np.hypot(*s.fields()[1:3])[act]
    rel = np.linalg.norm(u2 - ur) / np.linalg.norm(ur)
    oa, ob = ref.observe(), s.observe()
    announce(f"[precision] storage={storage} u L2 rel {rel:.3e} iop {oa['iop_gauge']:.6e} vs {ob['iop_gauge']:.6e} exps {s.info()['fp16_exp_flow']},{s.info()['fp16_exp_thermal']}")
    assert rel < tol_u
    assert abs(ob["iop_gauge"] - oa["iop_gauge"]) <= tol_iop * abs(oa["iop_gauge"])


def test_config1_size_fp64_parity(aq):
    """2048x1024 eye (sweep seed 0, the benchmark's workload and tile shape), FP64, 1000
    steps: every field vs the oracle, normwise 1e-12."""
    p, mask, walls, geo = A.sweep_instance(0, 2048, 1024)
    s, o, gf, of, gobs, oobs = _run_pair(aq, p, mask, walls, 1000)
    err = field_errors(gf, of, mask, p.T_ref)
    announce(f"[parity] 2048x1024 field errors {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err
    bad = obs_close(gobs, oobs, 1e-11, keys=["iop_gauge", "q_in", "q_out", "wss_cornea_mean",
                                              "wss_iris_mean", "resid_u", "resid_T", "u_max"])
    assert not bad, bad


@pytest.mark.parametrize("storage", [A.F64, A.F32, A.F32X])
@pytest.mark.parametrize("size", [(192, 96), (300, 150)])
def test_two_step_fusion_bitwise(aq, storage, size):
    """Two steps per launch (temporal blocking through LDS) gives bitwise the same state
    and observables as single-step launches in F64, F32 and F32X (F16S keeps the
    intermediate step in single precision: test_f16s_launch_against_the_oracle)."""
    nx, ny = size
    if (nx, ny) == (192, 96):
        p, mask, walls, geo = A.config0()
    else:
        p, mask, walls, geo = A.sweep_instance(4, nx, ny, tau_f="draw", phi_deg="draw")
    p = A.Params(**{**p.asdict(), "storage": storage})
    out = []
    for fuse in (False, True):
        s = aq.Solver(p, mask, walls)
        s.set_fusion(fuse)
        s.step(537)
        out.append(([s.read_field(f) for f in ("p", "ux", "uy", "T")], s.observe()))
        s.close()
    for x, y in zip(out[0][0], out[1][0]):
        assert np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0))
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("storage", [A.F32, A.F16S])
@pytest.mark.parametrize("size", [(300, 150), (2048, 1024)])
def test_fused_tile_rows_bitwise(aq, storage, size):
    """The two-step tiles of F32 and F16S come in 64 x 8 and 64 x 4: the state and the
    observables are bitwise the same with either (a node's step-A value does not depend on
    which tile's halo computes it)."""
    nx, ny = size
    p, mask, walls, geo = A.sweep_instance(4, nx, ny, tau_f="draw", phi_deg="draw", storage=storage)
    out = []
    for rows in (8, 4):
        s = aq.Solver(p, mask, walls)
        s.set_fusion(True)
        s.set_fused_tile_rows(rows)
        assert s.info()["fused_tile_rows"] == rows
        s.step(537)
        out.append(([s.read_field(f) for f in ("p", "ux", "uy", "T")], s.observe()))
        s.close()
    for x, y in zip(out[0][0], out[1][0]):
        assert np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0))
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("fused", [True, False])
def test_f16s_launch_against_the_oracle(aq, fused):
    """F16S stores binary16 and computes in single precision; a two-step launch keeps its
    intermediate step in single precision and rounds (mass-conserving) where it stores.
    From a binary16 state of a ragged lattice with every boundary rule, one two-step launch
    and the single step after it (fused), or three single steps, agree with three FP64
    oracle steps from the same state link by link, to within the binary16 rounding of the
    stores: 16 half-ulps of the node's largest population.  A wrong pull, halo or rule
    would be off by a good part of the population itself."""
    p, mask, walls, geo = A.sweep_instance(4, 300, 150, tau_f="draw", phi_deg="draw")
    s = aq.Solver(A.Params(**{**p.asdict(), "storage": A.F16S}), mask, walls)
    s.step(237)
    h, g = s.populations()
    o = O.Oracle(p, mask, walls)
    o.set_populations(h, g)
    if fused:
        s.time_fused_kernel(1)                 # one two-step launch, then one single step
    else:
        s.set_fusion(False)
        s.step(3)
    o.step(3)
    act = A.active(mask)
    for got, ref in zip(s.populations(), o.populations()):
        a, b = got[:, act], ref[:, act]
        assert np.all(np.isfinite(a))
        tol = 2.0 ** -7 * np.max(np.abs(b), axis=0) + 2.0 ** -20 * np.max(np.abs(b))
        err = np.abs(a - b)
        assert np.all(err <= tol), float(np.max(err / tol))
    s.close()
