"""The lumped trabecular-meshwork outlet on the GPU (section 2.2.4, section 2.3's coupling
paragraph): parity with the FP64 oracle, the steady closed form, read-out across a check
step (where the seepage speed changes), checkpoint/resume, two-step launches and batching."""
import os
import tempfile

import numpy as np
import pytest

import aqinputs as A
import oracle as O
from gpu_util import announce, field_errors, obs_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELD_TOL = 1e-12
OBS_KEYS = ["iop_gauge", "p_mean_fluid", "q_in", "q_out", "wss_cornea_mean", "wss_iris_max", "resid_u",
            "u_max", "u_seep"]


@pytest.fixture(scope="module")
def aq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    return aq


def _lumped0(storage=A.F64):
    """The 192x96 eye with the lumped meshwork, started 1e-4 above the canal pressure so
    the seepage speed is non-zero from the first interval and changes at every check."""
    mask, walls, geo = A.eye_mask(192, 96, 45.0, R=80.0, pupil_gap=2, tm="lumped")
    p = A.eye_params(192, 96, geo, tm="lumped", storage=storage)
    p.p_init = p.p_sc + 1e-4
    return p, mask, walls


def test_lumped_parity_canal_pressure_apart(aq):
    """The Schlemm's-canal pressure below p_ref and the outlet pressure above it: the
    seepage speed follows IOP - p_sc (eq. 4 over the meshwork), not IOP - p_ref."""
    p, mask, walls = _lumped0()
    p.p_sc = p.p_ref - 3e-5
    p.p_out = p.p_ref + 5e-5
    p.p_init = p.p_sc + 1e-4
    s = aq.Solver(p, mask, walls)
    s.step(1000)
    o = O.Oracle(p, mask, walls).step(1000)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    announce(f"[lumped] canal pressure apart: {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err
    gobs, oobs = s.observe(), o.observables()
    assert not obs_close(gobs, oobs, 1e-11, keys=OBS_KEYS)
    assert gobs["u_seep"] == pytest.approx(oobs["u_seep"], rel=1e-11)
    s.close()


def _duct(n=40, w=12):
    """A walled duct along +x: INLET cells across its left end, OUTLET cells across its
    right end, BOX walls along its sides."""
    m = np.full((w, n), A.encode(A.SOLID), np.uint8)
    m[1:w - 1, 1:n - 1] = A.encode(A.FLUID)
    m[1:w - 1, 0] = A.encode(A.INLET)
    m[1:w - 1, n - 1] = A.encode(A.OUTLET)
    return m


def _duct_mask(d):
    """The duct turned by d quarter turns, with the OUTLET cells' wall bits set to the
    outward direction (0 +x, 1 +y, 2 -x, 3 -y) of the side they landed on."""
    m = np.ascontiguousarray(np.rot90(_duct(), k=d))
    ny, nx = m.shape
    out = (m & 7) == A.OUTLET
    ys, xs = np.nonzero(out)
    if np.all(xs == nx - 1):
        bits = 0
    elif np.all(ys == ny - 1):
        bits = 1
    elif np.all(xs == 0):
        bits = 2
    else:
        bits = 3
    m[out] = A.encode(A.OUTLET, bits)
    return m, bits


@pytest.mark.parametrize("mode", [A.OUTLET_LUMPED, A.OUTLET_PRESSURE])
@pytest.mark.parametrize("bc", [A.BC_LINKWISE, A.BC_PAPER])
@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_outlet_every_direction(aq, d, bc, mode):
    """The outlet drains along +x, -y, -x or +y: a walled duct with the inlet flow along the
    same axis, the lumped meshwork (draining along the OUTLET cells' wall bits) or the
    pressure outlet, 1000 steps, against the oracle to 1e-12, under the link-wise and the
    paper's schemes."""
    m, bits = _duct_mask(d)
    ny, nx = m.shape
    ex, ey = [(1, 0), (0, 1), (-1, 0), (0, -1)][bits]
    U = 2e-3
    p = A.Params(nx=nx, ny=ny, tau_f=0.8, u_in_x=U * ex, u_in_y=U * ey, check_interval=50, bc_scheme=bc,
                 outlet_mode=mode, K_tm=0.05, h_tm=3.0, p_sc=1.0 / 3.0 - 2e-5, p_init=1.0 / 3.0 + 1e-4,
                 p_out=1.0 / 3.0 + 3e-5)
    s = aq.Solver(p, m, A.no_walls())
    s.step(1000)
    o = O.Oracle(p, m).step(1000)
    err = field_errors(s.fields(), o.fields(), m, p.T_ref)
    announce(f"[lumped] duct draining along {bits} bc {bc} outlet mode {mode}: {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err
    gobs, oobs = s.observe(), o.observables()
    assert oobs["q_out"] > 0
    assert gobs["u_seep"] == pytest.approx(oobs["u_seep"], rel=1e-11)
    assert gobs["q_out"] == pytest.approx(oobs["q_out"], rel=1e-11)
    s.close()


def _small(storage=A.F64):
    mask, walls, geo = A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2, tm="lumped")
    p = A.eye_params(96, 48, geo, Ra=0.0, Da=1e-3, tm="lumped", storage=storage)
    return p, mask, walls


def _fields_equal(a, b):
    return all(np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0)) for x, y in zip(a, b))


@pytest.mark.parametrize("steps", [1000, 1037])
def test_lumped_parity_at_and_between_check_steps(aq, steps):
    """1000 steps ends on a check step (the seepage speed has just been re-evaluated and
    the read-out must use the previous one); 1037 ends between checks."""
    p, mask, walls = _lumped0()
    announce(f"[lumped] parity 192x96 steps={steps}")
    s = aq.Solver(p, mask, walls)
    s.step(steps)
    o = O.Oracle(p, mask, walls).step(steps)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    announce(f"[lumped] errors {err}")
    assert all(v <= FIELD_TOL for v in err.values()), err
    gobs, oobs = s.observe(), o.observables()
    assert gobs["step"] == oobs["step"] == 1000
    assert oobs["u_seep"] != 0 and oobs["q_out"] > 0
    bad = obs_close(gobs, oobs, 1e-11, keys=OBS_KEYS)
    assert not bad, bad
    h, g = s.populations()
    ho, go = o.populations()
    act = A.active(mask)
    for q in range(8):
        assert np.max(np.abs(h[q][act] - ho[q][act])) <= FIELD_TOL * np.max(np.abs(ho[q][act]))
    s.close()


def test_lumped_steady_closed_form_gpu(aq):
    """At the steady state the outflow u_s A equals the inflow, so IOP - p_sc =
    nu h_tm Q_in / (K_tm A) with A counted from the mask."""
    p, mask, walls = _small()
    e = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    cls, d = mask & 7, (mask >> 3) & 3
    area = 0.0
    for y, x in zip(*np.nonzero(A.active(mask))):
        for i in range(1, 9):
            yy, xx = y + e[i][1], x + e[i][0]
            if cls[yy, xx] == A.OUTLET:
                n = e[d[yy, xx] + 1]
                area += 6 * w[i] * (e[i][0] * n[0] + e[i][1] * n[1])
    s = aq.Solver(p, mask, walls)
    ok, ob = s.run_to_steady(1e-10, 400000)
    assert ok, ob
    nu = (2 * p.tau_f - 1) / 6
    q_in = 2 * p.u_in_y
    assert ob["p_mean_fluid"] - p.p_sc == pytest.approx(nu * p.h_tm * q_in / (p.K_tm * area), rel=1e-6)
    assert ob["q_out"] == pytest.approx(q_in, rel=1e-6)
    s.close()


def test_lumped_checkpoint_resume_bitwise(aq):
    """A checkpoint taken right at a check step keeps both seepage speeds and the read-out
    slot: the resumed run and its read-outs are bitwise those of the uninterrupted one."""
    p, mask, walls = _lumped0()
    a = aq.Solver(p, mask, walls)
    a.step(600)
    with tempfile.TemporaryDirectory() as dd:
        path = os.path.join(dd, "ck.bin")
        a.save(path)
        f600 = a.fields()
        a.step(400)
        b = aq.Solver(p, mask, walls)
        b.load(path)
        assert _fields_equal(b.fields(), f600)
        b.step(400)
    assert _fields_equal(a.fields(), b.fields())
    assert a.observe() == b.observe()
    a.close()
    b.close()


@pytest.mark.parametrize("storage", [A.F64, A.F32])
def test_lumped_two_step_launches_bitwise(aq, storage):
    p, mask, walls = _lumped0(storage)
    out = []
    for fuse in (False, True):
        s = aq.Solver(p, mask, walls)
        s.set_fusion(fuse)
        s.step(537)
        out.append(([s.read_field(f) for f in ("p", "ux", "uy", "T")], s.observe()))
        s.close()
    assert _fields_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_lumped_in_a_batch_bitwise_and_f16_handoff(aq):
    """A lumped instance runs in a batch exactly as alone (next to a pressure-outlet one);
    an F16S lumped solve handed to FP32 keeps its seepage speed and reaches the closed
    form of the FP64 solve."""
    p, mask, walls = _lumped0()
    p2, m2, w2, geo2 = A.sweep_instance(3, 256, 128)
    b = aq.Batch(budget_bytes=1 << 30, max_slots=8)
    s1 = b.admit(p, mask, walls, tile=(64, 4), tol=1e-14, max_steps=10 ** 6, keep=True)
    s2 = b.admit(p2, m2, w2, tile=(64, 4), tol=1e-14, max_steps=10 ** 6, keep=True)
    b.run(7)
    alone = aq.Solver(p, mask, walls)
    alone.set_tile(64, 4)
    alone.step(700)
    assert _fields_equal([b.read_field(s1, f) for f in ("p", "ux", "uy", "T")],
                         [alone.read_field(f) for f in ("p", "ux", "uy", "T")])
    assert b.observe(s1) == alone.observe()
    alone.close()
    b.close()

    ps, ms, ws = _small()
    ref = aq.Solver(ps, ms, ws)
    ok, ro = ref.run_to_steady(1e-9, 400000)
    assert ok
    ref.close()
    p16 = A.Params(**{**ps.asdict(), "storage": A.F16S})
    c = aq.Batch(budget_bytes=512 << 20, max_slots=4)
    # residual 1e-6, the batched sweep's tolerance: FP32 rounding keeps this small Ra = 0
    # case's residual near 1e-7 (FP64 reaches 1e-15)
    c.admit(p16, ms, ws, tol=1e-6, drift_tol=1e-15, max_steps=800000, request_id=5)
    res = None
    for _ in range(5000):
        c.run(5)
        r = c.poll()
        if r:
            res = r[0]
            break
    c.close()
    announce(f"[lumped] f16 hand-off {res}")
    assert res is not None and res["status"] == aq.AQ_OK and res["fallback"] == 1
    assert res["obs"]["p_mean_fluid"] - ps.p_sc == pytest.approx(ro["p_mean_fluid"] - ps.p_sc, rel=1e-4)
