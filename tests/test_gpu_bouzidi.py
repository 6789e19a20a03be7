"""The paper's boundary schemes (section 2.3) on the GPU: interpolated bounce-back of
Bouzidi et al. on the walls (link fractions from the exact cornea circle), Guo et al.'s
non-equilibrium extrapolation at the inlet and outlet, the thermal extrapolation at the
Dirichlet walls.  Parity with the oracle on the eye (both outlet models, from the initial
state on) and on an off-lattice box, and bitwise two-step launches."""
import math

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


def _eye(tm="resolved", storage=A.F64):
    mask, walls, geo = A.eye_mask(192, 96, 45.0, R=80.0, pupil_gap=2, tm=tm)
    p = A.eye_params(192, 96, geo, tm=tm, storage=storage, phi_deg=30.0)
    p.bc_scheme = A.BC_PAPER
    return p, mask, walls


@pytest.mark.parametrize("tm", ["resolved", "lumped"])
def test_bouzidi_eye_parity(aq, tm):
    p, mask, walls = _eye(tm)
    if tm == "lumped":
        p.p_init = p.p_sc + 1e-4
    assert np.any((walls["q"] > 0) & (walls["q"] < 0.5)) and np.any(walls["q"] > 0.5)
    announce(f"[bouzidi] eye {tm} parity")
    s = aq.Solver(p, mask, walls)
    o = O.Oracle(p, mask, walls)
    # the initial state's extrapolated boundary populations agree
    h, g = s.populations()
    ho, go = o.populations()
    act = A.active(mask)
    assert np.max(np.abs(h[:, act] - ho[:, act])) <= 1e-15 and np.max(np.abs(g[:, act] - go[:, act])) <= 1e-15
    s.step(1000)
    o.step(1000)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    announce(f"[bouzidi] errors {err}")
    assert all(v <= 1e-12 for v in err.values()), err
    bad = obs_close(s.observe(), o.observables(), 1e-11,
                    keys=["iop_gauge", "q_out", "wss_cornea_mean", "wss_cornea_max", "resid_u", "u_max"])
    assert not bad, bad
    s.close()


def test_bouzidi_offgrid_box_parity(aq):
    """A closed box whose bottom and top walls sit off the half-way lines (fractions 0.3
    and 0.8), driven by a force along x: the recirculation matches the oracle."""
    nx, ny, qb, qt, F = 64, 24, 0.3, 0.8, 1e-6
    p = A.Params(nx=nx, ny=ny, tau_f=0.8, check_interval=100, gbeta=F,
                 gravity_angle=math.pi / 2, T_init=1.5, T0=0.5, bc_scheme=A.BC_PAPER)
    mask = A.box_mask(nx, ny)
    walls = np.zeros(2 * (nx - 2), dtype=A.WALL_DTYPE)
    for j, x in enumerate(range(1, nx - 1)):
        walls[j] = (nx + x, A.WALL_IRIS, 0.0, 1.0, [-1, -1, -1, qb, -1, -1, qb, qb])
        walls[nx - 2 + j] = ((ny - 2) * nx + x, A.WALL_CORNEA, 0.0, -1.0, [-1, qt, -1, -1, qt, qt, -1, -1])
    walls = np.sort(walls, order="node")
    s = aq.Solver(p, mask, walls)
    s.step(3000)
    o = O.Oracle(p, mask, walls).step(3000)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    assert all(v <= 1e-12 for v in err.values()), err
    s.close()


@pytest.mark.parametrize("storage", [A.F64, A.F32, A.F32X])
def test_bouzidi_two_step_launches_bitwise(aq, storage):
    """Two steps per launch give bitwise the single-step result with the paper's schemes
    (F16S rounds where it stores, so its schedule differs by design; its paper-scheme
    solve is checked alone against batched in test_paper_scheme_in_a_batch_bitwise)."""
    p, mask, walls = _eye(storage=storage)
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


def test_paper_scheme_in_a_batch_bitwise(aq):
    """Instances with the paper's schemes and link-wise ones share a batch (separate kernel
    classes); each computes exactly what it computes alone."""
    p1, m1, w1 = _eye()
    p2, m2, w2, geo2 = A.sweep_instance(3, 256, 128)
    p3 = A.Params(**{**p1.asdict(), "storage": A.F32})
    p4 = A.Params(**{**p1.asdict(), "storage": A.F16S})
    insts = ((p1, m1, w1), (p2, m2, w2), (p3, m1, w1), (p4, m1, w1))
    b = aq.Batch(budget_bytes=1 << 30, max_slots=8)
    slots = [b.admit(p, m, w, tile=(64, 4), tol=1e-14, max_steps=10 ** 6, keep=True) for p, m, w in insts]
    b.run(5)
    for sl, (p, m, w) in zip(slots, insts):
        alone = aq.Solver(p, m, w)
        alone.set_tile(64, 4)
        alone.step(500)
        for f in ("p", "ux", "uy", "T"):
            assert np.array_equal(np.nan_to_num(b.read_field(sl, f), nan=7.0), np.nan_to_num(alone.read_field(f), nan=7.0))
        assert b.observe(sl) == alone.observe()
        alone.close()
    b.close()
