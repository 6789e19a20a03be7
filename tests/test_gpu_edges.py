"""Edge cases of the HIP path: empty and one-node lattices, the paper-exact D2Q4 thermal
mode, a standing eye (gravity along -x), and properties at the 8192x4096 size."""
import math

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


def _parity(aq, p, mask, walls, steps, tol=1e-12):
    s = aq.Solver(p, mask, walls)
    s.step(steps)
    o = O.Oracle(p, mask, walls).step(steps)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    s.close()
    return err


def test_empty_lattice(aq):
    """No active node: every call works and the observables stay zero."""
    mask = np.zeros((32, 70), np.uint8)
    p = A.Params(nx=70, ny=32, check_interval=10)
    s = aq.Solver(p, mask, A.no_walls())
    s.step(35)
    ob = s.observe()
    assert ob["step"] == 30 and ob["mass_flow"] == 0 and ob["u_max"] == 0
    assert np.all(np.isnan(s.read_field("ux")))
    s.close()


def test_single_active_node(aq):
    """One fluid node surrounded by every kind of link rule (walls, inlet, outlet)."""
    mask = np.zeros((5, 5), np.uint8)
    mask[2, 2] = A.encode(A.FLUID)
    mask[1, 2] = A.encode(A.INLET)
    mask[2, 3] = A.encode(A.OUTLET)
    mask[3, 2] = A.encode(A.SOLID, A.WALL_CORNEA)
    mask[2, 1] = A.encode(A.SOLID, A.WALL_IRIS)
    p = A.Params(nx=5, ny=5, u_in_y=1e-3, p_out=1 / 3 + 1e-4, gbeta=1e-3, check_interval=10, T_init=0.3)
    err = _parity(aq, p, mask, A.no_walls(), 100)
    assert all(v <= 1e-12 for v in err.values()), err


def test_paper_d2q4_thermal_mode(aq):
    """w0 = 0: the thermal lattice is the paper's D2Q4 (eq. 11-14) exactly."""
    p, mask, walls, geo = A.config0()
    p.w0 = 0.0
    err = _parity(aq, p, mask, walls, 1000)
    assert all(v <= 1e-12 for v in err.values()), err


def test_standing_eye_gravity_along_x(aq):
    """Standing orientation (section 3.1): gravity along -x, one vortex."""
    p, mask, walls, geo = A.config0()
    p.gravity_angle = math.pi / 2
    p.gbeta *= 10
    err = _parity(aq, p, mask, walls, 1000)
    assert all(v <= 1e-12 for v in err.values()), err


def test_config2_size_fp64_parity_100_steps(aq):
    """8192x4096 (33.5M nodes), FP64, 100 steps: every field vs the oracle."""
    p, mask, walls, geo = A.sweep_instance(0, 8192, 4096)
    announce("[edges] 8192x4096 oracle run (CPU)")
    err = _parity(aq, p, mask, walls, 100)
    announce(f"[edges] 8192x4096 errors {err}")
    assert all(v <= 1e-12 for v in err.values()), err


@pytest.mark.parametrize("storage", [A.F64, A.F32, A.F16S, A.F32X])
def test_config2_size_mirror_symmetry(aq, storage):
    """Gravity along -y and a mirror-symmetric section: the state stays mirror symmetric
    at 8192x4096 (u_x odd, the rest even) in every storage."""
    p, mask, walls, geo = A.sweep_instance(0, 8192, 4096, storage=storage)
    s = aq.Solver(p, mask, walls)
    s.step(600)
    act = A.active(mask)
    dp, ux, uy, T = s.fields()
    tol = {A.F64: 1e-11, A.F32: 1e-5, A.F16S: 1e-2, A.F32X: 1e-5}[storage]
    for F, sign in ((dp, 1), (ux, -1), (uy, 1), (T - p.T_ref, 1)):
        sc = np.max(np.abs(F[act]))
        assert np.max(np.abs(F[act] - sign * F[:, ::-1][act])) <= tol * sc
    s.close()


def test_full_box_conservation_8192(aq):
    """All-interior box at 8192x4096 with buoyancy: sum h and sum g stay fixed."""
    nx, ny = 8192, 4096
    mask = A.box_mask(nx, ny)
    p = A.Params(nx=nx, ny=ny, gbeta=1e-4, check_interval=100, T_init=0.7, T_cornea=0.0)
    s = aq.Solver(p, mask, A.no_walls())
    s.step(100)
    a = s.observe()
    s.step(1000)
    b = s.observe()
    assert abs(b["mass_thermal"] - a["mass_thermal"]) <= 1e-12 * abs(a["mass_thermal"])
    assert abs(b["mass_flow"] - a["mass_flow"]) <= 1e-8
    s.close()


@pytest.mark.parametrize("storage,fused,tol", [(A.F32, False, 1e-4), (A.F32, True, 1e-4), (A.F16S, True, 1e-2)])
def test_largest_lattice_far_corner(aq, storage, fused, tol):
    """The largest lattice the single-precision storages accept (three padded population
    planes within the 4 GiB that a 32-bit byte offset spans): 16384 columns and 21844 rows in
    F32, 43690 in F16S.  The 192x96 eye sits in its far corner, where the offsets are
    largest, with solid nodes everywhere else.  After 200 steps the corner holds what the
    oracle computes for the eye alone: FP32 to 1e-4 of each field's largest value, single
    and two-step launches, and F16S to 1e-2."""
    p0, m0, w0, geo = A.config0()
    elem = 4 if storage == A.F32 else 2
    NX = 16384
    NY = ((1 << 32) // elem - NX - 1 - 3 * 704) // (3 * NX)     # plane: NY * NX + 704 elements
    ny, nx = m0.shape
    y0, x0 = NY - ny, NX - nx
    mask = np.full((NY, NX), A.encode(A.SOLID), np.uint8)
    mask[y0:, x0:] = m0
    walls = w0.copy()
    walls["node"] = (w0["node"] // nx + y0) * NX + w0["node"] % nx + x0
    p = A.Params(**{**p0.asdict(), "nx": NX, "ny": NY, "storage": storage})
    announce(f"[edges] {NX}x{NY} storage={storage} fused={fused}: the eye in the far corner")
    s = aq.Solver(p, mask, walls)
    s.set_fusion(fused)
    s.step(200)
    g = [s.read_field(f)[y0:, x0:] for f in ("p", "ux", "uy", "T")]
    s.close()
    g[0] = g[0] - p.p_ref
    o = O.Oracle(p0, m0, w0).step(200)
    err = field_errors(g, o.fields(), m0, p0.T_ref)
    announce(f"[edges] far corner errors {err}")
    assert all(v <= tol for v in err.values()), err


@pytest.mark.parametrize("storage", [A.F64, A.F32])
def test_non_finite_nodes_counted_like_the_oracle(aq, storage):
    """A NaN planted in one thermal population and an infinity in one flow population, far
    apart, spread through the lattice step by step.  After one check interval of 10 steps
    (387 of the 1,886 active nodes reached) the count of non-finite nodes equals the
    oracle's (every node whose pressure, velocity or temperature is not finite)."""
    p0, mask, walls, geo = A.config0()
    p0.check_interval = 10
    p = A.Params(**{**p0.asdict(), "storage": storage})
    s = aq.Solver(p, mask, walls)
    s.step(100)
    h, g = s.populations()
    ys, xs = np.nonzero(A.active(mask))
    g[2, ys[10], xs[10]] = np.nan
    h[5, ys[-10], xs[-10]] = np.inf
    s.write_populations(h, g)
    o = O.Oracle(p0, mask, walls)
    o.set_populations(h, g)
    s.step(10)
    o.step(10)
    got, want = s.observe()["n_nonfinite"], o.observables()["n_nonfinite"]
    announce(f"[edges] non-finite nodes after one interval, storage={storage}: {got} (oracle {want})")
    assert 0 < want < A.active(mask).sum() and got == want
    s.close()
