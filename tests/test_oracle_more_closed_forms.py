"""More pins of the oracle's full time step, each fixing a term that the other pins leave
free: the buoyancy reference temperature (eq. 16), the non-equilibrium part that the
paper's inlet/outlet extrapolation carries (section 2.3), the wall shear stress as the
tangential traction (section 3.6), the IOP as a mean over the chamber's fluid only
(section 2.2.4), and the residual per time step.
"""
import math

import numpy as np
import pytest

import aqinputs as A
import oracle as O
from _oracle_util import init_from_fields

# e_i of links 1..8 (slot q - 1 holds link q)
EX = np.array([1, 0, -1, 0, 1, -1, -1, 1], float)
EY = np.array([0, 1, 0, -1, 1, 1, -1, -1], float)
# zero-mass, zero-momentum patterns of the flow links (deviation form): a shear stress
# (Pi_xy = 4), an isotropic stress (Pi_xx = Pi_yy = -2) and a normal-stress difference
# (Pi_xx = 2, Pi_yy = -2)
SHEAR = EX * EY
ISO = np.array([1, 1, 1, 1, -1, -1, -1, -1], float)
NORMAL = np.array([1, -1, 1, -1, 0, 0, 0, 0], float)


def test_patterns_carry_only_stress():
    for v in (SHEAR, ISO, NORMAL):
        assert v.sum() == 0 and (EX * v).sum() == 0 and (EY * v).sum() == 0
    assert (EX * EY * SHEAR).sum() == 4 and (EX * EX * SHEAR).sum() == 0 and (EY * EY * SHEAR).sum() == 0
    assert (EX * EY * ISO).sum() == 0 and (EX * EX * ISO).sum() == -2 and (EY * EY * ISO).sum() == -2
    assert (EX * EY * NORMAL).sum() == 0 and (EX * EX * NORMAL).sum() == 2 and (EY * EY * NORMAL).sum() == -2


def test_buoyancy_is_measured_from_T0():
    """Eq. 16 measures the buoyant force from the Boussinesq reference T0, which need not
    be the deviation form's T_ref.  With T_ref = 0, T0 = 0.5 and a uniform T = 1.5, the
    force g beta (T - T0) along +x drives the exact lattice parabola: nu times the second
    difference of u is -F at every interior row."""
    nx, ny, tau, gb = 4, 16, 0.8, 1e-6
    P = A.Params(nx=nx, ny=ny, tau_f=tau, periodic_x=1, check_interval=1000, gbeta=gb,
                 gravity_angle=math.pi / 2, T_ref=0.0, T0=0.5, T_init=1.5)
    o = O.Oracle(P, A.channel_mask(nx, ny))
    nu = (2 * tau - 1) / 6
    o.step(12000)
    u = o.fields()[1][1:ny - 1, 1]
    F = gb * (1.5 - 0.5)
    assert np.max(np.abs(nu * (u[2:] - 2 * u[1:-1] + u[:-2]) / F + 1)) < 1e-8


def _duct(U=0.02, nx=24, ny=6, T=0.7):
    """Duct periodic in y: INLET column x = 0 (velocity U, temperature T), OUTLET column
    x = nx - 1 (p_out), no walls, the paper's extrapolation scheme."""
    mask = np.full((ny, nx), A.encode(A.FLUID), np.uint8)
    mask[:, 0] = A.encode(A.INLET)
    mask[:, nx - 1] = A.encode(A.OUTLET)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, tau_t=0.75, periodic_y=1, u_in_x=U, p_out=1.0 / 3.0 + 1e-4,
                 T_ref=0.0, T0=T, T_init=T, T_inlet=T, check_interval=100, bc_scheme=A.BC_PAPER)
    return mask, P


def test_extrapolation_carries_the_non_equilibrium_part():
    """Guo et al.'s extrapolation (section 2.3) gives the population entering from a
    boundary node as the boundary's equilibrium plus the fluid node's own non-equilibrium
    part.  A uniform flow at (p_out, u_in) with a uniform zero-mass, zero-momentum
    non-equilibrium part d is then uniform for all time: BGK relaxes d to (1 - 1/tau) d at
    every node, the inlet and the outlet included.  Likewise a uniform temperature T_inlet
    in that flow, with a zero-sum thermal non-equilibrium part, stays uniform upstream of
    the adiabatic outlet's reach."""
    mask, P = _duct()
    ny, nx = mask.shape
    o = O.Oracle(P, mask)
    init_from_fields(o, P, P.p_out, P.u_in_x, 0.0, P.T_inlet)
    h0, g0 = (a.copy() for a in o.populations())
    d = 1e-5 * (SHEAR + 0.5 * ISO - 0.3 * NORMAL)
    dg = 1e-3 * np.array([-4.0, 1.0, 1.0, 1.0, 1.0])
    act = A.active(mask)
    o.set_populations(h0 + d[:, None, None] * act, g0 + dg[:, None, None] * act)
    n = 6
    o.step(n)
    h, g = o.populations()
    want_h = h0 + (1 - 1 / P.tau_f) ** n * d[:, None, None]
    assert np.max(np.abs(h[:, act] - want_h[:, act])) < 1e-12 * np.max(np.abs(d))
    cols = slice(1, nx - 1 - n)   # columns the outlet's bounce-back has not reached yet
    want_g = g0 + (1 - 1 / P.tau_t) ** n * dg[:, None, None]
    assert np.max(np.abs(g[:, :, cols] - want_g[:, :, cols])) < 1e-12 * np.max(np.abs(dg))
    # the stress patterns carry no momentum: in and out flow U per boundary node
    ob = o.observe_now()
    assert ob["q_in"] == pytest.approx(P.u_in_x * ny, rel=1e-12)
    assert ob["q_out"] == pytest.approx(P.u_in_x * ny, rel=1e-12)


def _channel_state(tau, s, a, b):
    """A channel between an IRIS wall below (normal +y) and a CORNEA wall above (normal
    -y), at rest, with the non-equilibrium part s SHEAR + a ISO + b NORMAL at every node
    (s a scalar, or one value per column)."""
    nx, ny = 4, 8
    P = A.Params(nx=nx, ny=ny, tau_f=tau, periodic_x=1, check_interval=1000)
    mask = A.channel_mask(nx, ny)
    walls = np.zeros(2 * nx, dtype=A.WALL_DTYPE)
    for x in range(nx):
        walls[x] = (1 * nx + x, A.WALL_IRIS, 0.0, 1.0, [-1.0] * 8)
        walls[nx + x] = ((ny - 2) * nx + x, A.WALL_CORNEA, 0.0, -1.0, [-1.0] * 8)
    o = O.Oracle(P, mask, np.sort(walls, order="node"))
    init_from_fields(o, P, P.p_ref, 0.0, 0.0, P.T_ref)
    h, g = o.populations()
    act = A.active(mask)
    sx = np.broadcast_to(np.asarray(s, float), (nx,))
    d = SHEAR[:, None, None] * sx[None, None, :] + (a * ISO + b * NORMAL)[:, None, None]
    o.set_populations(h + d * act, g)
    return o


@pytest.mark.parametrize("tau", [0.6, 1.3])
def test_wall_shear_is_the_tangential_traction(tau):
    """The deviatoric stress of a node is -(1 - 1/(2 tau)) Pi^neq, and the wall shear stress
    is the part of the traction on the wall's normal that lies along the wall (section 3.6).
    For a state whose non-equilibrium part is s SHEAR + a ISO + b NORMAL, the traction on a
    wall of normal (0, 1) is -(1 - 1/(2 tau)) (4 s, -2 a - 2 b): its tangential magnitude
    (1 - 1/(2 tau)) 4 |s| does not depend on the normal stresses a and b."""
    s = 3e-6
    want = (1 - 1 / (2 * tau)) * 4 * s
    for a, b in ((0.0, 0.0), (5e-6, 0.0), (0.0, -7e-6), (2e-6, 4e-6)):
        ob = _channel_state(tau, s, a, b).observe_now()
        for k in ("wss_iris_mean", "wss_iris_max", "wss_cornea_mean", "wss_cornea_max"):
            assert ob[k] == pytest.approx(want, rel=1e-12), (a, b, k)


def test_wall_shear_mean_and_maximum():
    """With a different shear in every column, the mean and the maximum over a wall are
    those of the per-node values (1 - 1/(2 tau)) 4 |s(x)|."""
    tau = 0.9
    s = np.array([1.0, 3.0, 2.0, 0.5]) * 1e-6
    ob = _channel_state(tau, s, 2e-6, -1e-6).observe_now()
    f = (1 - 1 / (2 * tau)) * 4
    for w in ("iris", "cornea"):
        assert ob[f"wss_{w}_mean"] == pytest.approx(f * np.mean(s), rel=1e-12)
        assert ob[f"wss_{w}_max"] == pytest.approx(f * np.max(s), rel=1e-12)


def test_max_speed_is_the_magnitude():
    """A uniform flow of speed U at 30 degrees: the reported maximum speed is U."""
    n, U = 8, 0.01
    P = A.Params(nx=n, ny=n, periodic_x=1, periodic_y=1, check_interval=1000)
    o = O.Oracle(P, np.full((n, n), A.encode(A.FLUID), np.uint8))
    init_from_fields(o, P, P.p_ref, U * math.cos(math.pi / 6), U * math.sin(math.pi / 6), P.T_ref)
    assert o.observe_now()["u_max"] == pytest.approx(U, rel=1e-12)


def test_non_finite_count_covers_every_field():
    """The count of non-finite nodes reported at a check step covers the flow and the
    thermal populations alike: one NaN in either makes that node count."""
    n = 8
    P = A.Params(nx=n, ny=n, periodic_x=1, periodic_y=1, check_interval=1000)
    o = O.Oracle(P, np.full((n, n), A.encode(A.FLUID), np.uint8))
    init_from_fields(o, P, P.p_ref, 0.0, 0.0, P.T_ref)
    h, g = o.populations()
    g[3, 2, 5] = np.nan
    h[6, 4, 1] = np.inf
    o.set_populations(h, g)
    assert o.observe_now()["n_nonfinite"] == 2


def test_paper_scheme_initial_wall_populations():
    """At t = 0 the paper's scheme gives the populations entering from Dirichlet walls the
    extrapolation of the initial equilibrium: a node at rest beside a wall at T_w receives
    w^T (T_w - T_ref) from it, whatever T_init (section 2.3)."""
    nx, ny = 4, 8
    mask = A.channel_mask(nx, ny, bottom_wall=A.WALL_IRIS, top_wall=A.WALL_CORNEA)
    P = A.Params(nx=nx, ny=ny, periodic_x=1, check_interval=1000, T_ref=0.2, T_init=0.45, T_iris=0.9,
                 T_cornea=0.1, bc_scheme=A.BC_PAPER)
    g = O.Oracle(P, mask).populations()[1]
    w = (1 - P.w0) / 4
    assert np.allclose(g[2, 1, :], w * (P.T_iris - P.T_ref), rtol=0, atol=1e-15)
    assert np.allclose(g[4, ny - 2, :], w * (P.T_cornea - P.T_ref), rtol=0, atol=1e-15)
    assert np.allclose(g[2, 2:ny - 1, :], w * (P.T_init - P.T_ref), rtol=0, atol=1e-15)


def test_interpolation_falls_back_without_a_node_behind():
    """In a one-row channel every wall link with q < 1/2 has no fluid node behind it, so the
    paper's scheme keeps the half-way bounce-back (section 2.3): with q = 0.3 on every wall
    link it steps exactly as the link-wise scheme."""
    nx, ny = 4, 3
    mask = A.channel_mask(nx, ny)
    walls = np.zeros(2 * nx, dtype=A.WALL_DTYPE)
    for x in range(nx):
        walls[x] = (nx + x, A.WALL_IRIS, 0.0, 1.0, [0.3] * 8)
        walls[nx + x] = (nx + x, A.WALL_CORNEA, 0.0, -1.0, [0.3] * 8)
    out = []
    for bc in (A.BC_LINKWISE, A.BC_PAPER):
        P = A.Params(nx=nx, ny=ny, periodic_x=1, check_interval=1000, gbeta=1e-4, gravity_angle=math.pi / 2,
                     T_init=1.0, T0=0.5, bc_scheme=bc)
        o = O.Oracle(P, mask, walls[:nx])
        o.step(50)
        out.append(o.populations()[0][:, 1, :])
    assert np.array_equal(out[0], out[1])


def test_iop_is_the_mean_over_the_chamber_fluid():
    """The IOP is the mean pressure of the chamber's fluid, not of the meshwork (section
    2.2.4).  Uniform flow U through a porous slab near the inlet of a periodic duct: the
    pressure is flat at p_out + (nu/K) h U upstream of the slab and at p_out downstream
    (to O(U^2)), so the gauge IOP is that drop times the upstream share of the fluid nodes;
    counting the slab's nodes, whose pressure falls linearly, would give a different share."""
    nx, ny, U, c0, c1, K = 40, 3, 1e-4, 8, 18, 2.0
    m = np.full((ny, nx), A.encode(A.FLUID), np.uint8)
    m[:, c0:c1] = A.encode(A.POROUS)
    m[:, 0] = A.encode(A.INLET)
    m[:, nx - 1] = A.encode(A.OUTLET)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, periodic_y=1, check_interval=1000, u_in_x=U, K=K)
    o = O.Oracle(P, m)
    o.step(60000)
    drop = 0.1 / K * (c1 - c0) * U
    n_up, n_down = c0 - 1, nx - 1 - c1
    want = drop * n_up / (n_up + n_down)
    with_slab = drop * (n_up + (c1 - c0) / 2) / (n_up + (c1 - c0) + n_down)
    got = o.observables()["iop_gauge"]
    assert got == pytest.approx(want, rel=2e-3)
    assert abs(with_slab - want) > 0.1 * want


def test_residual_is_per_time_step():
    """The residual reported at a check step is the relative change of the field over the
    check interval divided by its D steps.  A shear wave decaying as exp(-nu k^2 t) gives
    (exp(nu k^2 D) - 1) / D for the velocity, a heat mode decaying as exp(-theta k^2 t)
    (exp(theta k^2 D) - 1) / D for the temperature."""
    n, D = 64, 50
    tau, tau_t, w0 = 0.8, 0.75, 1.0 / 3.0
    P = A.Params(nx=n, ny=n, tau_f=tau, tau_t=tau_t, w0=w0, periodic_x=1, periodic_y=1, check_interval=D)
    o = O.Oracle(P, np.full((n, n), A.encode(A.FLUID), np.uint8))
    k = 2 * math.pi / n
    y = np.arange(n)[:, None] * np.ones((1, n))
    x = np.ones((n, 1)) * np.arange(n)[None, :]
    init_from_fields(o, P, P.p_ref, 1e-6 * np.sin(k * y), 0.0, P.T_ref + 0.1 * np.sin(k * x))
    o.step(10 * D)
    ob = o.observables()
    nu = (2 * tau - 1) / 6
    theta = (1 - w0) * (2 * tau_t - 1) / 4
    assert ob["resid_u"] == pytest.approx((math.exp(nu * k * k * D) - 1) / D, rel=5e-3)
    assert ob["resid_T"] == pytest.approx((math.exp(theta * k * k * D) - 1) / D, rel=5e-3)
