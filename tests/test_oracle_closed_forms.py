"""Pins of the oracle's full time step against closed forms and conservation laws.

The continuum targets are the paper's eq. 1-4 and eq. 16 (section 2.2) with the viscosity
and diffusivity of eq. 10 and eq. 14; the lattice checks are exact discrete balances that
hold for any correct implementation of eq. 6-17 with link-wise boundaries.
"""
import math

import numpy as np
import pytest

import aqinputs as A
import oracle as O
from _oracle_util import init_from_fields

EX = np.array([1, 0, -1, 0, 1, -1, -1, 1], float)
EY = np.array([0, 1, 0, -1, 1, 1, -1, -1], float)


def _decay_rate(orc, field_index, warm, n, ref=0.0):
    orc.step(warm)
    a0 = np.nanmax(np.abs(orc.fields()[field_index] - ref))
    orc.step(n)
    a1 = np.nanmax(np.abs(orc.fields()[field_index] - ref))
    return -math.log(a1 / a0) / n


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_shear_wave_viscosity(tau):
    """A periodic shear wave u_x = A sin(k y) decays as exp(-nu k^2 t) with
    nu = (2 tau - 1)/6 (eq. 10).  The lattice error is second order in k."""
    errs = []
    for ny in (32, 64):
        nx = 4
        P = A.Params(nx=nx, ny=ny, tau_f=tau, periodic_x=1, periodic_y=1, check_interval=1000)
        o = O.Oracle(P, np.full((ny, nx), A.encode(A.FLUID), np.uint8))
        k = 2 * math.pi / ny
        y = np.arange(ny)[:, None] * np.ones((1, nx))
        init_from_fields(o, P, P.p_ref, 1e-3 * np.sin(k * y), 0.0, P.T0)
        nu = (2 * tau - 1) / 6
        errs.append(_decay_rate(o, 1, 200, 1000) / (k * k) / nu - 1)
    assert abs(errs[1]) < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("w0", [0.0, 1.0 / 3.0])
@pytest.mark.parametrize("tau_t", [0.6, 0.85])
def test_heat_mode_diffusivity(w0, tau_t):
    """A periodic temperature mode at rest decays as exp(-theta k^2 t) with
    theta = (1-w0)(2 tau_T - 1)/4 (eq. 14 at w0 = 0, eq. 3)."""
    errs = []
    for nx in (32, 64):
        ny = 4
        P = A.Params(nx=nx, ny=ny, tau_t=tau_t, w0=w0, periodic_x=1, periodic_y=1, check_interval=1000)
        o = O.Oracle(P, np.full((ny, nx), A.encode(A.FLUID), np.uint8))
        k = 2 * math.pi / nx
        x = np.ones((ny, 1)) * np.arange(nx)[None, :]
        init_from_fields(o, P, P.p_ref, 0.0, 0.0, P.T_ref + 0.1 * np.sin(k * x))
        th = (1 - w0) * (2 * tau_t - 1) / 4
        errs.append(_decay_rate(o, 3, 200, 1000, ref=P.T_ref) / (k * k) / th - 1)
    assert abs(errs[1]) < 1e-3
    if abs(errs[1]) > 1e-5:
        assert 3.5 < errs[0] / errs[1] < 4.5


def test_heat_mode_advection():
    """In a uniform flow U the temperature mode is carried at speed U (eq. 3): after t
    steps its phase has moved by U t."""
    nx, ny, U = 64, 4, 0.02
    P = A.Params(nx=nx, ny=ny, tau_t=0.8, periodic_x=1, periodic_y=1, check_interval=1000)
    o = O.Oracle(P, np.full((ny, nx), A.encode(A.FLUID), np.uint8))
    k = 2 * math.pi / nx
    x = np.ones((ny, 1)) * np.arange(nx)[None, :]
    init_from_fields(o, P, P.p_ref, U, 0.0, P.T_ref + 0.1 * np.sin(k * x))
    t = 800
    o.step(t)
    T = o.fields()[3][1] - P.T_ref
    z = np.sum(T * np.exp(-1j * k * np.arange(nx)))
    shift = (-np.angle(z) - math.pi / 2) / k       # sin(k(x - s)) has phase -pi/2 - k s
    shift = (shift + nx / 2) % nx - nx / 2
    assert shift == pytest.approx((U * t) % nx if (U * t) % nx < nx / 2 else (U * t) % nx - nx, abs=0.05)


def _poiseuille(ny, tau=0.8, F=1e-6):
    nx, H = 4, ny - 2
    P = A.Params(nx=nx, ny=ny, tau_f=tau, periodic_x=1, check_interval=1000, gbeta=F,
                 gravity_angle=math.pi / 2, T_init=1.5, T0=0.5)
    m = A.channel_mask(nx, ny)
    walls = np.zeros(2 * nx, dtype=A.WALL_DTYPE)
    for x in range(nx):
        walls[x] = (1 * nx + x, A.WALL_IRIS, 0.0, 1.0, [-1.0] * 8)
        walls[nx + x] = ((ny - 2) * nx + x, A.WALL_CORNEA, 0.0, -1.0, [-1.0] * 8)
    o = O.Oracle(P, m, np.sort(walls, order="node"))
    nu = (2 * tau - 1) / 6
    o.step((int(8 * H * H / nu) // 1000 + 1) * 1000)
    return o, P, F, nu, H


def test_plane_poiseuille_buoyancy_driven():
    """Uniform T != T0 with gravity along -x gives a uniform force F = g beta (T - T0)
    along +x (eq. 16); between no-slip walls the steady flow is the parabola
    u = F/(2 nu) (y - 1/2)(ny - 3/2 - y).  The lattice solution is exactly parabolic
    (third difference 0, nu * second difference = -F) and converges to the continuum
    profile at second order."""
    errs = []
    for ny in (16, 32):
        o, P, F, nu, H = _poiseuille(ny, F=1e-6 * (16 / ny) ** 2)
        u = o.fields()[1][1:ny - 1, 1]
        y = np.arange(1, ny - 1)
        exact = F / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
        d2 = u[2:] - 2 * u[1:-1] + u[:-2]
        assert np.max(np.abs(nu * d2 / F + 1)) < 1e-10
        assert np.max(np.abs(np.diff(u, 3))) < 1e-12 * np.max(u)
        errs.append(np.max(np.abs(u - exact)) / np.max(exact))
    assert errs[1] < 5e-4
    assert 3.5 < errs[0] / errs[1] < 5.0


def test_wall_shear_stress_momentum_balance():
    """At steady state the force on the fluid column is carried by the two walls, and the
    shear stress is linear across the channel: at the first node (half a cell from the
    wall) the wall-shear-stress reduction must give F (H/2 - 1/2) on both walls."""
    o, P, F, nu, H = _poiseuille(16)
    ob = o.observables()
    want = F * (H / 2 - 0.5)
    assert ob["wss_iris_mean"] == pytest.approx(want, rel=1e-10)
    assert ob["wss_cornea_mean"] == pytest.approx(want, rel=1e-10)
    assert ob["wss_cornea_max"] == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("w0", [0.0, 1.0 / 3.0])
def test_linear_conduction(w0):
    """Between a hot floor (T = 1) and a cold lid (T = 0) at rest, the steady temperature
    is linear (eq. 3): T = 1 - (y - 1/2)/(ny - 2) with the walls half a cell out.  The
    thermal anti-bounce-back is exact for linear profiles."""
    ny, nx, tau_t = 18, 4, 0.9
    P = A.Params(nx=nx, ny=ny, tau_t=tau_t, w0=w0, periodic_x=1, check_interval=1000)
    o = O.Oracle(P, A.channel_mask(nx, ny, bottom_wall=A.WALL_IRIS, top_wall=A.WALL_CORNEA))
    th = (1 - w0) * (2 * tau_t - 1) / 4
    o.step((int(40 * (ny - 2) ** 2 / th / math.pi ** 2) // 1000 + 1) * 1000)
    T = o.fields()[3][1:ny - 1, 1]
    y = np.arange(1, ny - 1)
    np.testing.assert_allclose(T, 1 - (y - 0.5) / (ny - 2), rtol=0, atol=1e-12)


@pytest.mark.parametrize("K", [0.5, 2.0, 8.0])
def test_darcy_slab_pressure_drop(K):
    """Uniform flow U through a porous slab of width h (periodic across): the pressure
    drop equals the Darcy drag (nu/K) h U (eq. 4), outside the slab the pressure is flat,
    and the Darcy velocity in the slab equals the inflow U."""
    nx, ny, U, c0, c1 = 40, 3, 1e-4, 15, 25
    m = np.full((ny, nx), A.encode(A.FLUID), np.uint8)
    m[:, c0:c1] = A.encode(A.POROUS)
    m[:, 0] = A.encode(A.INLET)
    m[:, nx - 1] = A.encode(A.OUTLET)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, periodic_y=1, check_interval=1000, u_in_x=U, K=K)
    o = O.Oracle(P, m)
    o.step(60000)
    dp, ux, uy, T = o.fields()
    nu = 0.1
    drop = np.mean(dp[:, 10]) - np.mean(dp[:, 30])
    assert drop == pytest.approx(nu / K * (c1 - c0) * U, rel=1e-8)
    assert abs(dp[1, 5] - dp[1, 8]) < 1e-12 * drop
    uD = ux[1, 20] / (1 + nu / (2 * K))
    assert uD == pytest.approx(U, rel=1e-8)
    ob = o.observables()
    assert ob["q_out"] == pytest.approx(ob["q_in"], rel=1e-8)


@pytest.mark.parametrize("sqK", [2.0, 4.0])
def test_brinkman_channel(sqK):
    """A porous channel driven by a uniform force G has the Brinkman profile
    u = (G K/nu)[1 - cosh((y - yc)/sqrt K) / cosh(H/(2 sqrt K))]."""
    nx, ny, G = 4, 34, 1e-6
    H, K = ny - 2, sqK ** 2
    m = A.channel_mask(nx, ny)
    m[1:ny - 1, :] = A.encode(A.POROUS)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, periodic_x=1, check_interval=1000, gbeta=G,
                 gravity_angle=math.pi / 2, T_init=1.5, K=K)
    o = O.Oracle(P, m)
    o.step(40000)
    u = o.fields()[1][:, 1]
    nu = 0.1
    uD = (u + G / 2) / (1 + nu / (2 * K))
    y = np.arange(ny)
    exact = G * K / nu * (1 - np.cosh((y - (ny - 1) / 2) / sqK) / np.cosh(H / (2 * sqK)))
    assert np.max(np.abs(uD[1:-1] - exact[1:-1])) / np.max(exact) < 1e-2


def test_closed_box_conservation():
    """In a closed box with bounce-back walls, adiabatic thermal walls, buoyancy and a
    Darcy patch, sum h and sum g are invariant (collision conserves them per node, the
    force has zero mass, bounce-back permutes populations)."""
    nx, ny = 24, 16
    m = A.box_mask(nx, ny, porous_rect=(5, 9, 3, 8))
    P = A.Params(nx=nx, ny=ny, tau_f=0.7, tau_t=0.8, gbeta=1e-3, check_interval=1, K=2.0)
    o = O.Oracle(P, m)
    rng = np.random.default_rng(0)
    h = rng.normal(0, 1e-4, (8, ny, nx))
    g = rng.normal(0, 1e-2, (5, ny, nx))
    o.set_populations(h, g)
    o.step(1)
    a = o.observables()
    o.step(2000)
    b = o.observables()
    scale_h = np.sum(np.abs(h[:, A.active(m)]))
    scale_g = np.sum(np.abs(g[:, A.active(m)]))
    assert abs(b["mass_flow"] - a["mass_flow"]) < 1e-13 * scale_h
    assert abs(b["mass_thermal"] - a["mass_thermal"]) < 1e-13 * scale_g
    assert b["n_nonfinite"] == 0


def test_periodic_momentum_conservation():
    """Without force or walls the total momentum sum_x sum_i e_i h_i is invariant."""
    nx, ny = 16, 12
    P = A.Params(nx=nx, ny=ny, tau_f=0.7, periodic_x=1, periodic_y=1, check_interval=1)
    o = O.Oracle(P, np.full((ny, nx), A.encode(A.FLUID), np.uint8))
    rng = np.random.default_rng(5)
    h0 = rng.normal(0, 1e-3, (8, ny, nx))
    o.set_populations(h0, np.zeros((5, ny, nx)))

    def mom():
        h, _ = o.populations()
        return np.array([np.einsum("q,qyx->", EX, h), np.einsum("q,qyx->", EY, h), h.sum()])

    a = mom()
    o.step(1000)
    np.testing.assert_allclose(mom(), a, rtol=0, atol=1e-13 * np.sum(np.abs(h0)))


def _rb_growth(fac, ny=19):
    """Growth rate (in units of theta/H^2) of a small roll in a layer heated from below."""
    H = ny - 2
    nx = int(round(2.016 * H))
    nu, th = 0.1, (2.0 / 3.0) * 0.4 / 4
    gb = fac * 1707.76 * nu * th / H ** 3
    m = A.channel_mask(nx, ny, bottom_wall=A.WALL_IRIS, top_wall=A.WALL_CORNEA)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, tau_t=0.7, periodic_x=1, gbeta=gb, check_interval=1000)
    o = O.Oracle(P, m)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    x = np.ones((ny, 1)) * np.arange(nx)[None, :]
    T = 1 - (y - 0.5) / H + 1e-3 * np.sin(math.pi * (y - 0.5) / H) * np.cos(2 * math.pi * x / nx)
    init_from_fields(o, P, P.p_ref, 0.0, 0.0, T)
    n = int(0.5 * H * H / th)
    o.step(4 * n)
    a = np.nanmax(np.abs(o.fields()[1]))
    o.step(2 * n)
    b = np.nanmax(np.abs(o.fields()[1]))
    return math.log(b / a) / (2 * n) * H * H / th


def test_rayleigh_benard_onset():
    """Buoyancy coupling magnitude (eq. 5, 15-17) with the thermal walls: a layer heated
    from below between no-slip walls becomes unstable at Ra_c = 1707.76 (rigid-rigid
    linear stability).  At H = 17 the lattice threshold must lie within 8% of Ra_c."""
    lo, hi = 0.95, 1.15
    glo, ghi = _rb_growth(lo), _rb_growth(hi)
    assert glo < 0 < ghi
    fac = lo - glo * (hi - lo) / (ghi - glo)
    assert abs(fac - 1) < 0.08


def _poiseuille_offgrid(ny, qb, qt, scheme, tau=0.8, F=1e-6):
    """Channel with its walls off the half-way lines: at y_b = 1 - qb below row 1 and at
    y_t = ny - 2 + qt above row ny - 2 (the link fractions of the wall list)."""
    nx = 4
    P = A.Params(nx=nx, ny=ny, tau_f=tau, periodic_x=1, check_interval=1000, gbeta=F,
                 gravity_angle=math.pi / 2, T_init=1.5, T0=0.5, bc_scheme=scheme)
    m = A.channel_mask(nx, ny)
    walls = np.zeros(2 * nx, dtype=A.WALL_DTYPE)
    down = [-1, -1, -1, qb, -1, -1, qb, qb]          # links 4, 7, 8 point to the bottom wall
    up = [-1, qt, -1, -1, qt, qt, -1, -1]            # links 2, 5, 6 point to the top wall
    for x in range(nx):
        walls[x] = (1 * nx + x, A.WALL_IRIS, 0.0, 1.0, down)
        walls[nx + x] = ((ny - 2) * nx + x, A.WALL_CORNEA, 0.0, -1.0, up)
    o = O.Oracle(P, m, np.sort(walls, order="node"))
    nu = (2 * tau - 1) / 6
    H = ny - 3 + qb + qt
    o.step((int(10 * H * H / nu) // 1000 + 1) * 1000)
    y = np.arange(1, ny - 1)
    exact = F / (2 * nu) * (y - (1 - qb)) * (ny - 2 + qt - y)
    u = o.fields()[1][1:ny - 1, 1]
    return np.max(np.abs(u - exact)) / np.max(exact)


def test_interpolated_bounce_back_places_the_wall():
    """The paper's wall scheme (section 2.3, Bouzidi et al.): with walls a fraction q of a
    link from the nodes, the steady channel flow converges at second order to the parabola
    between the true wall positions, while half-way bounce-back (the walls it assumes are at
    q = 1/2) misses it by far more."""
    qb, qt = 0.3, 0.8
    errs = [_poiseuille_offgrid(ny, qb, qt, A.BC_PAPER, F=1e-6 * (16 / ny) ** 2) for ny in (16, 32)]
    half = _poiseuille_offgrid(32, qb, qt, A.BC_LINKWISE, F=1e-6 * (16 / 32) ** 2)
    assert errs[1] < 3e-3
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert half > 10 * errs[1]


def test_interpolated_bounce_back_at_half_is_half_way():
    """q = 1/2 on every wall link reproduces the half-way bounce-back exactly."""
    a = _poiseuille_offgrid(16, 0.5, 0.5, A.BC_PAPER)
    b = _poiseuille_offgrid(16, 0.5, 0.5, A.BC_LINKWISE)
    assert a == b


def _plug(scheme, steps=300, U=0.02, nx=24, ny=6):
    """Duct periodic in y: INLET column x = 0 (velocity U along x), OUTLET column
    x = nx - 1 (p_out), no walls; started from the uniform flow U at p = p_out."""
    mask = np.full((ny, nx), A.encode(A.FLUID), np.uint8)
    mask[:, 0] = A.encode(A.INLET)
    mask[:, nx - 1] = A.encode(A.OUTLET)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, periodic_y=1, u_in_x=U, p_out=1.0 / 3.0 + 1e-4,
                 check_interval=100, bc_scheme=scheme)
    o = O.Oracle(P, mask)
    init_from_fields(o, P, P.p_out, U, 0.0, P.T_ref)
    h0 = o.populations()[0].copy()
    o.step(steps)
    act = A.active(mask)
    return np.max(np.abs(o.populations()[0][:, act] - h0[:, act])) / np.max(np.abs(h0[:, act]))


def test_extrapolated_inlet_outlet_keep_uniform_flow():
    """Guo et al.'s non-equilibrium extrapolation (the paper's inlet/outlet scheme, section
    2.3): uniform flow at the outlet pressure is an exact fixed point (the inlet gives the
    equilibrium at u_in and the fluid's pressure, the outlet at p_out and the fluid's
    velocity, with no non-equilibrium part), while the link-wise outlet, which drops the
    O(u^2) term, disturbs it."""
    assert _plug(A.BC_PAPER) < 1e-13
    assert _plug(A.BC_LINKWISE) > 1e-6


@pytest.mark.parametrize("scheme,ends", [(A.BC_PAPER, (0.0, 0.0)), (A.BC_LINKWISE, (0.5, 0.5))])
def test_thermal_walls_place_the_temperature(scheme, ends):
    """Conduction between Dirichlet walls (T = 1 below, 0 above): the extrapolation of the
    paper's scheme imposes the wall temperature on the solid rows themselves (T linear from
    y = 0 to y = ny - 1), the link-wise anti-bounce-back half a link inside them; both
    profiles are exactly linear.  The walls are at rest whatever the inlet velocity (set
    here although the channel has no inlet)."""
    nx, ny = 4, 12
    mask = A.channel_mask(nx, ny, bottom_wall=A.WALL_IRIS, top_wall=A.WALL_CORNEA)
    P = A.Params(nx=nx, ny=ny, tau_t=0.9, periodic_x=1, check_interval=1000, T_iris=1.0, T_cornea=0.0,
                 bc_scheme=scheme, u_in_x=0.01, u_in_y=0.02)
    o = O.Oracle(P, mask)
    o.step(40000)
    T = o.fields()[3][1:ny - 1, 1]
    y = np.arange(1, ny - 1)
    y0, y1 = ends[0], ny - 1 - ends[1]
    assert np.max(np.abs(T - (1.0 - (y - y0) / (y1 - y0)))) < 1e-12
