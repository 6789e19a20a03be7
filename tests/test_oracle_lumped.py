"""Pins of the oracle's lumped trabecular-meshwork outlet (section 2.2.4 with eq. 2 and 4;
section 2.3, the coupling paragraph; section 3.1, Fig. 2; Tables 4-6).

The meshwork is not resolved: its pressure falls linearly over the thickness h_TM from the
IOP to the Schlemm's-canal pressure p_sc, so Darcy's law gives the seepage speed
u_s = (K/mu)(IOP - p_sc)/h_TM, applied as a velocity condition on the chamber and
re-evaluated at every check step.

What fixes the results independently of the oracle's own code:

* Steady state: the flow mass of the chamber is constant, so the outflow equals the
  secretion inflow Q_in; the outflow is u_s times the outflow area A (each link into an
  outlet node moves 6 w_i e_i.n u_s), so IOP - p_sc = mu h_TM Q_in / (K A) exactly.  Q_in
  and A are counted here by brute force from the mask.
* Transient: the chamber's flow mass (5/3) N dp relaxes by the factor 1 - D r per check
  interval D, with r = 3 A K / (5 N mu h_TM).
* The paper's Tables 4-6 follow the same law (IOP - p_0 proportional to the inflow, to
  1/K and to mu) within their printed scatter.
* Fig. 2: starting above or below, the IOP settles on the same value (negative feedback).
"""
import os

import numpy as np
import pytest

import aqinputs as A
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def _eye():
    return A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2, tm="lumped")


def _counts(mask, p):
    """Brute-force outflow area A = sum 6 w_i e_i.n over links into OUTLET nodes, inflow
    Q_in = sum 6 w_i |e_i.u_in| over links into INLET nodes, active node count N."""
    act = A.active(mask)
    cls = mask & 7
    d = (mask >> 3) & 3
    area = q_in = 0.0
    ny, nx = mask.shape
    for y, x in zip(*np.nonzero(act)):
        for i in range(1, 9):
            yy, xx = y + E[i][1], x + E[i][0]
            if cls[yy, xx] == A.OUTLET:
                n = E[d[yy, xx] + 1]
                area += 6 * W[i] * (E[i][0] * n[0] + E[i][1] * n[1])
            elif cls[yy, xx] == A.INLET:
                q_in += 6 * W[i] * abs(E[i][0] * p.u_in_x + E[i][1] * p.u_in_y)
    return area, q_in, int(act.sum())


def _params(geo, **kw):
    return A.eye_params(96, 48, geo, Ra=0.0, Da=1e-3, check_interval=100, tm="lumped", **kw)


def _to_steady(p, mask, walls, tol=1e-10, max_intervals=2000):
    o = O.Oracle(p, mask, walls)
    for _ in range(max_intervals):
        o.step(p.check_interval)
        ob = o.observables()
        if ob["resid_u"] < tol:
            return ob
    raise AssertionError(f"not steady: {ob}")


def _nu(p):
    return (2 * p.tau_f - 1) / 6


def test_lumped_mask_and_outflow_area():
    """The lumped mask keeps the chamber of the resolved one, turns both meshwork blocks
    into OUTLET nodes pointing away from the chamber, and leaves a positive outflow area."""
    m0, _, _ = A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2)
    m1, walls, geo = _eye()
    assert np.array_equal(m1 & 7, (m1 & 7)[:, ::-1])             # classes mirror symmetric
    assert np.array_equal(A.active(m1), (m0 & 7) == A.FLUID)      # the meshwork is no longer resolved
    out = (m1 & 7) == A.OUTLET
    left = out[:, : m1.shape[1] // 2]
    assert np.all(((m1 >> 3) & 3)[:, : m1.shape[1] // 2][left] == A.DIR_MX)
    assert np.all(((m1 >> 3) & 3)[:, m1.shape[1] // 2:][out[:, m1.shape[1] // 2:]] == A.DIR_PX)
    area, q_in, n = _counts(m1, _params(geo))
    assert area > 0 and q_in == pytest.approx(2 * 1e-4, rel=1e-12)   # pupil gap of 2 cells


@pytest.mark.parametrize("canal", [0.0, -3e-5])
def test_steady_iop_closed_form(canal):
    """IOP - p_sc = mu h Q_in / (K A) at the steady state, and the outflow equals the inflow;
    also with the canal pressure p_sc below the reference pressure p_ref."""
    mask, walls, geo = _eye()
    p = _params(geo, p_sc=1.0 / 3.0 + canal)
    area, q_in, n = _counts(mask, p)
    ob = _to_steady(p, mask, walls)
    expect = _nu(p) * p.h_tm * q_in / (p.K_tm * area)
    assert ob["p_mean_fluid"] - p.p_sc == pytest.approx(expect, rel=1e-6)
    assert ob["q_out"] == pytest.approx(q_in, rel=1e-6)
    assert ob["u_seep"] * area == pytest.approx(q_in, rel=1e-6)
    assert ob["u_seep"] == pytest.approx(p.K_tm / _nu(p) * (ob["p_mean_fluid"] - p.p_sc) / p.h_tm, rel=1e-14)


@pytest.mark.parametrize("dr", [0.5, 0.8])
def test_relaxation_factor_per_check_interval(dr):
    """The IOP error shrinks by 1 - D r per check interval (explicit coupling)."""
    mask, walls, geo = _eye()
    p = _params(geo)
    area, q_in, n = _counts(mask, p)
    r = 3 * area * p.K_tm / (5 * n * _nu(p) * p.h_tm)
    p.K_tm *= dr / (p.check_interval * r)
    star = _nu(p) * p.h_tm * q_in / (p.K_tm * area)
    o = O.Oracle(p, mask, walls)
    err = []
    for _ in range(6):
        o.step(p.check_interval)
        err.append(o.observables()["p_mean_fluid"] - p.p_sc - star)
    # while the mass mode dominates (later the flow field's own slower settling shows)
    ratios = [err[k + 1] / err[k] for k in range(5)]
    assert np.allclose(ratios, 1 - dr, atol=1e-3), ratios


def test_fig2_iop_settles_from_above_and_below():
    """Fig. 2: initial pressures on either side of the steady IOP converge to it, each
    monotonically (D r < 1), and to the same value."""
    mask, walls, geo = _eye()
    base = _params(geo)
    area, q_in, n = _counts(mask, base)
    star = _nu(base) * base.h_tm * q_in / (base.K_tm * area)
    finals = []
    for sign in (+1, -1):
        p = _params(geo)
        p.p_init = p.p_sc + star * (1 + sign * 0.01)
        o = O.Oracle(p, mask, walls)
        prev = None
        for _ in range(60):
            o.step(p.check_interval)
            e = o.observables()["p_mean_fluid"] - p.p_sc - star
            if prev is not None and abs(prev) > 1e-3 * star:
                assert abs(e) < abs(prev)
            prev = e
        finals.append(o.observables()["p_mean_fluid"])
    assert finals[0] == pytest.approx(finals[1], rel=1e-9)
    assert finals[0] - base.p_sc == pytest.approx(star, rel=1e-5)


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name))


def test_tables_4_5_6_scaling():
    """The steady IOP rise of the oracle scales with the inflow, 1/K and mu as the closed
    form says, and the paper's printed values follow the same scalings: Table 5 within
    0.5% (its (IOP - 1200) K varies by 0.4%), Table 4 (healthy column) within 1.5% and
    Table 6 (healthy column) within 2%."""
    mask, walls, geo = _eye()
    base = _params(geo)
    rise0 = _to_steady(base, mask, walls)["p_mean_fluid"] - base.p_sc

    def rise(**change):
        p = _params(geo)
        for k, v in change.items():
            setattr(p, k, v)
        return _to_steady(p, mask, walls)["p_mean_fluid"] - p.p_sc

    # Table 5: K from 1.19e-14 to 1.99e-15 (rows 0.25 and 0.15): rise scales as 1/K
    t5 = _golden("table5_iop_vs_permeability.txt")
    k_ratio = t5[6, 1] / t5[2, 1]
    mine = rise(K_tm=base.K_tm * k_ratio) / rise0
    assert mine == pytest.approx(1 / k_ratio, rel=1e-5)
    paper = (t5[6, 2] - 1200.0) / (t5[2, 2] - 1200.0)
    assert mine == pytest.approx(paper, rel=5e-3)
    for row in t5:                       # every row of Table 5 on the 1/K law
        assert (row[2] - 1200.0) * row[1] == pytest.approx((t5[0, 2] - 1200.0) * t5[0, 1], rel=5e-3)
    # Table 4: doubling the secretion rate doubles the rise
    t4 = _golden("table4_iop_vs_inflow.txt")
    mine = rise(u_in_y=2 * base.u_in_y) / rise0
    assert mine == pytest.approx(2.0, rel=1e-5)
    paper = (t4[t4[:, 0] == 2.0, 2][0] - 1200.0) / (t4[t4[:, 0] == 1.0, 2][0] - 1200.0)
    assert mine == pytest.approx(paper, rel=1.5e-2)
    # Table 6: the rise is proportional to mu (nu at unit density)
    t6 = _golden("table6_iop_vs_viscosity.txt")
    mu_ratio = t6[-1, 0] / t6[0, 0]
    nu1 = _nu(base) * mu_ratio
    mine = rise(tau_f=0.5 + 3 * nu1) / rise0
    assert mine == pytest.approx(mu_ratio, rel=1e-5)
    paper = (t6[-1, 1] - 1200.0) / (t6[0, 1] - 1200.0)
    assert mine == pytest.approx(paper, rel=2e-2)


def test_calibration_loop_reaches_closed_form_thickness():
    """The healthy-eye procedure of section 3.1: adjust the meshwork thickness until the
    steady IOP is the target.  With warm restarts (new thickness, same state) and the
    library's update rule, the loop lands on h* = target K A / (mu Q_in) in two or three
    rounds."""
    from paper_2102_12663_amd.serve import thickness_update
    mask, walls, geo = _eye()
    p = _params(geo)
    area, q_in, n = _counts(mask, p)
    target = 1.3 * _nu(p) * p.h_tm * q_in / (p.K_tm * area)
    h_star = target * p.K_tm * area / (_nu(p) * q_in)
    o = O.Oracle(p, mask, walls)
    h, history, rounds = p.h_tm, [], 0
    while True:
        rounds += 1
        for _ in range(3000):
            o.step(p.check_interval)
            ob = o.observables()
            if ob["resid_u"] < 1e-11:
                break
        rise = ob["p_mean_fluid"] - p.p_sc
        if abs(rise / target - 1) < 1e-8 or rounds >= 5:
            break
        h = thickness_update(h, rise, target, history)
        o.set_outlet(p.K_tm, h, p.p_sc)
    assert rounds <= 3
    assert h == pytest.approx(h_star, rel=2e-8)


def _lumped_duct(bc, U=1e-3, nx=24, ny=4, K_tm=0.05, h_tm=3.0, D=10, along_y=False):
    """Duct periodic across: INLET column (velocity U along x), lumped OUTLET column
    draining along +x, no walls; or the same duct turned to run along +y."""
    m = np.full((ny, nx), A.encode(A.FLUID), np.uint8)
    m[:, 0] = A.encode(A.INLET)
    m[:, nx - 1] = A.encode(A.OUTLET, 0)
    kw = dict(periodic_y=1, u_in_x=U)
    if along_y:
        m = np.ascontiguousarray(m.T)
        m[nx - 1, :] = A.encode(A.OUTLET, 1)
        nx, ny = ny, nx
        kw = dict(periodic_x=1, u_in_y=U)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, check_interval=D, bc_scheme=bc, outlet_mode=A.OUTLET_LUMPED,
                 K_tm=K_tm, h_tm=h_tm, p_sc=1.0 / 3.0 - 2e-5, p_init=1.0 / 3.0, **kw)
    return m, P


@pytest.mark.parametrize("along_y", [False, True])
@pytest.mark.parametrize("bc", [A.BC_LINKWISE, A.BC_PAPER])
def test_lumped_duct_closed_form(bc, along_y):
    """Plug flow U into a duct drained by the lumped meshwork: the steady state is the
    uniform flow with u_s = U, so IOP - p_sc = mu h U / K exactly (eq. 4 over the meshwork),
    with the link-wise moving wall and with the paper's extrapolation at the outlet, for a
    meshwork draining along x or along y."""
    m, P = _lumped_duct(bc, along_y=along_y)
    o = O.Oracle(P, m).step(30000)
    ob = o.observables()
    U = max(P.u_in_x, P.u_in_y)
    assert ob["p_mean_fluid"] - P.p_sc == pytest.approx(_nu(P) * P.h_tm * U / P.K_tm, rel=1e-12)
    assert ob["u_seep"] == pytest.approx(U, rel=1e-12)
    assert ob["q_out"] == pytest.approx(ob["q_in"], rel=1e-12)


def test_first_interval_drains_at_the_initial_pressure():
    """Before the first check step the seepage speed is that of p_init, and the moving-wall
    outlet drains u_s per outlet node (6 w_i e_i.n summed over the three outgoing links is
    1): the outflow of the last step of the first interval is (K/mu)(p_init - p_sc)/h per node."""
    m, P = _lumped_duct(A.BC_LINKWISE)
    ny = m.shape[0]
    ob = O.Oracle(P, m).step(P.check_interval).observables()
    assert ob["q_out"] == pytest.approx(P.K_tm / _nu(P) * (P.p_init - P.p_sc) / P.h_tm * ny, rel=1e-12)


def test_recalibration_drains_at_the_last_iop():
    """A new thickness takes effect at once, with the seepage speed of the IOP of the last
    check step (the warm restart of the calibration loop, section 3.1)."""
    m, P = _lumped_duct(A.BC_LINKWISE)
    ny = m.shape[0]
    o = O.Oracle(P, m).step(3 * P.check_interval)
    iop = o.observables()["p_mean_fluid"]
    h2 = 1.7 * P.h_tm
    o.set_outlet(P.K_tm, h2, P.p_sc)
    o.step(1)
    ob = o.observe_now()
    assert ob["q_out"] == pytest.approx(P.K_tm / _nu(P) * (iop - P.p_sc) / h2 * ny, rel=1e-12)
