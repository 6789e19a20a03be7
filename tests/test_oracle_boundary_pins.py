"""Pins of the oracle's outlet-pressure and inlet-temperature branches.

Both are exact consequences of the model (section 2.3): the incompressible equilibrium of
eq. 7 is affine in p with sum_i e_i lambda_i = 0, so a uniform pressure shift is invisible
to the velocity; and a closed adiabatic box whose only Dirichlet links lead into INLET
cells must settle at the inlet temperature.
"""
import numpy as np
import pytest

import aqinputs as A
import oracle as O


def _run_config0(delta, scheme, steps=1000):
    p, mask, walls, geo = A.config0()
    p.bc_scheme = scheme
    p.p_out = p.p_ref + delta
    p.p_init = p.p_ref + delta
    o = O.Oracle(p, mask, walls).step(steps)
    return o.fields(), o.observables(), A.active(mask)


@pytest.mark.parametrize("scheme", [A.BC_LINKWISE, A.BC_PAPER])
def test_pressure_shift_invariance(scheme):
    """Shifting the outlet pressure and the initial pressure together by delta shifts every
    flow population by lambda_i delta and nothing else: eq. 9 then gives the same u and
    p - p_ref larger by exactly delta, the collision (eq. 6-8) and every link rule map the
    shifted state onto the shifted state, and the IOP measured against p_out is unchanged.
    A wrong coefficient of the outlet's p_out term (anti-bounce-back: 2 lambda_i (p_out -
    p_ref); extrapolation: lambda_i (p_out - p_ref) inside h^eq) breaks all three."""
    delta = 1e-4
    (dp0, ux0, uy0, T0), ob0, act = _run_config0(0.0, scheme)
    (dp1, ux1, uy1, T1), ob1, _ = _run_config0(delta, scheme)
    umax = max(np.max(np.abs(ux0[act])), np.max(np.abs(uy0[act])))
    assert umax > 1e-6                      # a flowing state, not the trivial one
    assert np.max(np.abs(ux1[act] - ux0[act])) <= 1e-10 * umax
    assert np.max(np.abs(uy1[act] - uy0[act])) <= 1e-10 * umax
    assert np.max(np.abs(dp1[act] - dp0[act] - delta)) <= 1e-10 * delta
    assert np.max(np.abs(T1[act] - T0[act])) <= 1e-13
    assert abs(ob1["iop_gauge"] - ob0["iop_gauge"]) <= 1e-10 * abs(ob0["iop_gauge"])
    assert ob1["q_out"] == pytest.approx(ob0["q_out"], rel=1e-9)


def _inlet_box(scheme, gbeta):
    """Closed box (outer walls adiabatic, BOX) with four INLET cells in its floor, at rest
    (u_in = 0): the inlet links are the only Dirichlet links of the thermal lattice."""
    nx, ny = 12, 12
    mask = A.box_mask(nx, ny)
    mask[0, 4:8] = A.encode(A.INLET)
    P = A.Params(nx=nx, ny=ny, tau_f=0.8, tau_t=0.9, T_init=0.5, T0=0.5, T_inlet=0.7,
                 T_cornea=0.0, T_iris=1.0, gbeta=gbeta, check_interval=1000, bc_scheme=scheme)
    return O.Oracle(P, mask), P, A.active(mask)


@pytest.mark.parametrize("scheme", [A.BC_LINKWISE, A.BC_PAPER])
def test_inlet_temperature_sets_closed_box(scheme):
    """Every heat flux into the box passes the INLET links, whose Dirichlet rule
    (anti-bounce-back, or the paper's extrapolation) imposes T_inlet; the adiabatic walls
    let nothing through, so the steady state is T = T_inlet at every node, with the fluid
    at rest.  Taking T_cornea or T_iris at these links would land on 0 or 1.  (Without
    buoyancy: under the literal first-order force of eq. 6 and eq. 9 a hydrostatic state
    carries the moment u = -F/2, which would advect heat.)"""
    o, P, act = _inlet_box(scheme, 0.0)
    o.step(30000)
    dp, ux, uy, T = o.fields()
    assert np.max(np.abs(T[act] - P.T_inlet)) < 1e-12
    assert np.max(np.abs(ux[act])) < 1e-12 and np.max(np.abs(uy[act])) < 1e-12
