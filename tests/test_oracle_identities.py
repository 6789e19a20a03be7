"""Pins of the oracle's per-node arithmetic against properties the paper's model fixes.

Each check is a moment identity the equilibria and force term must satisfy for the
scheme to recover eq. 1-3 and eq. 16 (section 2.3), evaluated on the oracle's own output,
not a re-typing of its formulas.
"""
import math

import numpy as np
import pytest

import aqinputs as A
import oracle as O

EX = np.array([1, 0, -1, 0, 1, -1, -1, 1], float)     # e_1..e_8
EY = np.array([0, 1, 0, -1, 1, 1, -1, -1], float)
TX = np.array([0, 1, 0, -1, 0], float)                 # e_0..e_4
TY = np.array([0, 0, 1, 0, -1], float)


def _params(**kw):
    base = dict(nx=8, ny=8, tau_f=0.8, tau_t=0.7, w0=1.0 / 3.0, gbeta=0.0, K=1e30)
    base.update(kw)
    return A.Params(**base)


@pytest.mark.parametrize("w0", [0.0, 1.0 / 3.0, 0.2])
def test_equilibrium_moments(w0):
    """eq. 7-9 and 12-13: the equilibrium carries the macroscopic (p, u, T) it was built
    from; its momentum flux is p I + u u (the Euler flux of eq. 2); the thermal
    equilibrium carries T, the advective flux T u and an isotropic second moment."""
    P = _params(w0=w0)
    rng = np.random.default_rng(1)
    for _ in range(50):
        p = P.p_ref + rng.uniform(-1e-2, 1e-2)
        ux, uy = rng.uniform(-0.05, 0.05, 2)
        T = rng.uniform(0.0, 1.0)
        h, g = O.equilibrium(P, p, ux, uy, T)
        m = O.moments(P, h, g)
        assert m[0] == pytest.approx(p - P.p_ref, abs=1e-16)
        assert m[1] == pytest.approx(ux, abs=1e-15)
        assert m[2] == pytest.approx(uy, abs=1e-15)
        assert m[3] == pytest.approx(T, abs=1e-15)
        # absolute populations f_i = h_i + lambda_i p_ref, lambda = 3 w_i
        lam = np.array([1 / 3] * 4 + [1 / 12] * 4)
        f = h + lam * P.p_ref
        assert np.sum(EX * EX * f) == pytest.approx(p + ux * ux, abs=1e-15)
        assert np.sum(EY * EY * f) == pytest.approx(p + uy * uy, abs=1e-15)
        assert np.sum(EX * EY * f) == pytest.approx(ux * uy, abs=1e-15)
        # third moment isotropy: sum e_a e_b e_c f = (u_a d_bc + u_b d_ac + u_c d_ab)/3
        assert np.sum(EX ** 3 * f) == pytest.approx(ux, abs=1e-15)
        assert np.sum(EX * EX * EY * f) == pytest.approx(uy / 3, abs=1e-15)
        # thermal
        wT = np.array([w0] + [(1 - w0) / 4] * 4)
        Ti = g + wT * P.T_ref
        cs2 = (1 - w0) / 2
        assert np.sum(Ti) == pytest.approx(T, abs=1e-15)
        assert np.sum(TX * Ti) == pytest.approx(T * ux, abs=1e-15)
        assert np.sum(TY * Ti) == pytest.approx(T * uy, abs=1e-15)
        assert np.sum(TX * TX * Ti) == pytest.approx(cs2 * T, abs=1e-15)
        assert np.sum(TY * TY * Ti) == pytest.approx(cs2 * T, abs=1e-15)
        assert np.sum(TX * TY * Ti) == 0.0


def test_equilibrium_at_rest_is_weights():
    """At p = 1/3 (rho = 1) and u = 0 the flow equilibrium is w_i (i >= 1): the deviation
    shift lambda_i p_ref is exactly the D2Q9 weight, so the rest state is all zeros."""
    P = _params()
    h, g = O.equilibrium(P, 1.0 / 3.0, 0.0, 0.0, P.T_ref)
    assert np.all(h == 0.0) and np.all(g == 0.0)


def test_d2q4_reduces_to_eq12():
    """w0 = 0 gives the paper's D2Q4 equilibrium T_i^eq = T/4 (1 + 2 e_i.u), eq. 12."""
    P = _params(w0=0.0)
    T, ux, uy = 0.37, 0.013, -0.021
    h, g = O.equilibrium(P, P.p_ref, ux, uy, T)
    Ti = g + np.array([0, 0.25, 0.25, 0.25, 0.25]) * P.T_ref
    want = [0.0] + [T / 4 * (1 + 2 * (TX[i] * ux + TY[i] * uy)) for i in range(1, 5)]
    np.testing.assert_allclose(Ti, want, rtol=0, atol=1e-16)


@pytest.mark.parametrize("phi_deg", [0.0, 90.0, 33.0])
@pytest.mark.parametrize("porous", [False, True])
def test_collision_moments(phi_deg, porous):
    """One BGK collision (eq. 6, 11) conserves sum h and sum g, and changes the momentum
    by exactly the body force: buoyancy (eq. 16-17) in fluid, plus the Darcy drag (eq. 4)
    on the mid-step velocity in porous nodes.  Hot fluid (T > T0) is pushed against
    gravity."""
    P = _params(gbeta=3e-3, gravity_angle=math.radians(phi_deg), K=0.5, tau_f=0.9)
    rng = np.random.default_rng(7)
    for _ in range(20):
        h = rng.normal(0, 1e-3, 8)
        g = rng.normal(0, 1e-2, 5)
        hs, gs = O.collide_node(P, porous, h, g)
        m = O.moments(P, h, g)
        T = m[3]
        Fb = P.gbeta * (T - P.T0) * np.array([math.sin(P.gravity_angle), math.cos(P.gravity_angle)])
        du = np.array([np.sum(EX * hs), np.sum(EY * hs)]) - m[1:3]
        assert np.sum(hs) == pytest.approx(np.sum(h), abs=1e-17)
        assert np.sum(gs) == pytest.approx(np.sum(g), abs=1e-16)
        if not porous:
            np.testing.assert_allclose(du, Fb, rtol=0, atol=1e-17)
        else:
            # drag opposes the mid-step velocity and makes the implicit midpoint relation
            # u_D = u + (F_b + F_D)/2 hold with F_D = -(nu/K) u_D
            nu = (2 * P.tau_f - 1) / 6
            FD = du - Fb
            uD = -FD * P.K / nu
            np.testing.assert_allclose(uD, m[1:3] + (Fb + FD) / 2, rtol=1e-12, atol=1e-17)


def test_buoyancy_direction():
    """Gravity along -y (phi = 0): a hot node gains +y momentum, a cold one -y."""
    P = _params(gbeta=1e-3)
    h = np.zeros(8)
    for T, sign in ((0.9, +1), (0.1, -1)):
        g = np.array([P.w0] + [(1 - P.w0) / 4] * 4) * (T - P.T_ref)
        hs, _ = O.collide_node(P, False, h, g)
        assert np.sign(np.sum(EY * hs)) == sign
        assert abs(np.sum(EX * hs)) < 1e-20


def test_relaxation_toward_equilibrium():
    """Without force the non-equilibrium part decays by (1 - 1/tau) per collision."""
    P = _params(tau_f=0.77, tau_t=1.3)
    rng = np.random.default_rng(3)
    h = rng.normal(0, 1e-3, 8)
    g = rng.normal(0, 1e-3, 5)
    g[:] -= np.sum(g) - (P.T0 - P.T_ref)   # T = T0: no buoyancy
    m = O.moments(P, h, g)
    heq, geq = O.equilibrium(P, P.p_ref + m[0], m[1], m[2], m[3])
    hs, gs = O.collide_node(P, False, h, g)
    np.testing.assert_allclose(hs - heq, (1 - 1 / P.tau_f) * (h - heq), rtol=0, atol=2e-17)
    np.testing.assert_allclose(gs - geq, (1 - 1 / P.tau_t) * (g - geq), rtol=0, atol=2e-17)
