"""The oracle's deviation form against a literal absolute-form statement of the model.

The oracle holds h_i = f_i - lambda_i p_ref and g_i = T_i - w^T_i T_ref (an exact affine
change of variables that keeps the small pressure signal from cancelling against p_ref).
This module steps the paper's own variables instead: absolute f_0..f_8 (f_0 included,
with its equilibrium -4 sigma p + S_0(u) of eq. 7) and T_0..T_4, with the moments of
eq. 9 and eq. 13, the collisions of eq. 6 and eq. 11, the force of eq. 17 and the link
rules written for absolute populations.  It shares nothing with the oracle but the
inputs.  A mistake in the change of variables (a shift on a wrong link, a boundary term
carried over without its p_ref or T_ref part, a wrong constant in eq. 9) shows up as a
difference far above the rounding of the absolute form.
"""
import math

import numpy as np
import pytest

import aqinputs as A
import oracle as O

# D2Q9 velocities in the paper's order: rest, four axis links, four diagonals
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)           # eq. 8
SIGMA = 5.0 / 12.0                                            # reading of eq. 7's constraints
LAMBDA = np.array([0.0] + [1 / 3] * 4 + [1 / 12] * 4)         # lambda, gamma: lambda + gamma = sigma,
assert abs(LAMBDA[1] + LAMBDA[5] - SIGMA) < 1e-16             # lambda + 2 gamma = 1/2
assert abs(LAMBDA[1] + 2 * LAMBDA[5] - 0.5) < 1e-16


def S(i, ux, uy):
    """eq. 8 with c = 1."""
    eu = EX[i] * ux + EY[i] * uy
    return W[i] * (3 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))


def feq(i, p, ux, uy):
    """eq. 7: f_0^eq = -4 sigma p + S_0(u), f_i^eq = lambda_i p + S_i(u)."""
    return (-4 * SIGMA * p if i == 0 else LAMBDA[i] * p) + S(i, ux, uy)


class Literal:
    """Absolute-form lattice with link-wise boundaries (push streaming)."""

    def __init__(self, P, mask):
        self.P = P
        self.ny, self.nx = mask.shape
        self.cls = A.node_class(mask)
        self.wall = A.wall_of(mask)
        self.act = A.active(mask)
        self.wT = np.array([P.w0] + [(1 - P.w0) / 4] * 4)
        self.cs2T = (1 - P.w0) / 2
        self.f = np.zeros((9, self.ny, self.nx))
        self.T = np.zeros((5, self.ny, self.nx))
        for i in range(9):
            self.f[i][self.act] = feq(i, P.p_init, 0.0, 0.0)
        for i in range(5):
            self.T[i][self.act] = self.wT[i] * P.T_init

    def moments(self, f, Ti):
        ux = sum(EX[i] * f[i] for i in range(9))
        uy = sum(EY[i] * f[i] for i in range(9))
        p = (sum(f[i] for i in range(1, 9)) + S(0, ux, uy)) / (4 * SIGMA)      # eq. 9
        T = sum(Ti[i] for i in range(5))                                        # eq. 13
        return p, ux, uy, T

    def step(self):
        P = self.P
        f, Ti = self.f, self.T
        p, ux, uy, T = self.moments(f, Ti)
        # eq. 15-16: buoyant force g beta (T - T0) opposite to gravity (sin phi, cos phi)
        Bx = P.gbeta * (T - P.T0) * math.sin(P.gravity_angle)
        By = P.gbeta * (T - P.T0) * math.cos(P.gravity_angle)
        # eq. 4 as a drag on the mid-step velocity in porous nodes
        nu = (2 * P.tau_f - 1) / 6
        por = self.cls == A.POROUS
        uDx = (ux + Bx / 2) / (1 + nu / (2 * P.K))
        uDy = (uy + By / 2) / (1 + nu / (2 * P.K))
        Dx = np.where(por, -nu / P.K * uDx, 0.0)
        Dy = np.where(por, -nu / P.K * uDy, 0.0)
        fs = np.empty_like(f)
        for i in range(9):
            Fi = (0.5 * (EX[i] * Bx + EY[i] * By) if 1 <= i <= 4 else 0.0) + 3 * W[i] * (EX[i] * Dx + EY[i] * Dy)
            fs[i] = f[i] - (f[i] - feq(i, p, ux, uy)) / P.tau_f + Fi                  # eq. 6
        Ts = np.empty_like(Ti)
        for i in range(5):
            eu = EX[i] * ux + EY[i] * uy
            Ts[i] = Ti[i] - (Ti[i] - self.wT[i] * T * (1 + eu / self.cs2T)) / P.tau_t  # eq. 11-12
        fn = np.full_like(f, np.nan)
        Tn = np.full_like(Ti, np.nan)
        ys, xs = np.nonzero(self.act)
        fn[0, ys, xs] = fs[0, ys, xs]
        Tn[0, ys, xs] = Ts[0, ys, xs]
        for i in range(1, 9):
            y2, x2 = ys + EY[i], xs + EX[i]
            c = self.cls[y2, x2]
            o = OPP[i]
            v = fs[i, ys, xs]
            go = (c == A.FLUID) | (c == A.POROUS)
            fn[i, y2[go], x2[go]] = v[go]
            m = c == A.SOLID                                              # half-way bounce-back
            fn[o, ys[m], xs[m]] = v[m]
            m = c == A.INLET                                              # wall moving at u_in
            fn[o, ys[m], xs[m]] = v[m] - 6 * W[i] * (EX[i] * P.u_in_x + EY[i] * P.u_in_y)
            m = c == A.OUTLET                                             # anti-bounce-back at p_out
            fn[o, ys[m], xs[m]] = -v[m] + 2 * LAMBDA[i] * P.p_out
        for i in range(1, 5):
            y2, x2 = ys + EY[i], xs + EX[i]
            c = self.cls[y2, x2]
            wl = self.wall[y2, x2]
            o = OPP[i]
            v = Ts[i, ys, xs]
            go = (c == A.FLUID) | (c == A.POROUS)
            Tn[i, y2[go], x2[go]] = v[go]
            for sel, Tw in (((c == A.SOLID) & (wl == A.WALL_CORNEA), P.T_cornea),
                            ((c == A.SOLID) & (wl == A.WALL_IRIS), P.T_iris),
                            (c == A.INLET, P.T_inlet)):
                Tn[o, ys[sel], xs[sel]] = -v[sel] + 2 * self.wT[i] * Tw   # Dirichlet anti-bounce-back
            m = ((c == A.SOLID) & (wl == A.WALL_BOX)) | (c == A.OUTLET)   # adiabatic
            Tn[o, ys[m], xs[m]] = v[m]
        self.f, self.T = fn, Tn

    def fields(self):
        p, ux, uy, T = self.moments(self.f, self.T)
        nan = ~self.act
        return [np.where(nan, np.nan, a) for a in (p - self.P.p_ref, ux, uy, T)]


def _case():
    """The 192x96 eye section with every link rule in play and a strong signal: faster
    secretion, stronger buoyancy, a porous meshwork and an outlet pressure off p_ref."""
    p, mask, walls, geo = A.config0()
    p.u_in_y = 2e-3
    p.gbeta *= 4.0
    p.p_out = p.p_ref + 1e-3
    p.p_init = p.p_ref + 5e-4
    p.T_init = 0.3
    return p, mask, walls


@pytest.mark.slow
def test_deviation_form_matches_literal_absolute_form():
    """After 1000 steps every field of the oracle equals the literal absolute form to
    1e-10 of the field's range (normwise per field).  The absolute form rounds about
    1e-16 of p ~ 1/3 per operation, far below this on a signal of ~1e-3."""
    P, mask, walls = _case()
    lit = Literal(P, mask)
    o = O.Oracle(P, mask, walls)
    for _ in range(1000):
        lit.step()
    o.step(1000)
    act = A.active(mask)
    got = o.fields()
    want = lit.fields()
    for k, (G, R) in enumerate(zip(got, want)):
        ref = R[act] - (P.T_ref if k == 3 else 0.0)
        scale = np.max(np.abs(ref))
        assert scale > 1e-5
        err = np.max(np.abs(G[act] - R[act])) / scale
        assert err <= 1e-10, (k, err)


def test_rest_population_is_dead():
    """f_0 never enters u or p (eq. 9 sums i >= 1, e_0 = 0) and never streams: replacing it
    by arbitrary values changes no other population, bit for bit.  This is why neither the
    oracle nor the library stores it."""
    P, mask, walls = _case()
    a = Literal(P, mask)
    b = Literal(P, mask)
    rng = np.random.default_rng(11)
    b.f[0][b.act] = rng.uniform(-1.0, 1.0, int(b.act.sum()))
    for _ in range(50):
        a.step()
        b.step()
    assert np.array_equal(a.f[1:][:, a.act], b.f[1:][:, b.act])
    assert np.array_equal(a.T[:, a.act], b.T[:, b.act])
