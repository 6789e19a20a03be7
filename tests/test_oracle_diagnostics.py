"""Pins of the vortex diagnostics (oracle/diagnostics.py; eq. 18, Table 3, section 3.5).

* Rigid rotation u = W (-(y - yc), x - xc) on a disc: omega_z = W at every node (the
  difference stencils are exact for linear fields), so I = 2 W N; the stream function
  psi = sum_{y' <= y} u_x peaks where u_x changes sign, at the column with the most nodes
  below the centre, with the value W * sum (yc - y').
* Uniform flow: I = 0 and psi(x, y) = U * (number of active nodes at or below y).
* The standing eye (gravity across the chamber) in the Stokes regime: the intensity and
  the maximum speed both scale with the temperature difference, so I / u_max is constant,
  as in Table 3 (within its 5%), and the single vortex's centre stays put.
"""
import os

import numpy as np
import pytest

import aqinputs as A
import oracle as O
from oracle import diagnostics as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _disc(n=41, r=17.3, cx=20.0, cy=20.5):
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    inside = (ii - cx) ** 2 + (jj - cy) ** 2 < r * r
    mask = np.where(inside, A.encode(A.FLUID), A.encode(A.SOLID)).astype(np.uint8)
    return mask, ii, jj


def test_rigid_rotation_intensity_and_centre():
    W, cx, cy = 2.5e-4, 20.0, 20.5
    mask, ii, jj = _disc(cx=cx, cy=cy)
    fluid = (mask & 7) == A.FLUID
    ux = np.where(fluid, -W * (jj - cy), np.nan)
    uy = np.where(fluid, W * (ii - cx), np.nan)
    w = D.vorticity(ux, uy, mask)
    assert np.allclose(w[fluid], W, rtol=1e-12, atol=0)
    d = D.diagnose(ux, uy, mask)
    assert d["vortex_intensity"] == pytest.approx(2 * W * fluid.sum(), rel=1e-12)
    # u_x = W (cy - y) > 0 below the centre: psi grows up to row 20 (the last row below
    # 20.5) and is largest in the columns reaching lowest (the first of them on ties)
    per_col = [W * np.sum(cy - np.nonzero(fluid[:, c])[0][np.nonzero(fluid[:, c])[0] <= 20])
               if fluid[:, c].any() else -np.inf for c in range(mask.shape[1])]
    best = max(per_col)
    first = next(c for c, v in enumerate(per_col) if v >= best * (1 - 1e-12))
    assert (d["psi_max_x"], d["psi_max_y"]) == (first, 20)
    assert abs(first - cx) <= 5
    assert d["psi_max"] == pytest.approx(best, rel=1e-12)
    assert d["u_max_fluid"] == pytest.approx(W * np.max(np.hypot(ii - cx, jj - cy)[fluid]), rel=1e-12)


def test_uniform_flow():
    U = 3e-5
    mask, ii, jj = _disc()
    fluid = (mask & 7) == A.FLUID
    ux = np.where(fluid, U, np.nan)
    uy = np.where(fluid, 0.0, np.nan)
    d = D.diagnose(ux, uy, mask)
    assert d["vortex_intensity"] == 0.0
    psi = D.stream_function(ux, mask)
    assert np.allclose(psi, U * np.cumsum(fluid, axis=0), rtol=1e-12)


def test_fluid_only_definitions():
    """u_max and the vortex measures count FLUID nodes only, and the stream function sums
    active nodes only: a faster POROUS node does not set u_max, and values at inactive
    nodes (here finite, as a caller might pass them) change nothing."""
    U = 3e-5
    mask, ii, jj = _disc()
    fluid = (mask & 7) == A.FLUID
    porous = mask.copy()
    porous[20, 20] = A.encode(A.POROUS)
    act = A.active(porous)
    ux = np.where(act, U, 7.0)
    uy = np.where(act, 0.0, -3.0)
    ux[20, 20] = 5 * U
    d = D.diagnose(ux, uy, porous)
    assert d["u_max_fluid"] == pytest.approx(U, rel=1e-15)
    psi = D.stream_function(ux, porous)
    assert np.allclose(psi, np.cumsum(np.where(act, ux, 0.0), axis=0), rtol=1e-15, atol=0)
    assert np.allclose(psi[:, 0], 0.0) and psi[-1, 20] == pytest.approx(U * (fluid[:, 20].sum() + 4), rel=1e-12)


def _standing(dT):
    mask, walls, geo = A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2)
    p = A.eye_params(96, 48, geo, u_in=0.0, Ra=0.0, Da=1e-3, phi_deg=90.0, check_interval=500)
    nu = A.viscosity_of(p.tau_f)
    th = A.diffusivity_of(p.tau_t, p.w0)
    p.T_cornea, p.T_iris = 0.5 - dT / 2, 0.5 + dT / 2
    p.T_inlet = p.T_iris                                 # the closed pupil is part of the iris
    p.gbeta = 30.0 * nu * th / geo.depth ** 3           # Ra = 30 at dT = 1: Stokes regime
    o = O.Oracle(p, mask, walls)
    for _ in range(200):
        o.step(p.check_interval)
        if o.observables()["resid_u"] < 1e-9:
            break
    dp, ux, uy, T = o.fields()
    return D.diagnose(ux, uy, mask), mask


def test_standing_eye_scalings_table3():
    t3 = np.loadtxt(os.path.join(GOLDEN, "table3_vortex_standing.txt"))
    ratio_paper = t3[:, 3] / t3[:, 2]                     # I / u_max per row
    assert np.ptp(ratio_paper) / np.mean(ratio_paper) < 0.05
    d1, mask = _standing(1.0)
    d2, _ = _standing(2.0)
    # the buoyant flow is linear in dT in the Stokes regime: both measures double
    assert d2["vortex_intensity"] / d1["vortex_intensity"] == pytest.approx(2.0, rel=5e-3)
    assert d2["u_max_fluid"] / d1["u_max_fluid"] == pytest.approx(2.0, rel=5e-3)
    r1 = d1["vortex_intensity"] / d1["u_max_fluid"]
    r2 = d2["vortex_intensity"] / d2["u_max_fluid"]
    assert r2 == pytest.approx(r1, rel=0.05)
    # the paper's intensity per unit dT over dT = 1..2 (Table 3 rows 36 and 35 degC)
    paper = (t3[3, 3] / t3[3, 1]) / (t3[4, 3] / t3[4, 1])
    assert (d2["vortex_intensity"] / 2) / d1["vortex_intensity"] == pytest.approx(paper, rel=0.03)
    # one vortex, its centre inside the chamber and fixed to a node as dT doubles
    c1 = (d1["psi_max_x"], d1["psi_max_y"]) if abs(d1["psi_max"]) >= abs(d1["psi_min"]) else (d1["psi_min_x"], d1["psi_min_y"])
    c2 = (d2["psi_max_x"], d2["psi_max_y"]) if abs(d2["psi_max"]) >= abs(d2["psi_min"]) else (d2["psi_min_x"], d2["psi_min_y"])
    assert abs(c1[0] - c2[0]) <= 1 and abs(c1[1] - c2[1]) <= 1
    assert (mask[c1[1], c1[0]] & 7) == A.FLUID
