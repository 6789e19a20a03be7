"""Vortex diagnostics of section 3.5 (eq. 18, Table 3, Figs. 6-7), plain numpy.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: the tests and the smoke check compare
the library's device diagnostics (aq_diagnose) with these, computed from the oracle's own
velocity field.  Loops are explicit where the definition is local, so the statement can
be checked by eye.

Definitions (reading of eq. 18, whose signed area integral of omega_z would be the
circulation around the no-slip boundary, i.e. zero):
  omega_z = (d u_y/dx - d u_x/dy) / 2; each derivative is the central difference where
  both neighbours along the axis are active nodes, the one-sided difference toward the
  active one where only one is, and 0 where neither is;
  vortex intensity I = 2 * sum over FLUID nodes of |omega_z| (unit cell area);
  u_max_fluid = max |u| over FLUID nodes;
  stream function psi(x, y) = sum over active nodes (x, y') with y' <= y of u_x(x, y'),
  so that u_x = d psi / dy; the vortex centres are the FLUID nodes where psi is largest and
  smallest (the first in y * nx + x order on ties).
"""
from __future__ import annotations

import numpy as np

FLUID, POROUS = 1, 2


def _active(mask):
    c = mask & 7
    return (c == FLUID) | (c == POROUS)


def _derivative(f, act, x, y, dx, dy):
    ny, nx = act.shape

    def on(xx, yy):
        return 0 <= xx < nx and 0 <= yy < ny and act[yy, xx]

    up, dn = on(x + dx, y + dy), on(x - dx, y - dy)
    if up and dn:
        return (f[y + dy, x + dx] - f[y - dy, x - dx]) / 2.0
    if up:
        return f[y + dy, x + dx] - f[y, x]
    if dn:
        return f[y, x] - f[y - dy, x - dx]
    return 0.0


def vorticity(ux, uy, mask):
    """omega_z at FLUID nodes (NaN elsewhere)."""
    act = _active(mask)
    fluid = (mask & 7) == FLUID
    w = np.full(ux.shape, np.nan)
    for y, x in zip(*np.nonzero(fluid)):
        w[y, x] = 0.5 * (_derivative(uy, act, x, y, 1, 0) - _derivative(ux, act, x, y, 0, 1))
    return w


def stream_function(ux, mask):
    act = _active(mask)
    return np.cumsum(np.where(act, ux, 0.0), axis=0)


def diagnose(ux, uy, mask) -> dict:
    fluid = (mask & 7) == FLUID
    w = vorticity(ux, uy, mask)
    psi = stream_function(ux, mask)
    out = {"vortex_intensity": float(2.0 * np.sum(np.abs(w[fluid]))),
           "u_max_fluid": float(np.max(np.hypot(ux, uy)[fluid])) if fluid.any() else 0.0}
    ny, nx = mask.shape
    flat = np.where(fluid, psi, np.nan).ravel()
    if fluid.any():
        imax = int(np.nanargmax(flat))      # first occurrence in y * nx + x order
        imin = int(np.nanargmin(flat))
        out.update(psi_max=float(flat[imax]), psi_max_x=imax % nx, psi_max_y=imax // nx,
                   psi_min=float(flat[imin]), psi_min_x=imin % nx, psi_min_y=imin // nx)
    else:
        out.update(psi_max=float("-inf"), psi_max_x=-1, psi_max_y=-1, psi_min=float("inf"), psi_min_x=-1,
                   psi_min_y=-1)
    return out
