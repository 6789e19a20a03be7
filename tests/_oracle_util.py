"""Helpers for the oracle pins: initial states built from the oracle's own equilibrium."""
import numpy as np

import aqinputs as A
import oracle as O


def init_from_fields(orc: O.Oracle, params, p, ux, uy, T):
    """Set the oracle's state to the equilibrium of the given fields ([ny, nx] arrays or
    scalars), node by node, through the oracle's equilibrium routine."""
    ny, nx = orc.ny, orc.nx
    h = np.zeros((8, ny, nx))
    g = np.zeros((5, ny, nx))
    act = A.active(orc.mask)
    bc = lambda a: np.broadcast_to(np.asarray(a, float), (ny, nx))
    p, ux, uy, T = bc(p), bc(ux), bc(uy), bc(T)
    for y in range(ny):
        for x in range(nx):
            if act[y, x]:
                h[:, y, x], g[:, y, x] = O.equilibrium(params, p[y, x], ux[y, x], uy[y, x], T[y, x])
    orc.set_populations(h, g)
    return orc


def mirror_field(F):
    return F[:, ::-1]
