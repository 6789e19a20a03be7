"""Seeded synthetic inputs for the coupled aqueous-humour lattice Boltzmann model.

This module builds what a solve is given, and nothing else:

* node-type masks (one byte per node) for the synthetic anterior-chamber section and for
  the small test geometries (closed box, channels, slabs);
* the wall-node list (node, wall id, analytic unit normal into the fluid) used for the
  wall-shear-stress reduction;
* seeded parameter draws (splitmix64 counter generator, published definition by
  Steele, Lea and Flood, 2014) for the parameter-sweep workloads;
* the lattice-unit parameter set of a workload (relaxation times, inlet velocity,
  buoyancy strength g*beta, permeability K, wall temperatures).

It holds none of the method's per-step arithmetic.  The oracle and the HIP library each
implement the lattice Boltzmann step on their own, from the paper, and only share these
inputs.

Mask byte encoding (an input format, read independently by both implementations):
  bits 0-2  node class: SOLID=0, FLUID=1, POROUS=2, INLET=3, OUTLET=4
  bits 3-4  wall id of a SOLID node: BOX=0 (adiabatic), CORNEA=1, IRIS=2; for an OUTLET
            node of a lumped-meshwork outlet, the outward seepage direction
            (+x=0, +y=1, -x=2, -y=3)
FLUID and POROUS nodes are "active" (they carry populations).  The outer one-node frame
of a non-periodic lattice is never active.

The anterior-chamber geometry follows the paper's section 2.1 (Table 1: circular cornea,
flat iris/lens floor, pupil gap feeding the chamber, trabecular meshwork at the chamber
angle), rasterised parametrically because the paper's Fig. 1 mask is not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, field

import numpy as np

SOLID, FLUID, POROUS, INLET, OUTLET = 0, 1, 2, 3, 4
WALL_BOX, WALL_CORNEA, WALL_IRIS = 0, 1, 2
# For OUTLET nodes of a lumped-meshwork outlet the wall bits hold the outward direction
# of the seepage flow (the axis link it points along).
DIR_PX, DIR_PY, DIR_MX, DIR_MY = 0, 1, 2, 3
OUTLET_PRESSURE, OUTLET_LUMPED = 0, 1

# Wall-node list entry: node index, wall id, analytic unit normal into the fluid, and for
# each link i = 1..8 (q[i-1]) the fraction of the link from the node to the wall surface
# when the neighbour along e_i is a CORNEA or IRIS solid (in (0, 1]), else -1.
WALL_DTYPE = np.dtype([("node", "<i4"), ("wall", "<i4"), ("nx", "<f8"), ("ny", "<f8"), ("q", "<f8", (8,))])
BC_LINKWISE, BC_PAPER = 0, 1

# D2Q9 link directions, used here only to find which active nodes touch a wall.
_LINKS = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def encode(cls: int, wall: int = 0) -> int:
    return (cls & 7) | ((wall & 3) << 3)


def node_class(mask: np.ndarray) -> np.ndarray:
    return mask & 7


def wall_of(mask: np.ndarray) -> np.ndarray:
    return (mask >> 3) & 3


def active(mask: np.ndarray) -> np.ndarray:
    c = node_class(mask)
    return (c == FLUID) | (c == POROUS)


# ----------------------------------------------------------------------------------------
# splitmix64 counter generator
# ----------------------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64(seed: int, k: int) -> int:
    """Output number k (k >= 0) of the splitmix64 sequence started at `seed`.

    state_k = seed + (k+1) * 0x9E3779B97F4A7C15; output = mix(state_k), with the mix
    function of the published splitmix64 definition.
    """
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform01(seed: int, k: int) -> float:
    """U in [0, 1) from the top 53 bits of splitmix64 output k."""
    return (splitmix64(seed, k) >> 11) * (2.0 ** -53)


# Field order of the per-instance draws (counter k).
DRAW_FIELDS = ("alpha", "u_in", "log10_da", "log10_ra", "tau_f", "phi", "size", "arrival")


def draw(seed: int, name: str) -> float:
    return uniform01(seed, DRAW_FIELDS.index(name))


# ----------------------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------------------
@dataclass
class EyeGeometry:
    nx: int
    ny: int
    alpha_deg: float
    R: float
    xc: float
    yc: float
    jf: int
    s: int
    depth: float
    tm_cols: list = field(default_factory=list)   # [(c0, c1) inclusive] per block
    outlet_cols: list = field(default_factory=list)
    inlet_cols: tuple = (0, 0)


D0_DEPTH = 80.0 * (1.0 - math.cos(math.radians(45.0)))   # chamber depth of the 192x96 case


def eye_mask(nx: int, ny: int, alpha_deg: float = 45.0, R: float | None = None,
             jf: int = 2, pupil_gap: int | None = None, tm: str = "resolved"):
    """Synthetic anterior-chamber section.

    Rows j < jf are the iris/lens floor (SOLID, wall IRIS).  A pupil gap of `pupil_gap`
    INLET cells sits in row jf-1 at the centre.  The chamber is the part of the disc of
    radius R centred at (xc, yc) = ((nx-1)/2, jf - 1/2 - R cos(alpha)) with j >= jf, so the
    cornea arc meets the floor's half-way line at the chamber angle alpha and the depth is
    R(1 - cos alpha).  At each chamber angle a POROUS trabecular-meshwork block 4s wide and
    8s tall is centred on the corner, with a one-column OUTLET strip on its outer side.
    Every other node is SOLID: CORNEA above the floor, IRIS in it.

    tm="lumped" instead makes each meshwork block and its strip OUTLET nodes whose
    seepage direction points away from the chamber along x (-x on the left, +x on the
    right): the lumped-meshwork outlet, where the flow leaves at the Darcy seepage speed.

    Returns (mask[ny, nx] uint8, walls (WALL_DTYPE), EyeGeometry).
    """
    a = math.radians(alpha_deg)
    if R is None:
        s = 1
        for _ in range(20):
            R_try = (nx - 2 * (4 * s + 3)) / (2.0 * math.sin(a))
            s_new = max(1, int(math.floor(R_try * (1.0 - math.cos(a)) / D0_DEPTH + 0.5)))
            if s_new == s:
                break
            s = s_new
        R = (nx - 2 * (4 * s + 3)) / (2.0 * math.sin(a))
    depth = R * (1.0 - math.cos(a))
    s = max(1, int(math.floor(depth / D0_DEPTH + 0.5)))
    if pupil_gap is None:
        pupil_gap = 2 * s
    xc = (nx - 1) / 2.0
    yc = (jf - 0.5) - R * math.cos(a)
    if jf + depth + 2 > ny - 1:
        raise ValueError("lattice too short for the chamber")

    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    mask = np.where(jj >= jf, encode(SOLID, WALL_CORNEA), encode(SOLID, WALL_IRIS)).astype(np.uint8)
    inside = ((ii - xc) ** 2 + (jj - yc) ** 2 < R * R) & (jj >= jf)
    mask[inside] = encode(FLUID)

    g0 = nx // 2 - pupil_gap // 2
    mask[jf - 1, g0:g0 + pupil_gap] = encode(INLET)

    geo = EyeGeometry(nx, ny, alpha_deg, R, xc, yc, jf, s, depth, inlet_cols=(g0, g0 + pupil_gap - 1))
    half = R * math.sin(a)
    w, h = 4 * s, 8 * s
    # left block centred on the left corner; the right block is its exact mirror image
    c0 = int(math.floor(xc - half - w / 2.0 + 0.5))
    c1 = c0 + w - 1
    if tm not in ("resolved", "lumped"):
        raise ValueError("tm is 'resolved' or 'lumped'")
    for lo, hi, oc, d in ((c0, c1, c0 - 1, DIR_MX), (nx - 1 - c1, nx - 1 - c0, nx - c0, DIR_PX)):
        if tm == "lumped":
            mask[jf:jf + h, min(lo, oc):max(hi, oc) + 1] = encode(OUTLET, d)
        else:
            mask[jf:jf + h, lo:hi + 1] = encode(POROUS)
            mask[jf:jf + h, oc] = encode(OUTLET)
        geo.tm_cols.append((lo, hi))
        geo.outlet_cols.append(oc)

    _frame(mask)
    walls = wall_list(mask, normal_fn=lambda x, y, wall: _eye_normal(geo, x, y, wall),
                      q_fn=lambda x, y, ex, ey, wall: _eye_fraction(geo, x, y, ex, ey, wall))
    return mask, walls, geo


def _eye_fraction(geo: EyeGeometry, x, y, ex, ey, wall):
    """Fraction t in (0, 1] of the link from node (x, y) along (ex, ey) at which it meets
    the wall: the cornea circle for a CORNEA neighbour, the floor's half-way line
    y = jf - 1/2 for an IRIS neighbour."""
    if wall == WALL_IRIS:
        return (geo.jf - 0.5 - y) / ey if ey != 0 else 0.5
    dx, dy = x - geo.xc, y - geo.yc
    a = ex * ex + ey * ey
    b = dx * ex + dy * ey
    c = dx * dx + dy * dy - geo.R * geo.R
    t = (-b + math.sqrt(max(b * b - a * c, 0.0))) / a
    return min(max(t, 1e-6), 1.0)


def _eye_normal(geo: EyeGeometry, x, y, wall):
    """Analytic unit normals into the fluid: toward the cornea circle's centre, or +y
    for the flat iris floor."""
    dx, dy = geo.xc - x, geo.yc - y
    r = np.hypot(dx, dy)
    iris = wall == WALL_IRIS
    return np.where(iris, 0.0, dx / r), np.where(iris, 1.0, dy / r)


def _frame(mask: np.ndarray, periodic_x: bool = False, periodic_y: bool = False):
    """Force the outer one-node frame of a non-periodic axis to be non-active."""
    ny, nx = mask.shape
    edges = []
    if not periodic_y:
        edges += [(0, slice(None)), (ny - 1, slice(None))]
    if not periodic_x:
        edges += [(slice(None), 0), (slice(None), nx - 1)]
    for e in edges:
        m = mask[e]
        bad = ((m & 7) == FLUID) | ((m & 7) == POROUS)
        m[bad] = encode(SOLID, WALL_BOX)
        mask[e] = m


def wall_list(mask: np.ndarray, normal_fn, periodic_x: bool = False, periodic_y: bool = False,
              q_fn=None):
    """FLUID nodes with at least one link to a CORNEA or IRIS solid, sorted by node index.

    A node touching both walls is listed once, as CORNEA.  The normal comes from
    `normal_fn(x, y, wall)` on arrays (analytic, unit length, pointing into the fluid).
    The link fractions come from `q_fn(x, y, ex, ey, wall_of_neighbour)` (scalars), or are
    1/2 (the half-way wall) without one.
    """
    ny, nx = mask.shape
    cls = mask & 7
    wl = (mask >> 3) & 3
    touch_c = np.zeros((ny, nx), bool)
    touch_i = np.zeros((ny, nx), bool)
    for ex, ey in _LINKS:
        # neighbour (x+ex, y+ey) of node (x, y)
        nb_c = np.zeros((ny, nx), bool)
        nb_i = np.zeros((ny, nx), bool)
        sc = (cls == SOLID) & (wl == WALL_CORNEA)
        si = (cls == SOLID) & (wl == WALL_IRIS)
        if periodic_x or periodic_y:
            rc = np.roll(sc, shift=(-ey if periodic_y else 0, -ex if periodic_x else 0), axis=(0, 1))
            ri = np.roll(si, shift=(-ey if periodic_y else 0, -ex if periodic_x else 0), axis=(0, 1))
        else:
            rc, ri = sc, si
        ys = slice(max(0, -ey), ny - max(0, ey))
        xs = slice(max(0, -ex), nx - max(0, ex))
        ys2 = slice(max(0, ey), ny - max(0, -ey))
        xs2 = slice(max(0, ex), nx - max(0, -ex))
        if periodic_x or periodic_y:
            nb_c, nb_i = rc, ri
        else:
            nb_c[ys, xs] = rc[ys2, xs2]
            nb_i[ys, xs] = ri[ys2, xs2]
        touch_c |= nb_c
        touch_i |= nb_i
    fl = cls == FLUID
    wall = np.where(fl & touch_c, WALL_CORNEA, np.where(fl & touch_i, WALL_IRIS, 0))
    idx = np.flatnonzero(wall.ravel())
    out = np.zeros(idx.size, dtype=WALL_DTYPE)
    out["node"] = idx
    w = wall.ravel()[idx]
    out["wall"] = w
    x = (idx % nx).astype(np.float64)
    y = (idx // nx).astype(np.float64)
    n_x, n_y = normal_fn(x, y, w)
    out["nx"] = n_x
    out["ny"] = n_y
    out["q"] = -1.0
    for k, node in enumerate(idx):
        xx, yy = int(node % nx), int(node // nx)
        for i, (ex, ey) in enumerate(_LINKS):
            x2, y2 = xx + ex, yy + ey
            if periodic_x:
                x2 %= nx
            if periodic_y:
                y2 %= ny
            if not (0 <= x2 < nx and 0 <= y2 < ny) or cls[y2, x2] != SOLID or wl[y2, x2] == WALL_BOX:
                continue
            out["q"][k, i] = 0.5 if q_fn is None else q_fn(xx, yy, ex, ey, int(wl[y2, x2]))
    return out


def box_mask(nx: int, ny: int, porous_rect=None, wall_ids=(WALL_BOX, WALL_BOX, WALL_BOX, WALL_BOX)):
    """Closed box: interior FLUID, frame SOLID.  wall_ids = (bottom, top, left, right)."""
    mask = np.full((ny, nx), encode(FLUID), np.uint8)
    b, t, l, r = wall_ids
    mask[0, :] = encode(SOLID, b)
    mask[ny - 1, :] = encode(SOLID, t)
    mask[:, 0] = encode(SOLID, l)
    mask[:, nx - 1] = encode(SOLID, r)
    if porous_rect is not None:
        x0, x1, y0, y1 = porous_rect
        mask[y0:y1, x0:x1] = encode(POROUS)
    return mask


def channel_mask(nx: int, ny: int, bottom_wall=WALL_BOX, top_wall=WALL_BOX):
    """Channel periodic in x: rows 0 and ny-1 SOLID, the rest FLUID."""
    mask = np.full((ny, nx), encode(FLUID), np.uint8)
    mask[0, :] = encode(SOLID, bottom_wall)
    mask[ny - 1, :] = encode(SOLID, top_wall)
    return mask


def duct_mask(nx: int, ny: int, inlet_len: int = 1, porous_cols=None, porous_all=False):
    """Straight duct along x: SOLID rows 0 and ny-1, an INLET column at x=0 and an
    OUTLET column at x=nx-1 (both on interior rows), FLUID between (POROUS in
    `porous_cols` = (c0, c1) half-open, or everywhere if porous_all)."""
    mask = np.full((ny, nx), encode(POROUS if porous_all else FLUID), np.uint8)
    if porous_cols is not None:
        mask[:, porous_cols[0]:porous_cols[1]] = encode(POROUS)
    mask[:, 0] = encode(INLET)
    mask[:, nx - 1] = encode(OUTLET)
    mask[0, :] = encode(SOLID, WALL_BOX)
    mask[ny - 1, :] = encode(SOLID, WALL_BOX)
    return mask


def no_walls():
    return np.zeros(0, dtype=WALL_DTYPE)


# ----------------------------------------------------------------------------------------
# Lattice-unit parameter sets (the workload recipe)
# ----------------------------------------------------------------------------------------
F64, F32, F16S, F32X = 0, 1, 2, 3


@dataclass
class Params:
    nx: int
    ny: int
    tau_f: float = 0.8
    tau_t: float = 0.7
    w0: float = 1.0 / 3.0
    u_in_x: float = 0.0
    u_in_y: float = 0.0
    p_ref: float = 1.0 / 3.0
    p_out: float = 1.0 / 3.0
    p_init: float = 1.0 / 3.0
    T_ref: float = 0.5
    T_init: float = 0.5
    T0: float = 0.5
    T_cornea: float = 0.0
    T_iris: float = 1.0
    T_inlet: float = 1.0
    gbeta: float = 0.0
    gravity_angle: float = 0.0
    K: float = 1.0e30
    storage: int = F64
    check_interval: int = 100
    fp16_exp_flow: int = -1
    fp16_exp_thermal: int = -1
    periodic_x: int = 0
    periodic_y: int = 0
    # lumped meshwork outlet (outlet_mode = OUTLET_LUMPED): permeability, thickness and
    # Schlemm's-canal pressure, lattice units
    outlet_mode: int = OUTLET_PRESSURE
    # boundary scheme: BC_LINKWISE (half-way bounce-back) or BC_PAPER (interpolated
    # bounce-back of Bouzidi et al. on CORNEA / IRIS walls with the wall list's fractions)
    bc_scheme: int = BC_LINKWISE
    K_tm: float = 1.0
    h_tm: float = 1.0
    p_sc: float = 1.0 / 3.0

    def asdict(self):
        return asdict(self)


def viscosity_of(tau_f: float) -> float:
    """Kinematic viscosity in lattice units for a relaxation time (the paper's eq. 10)."""
    return (2.0 * tau_f - 1.0) / 6.0


def diffusivity_of(tau_t: float, w0: float) -> float:
    """Thermal diffusivity in lattice units, (1-w0)(2 tau_T - 1)/4 (eq. 14 at w0 = 0)."""
    return (1.0 - w0) * (2.0 * tau_t - 1.0) / 4.0


def eye_params(nx, ny, geo: EyeGeometry, *, u_in=1e-4, Da=1e-4, Ra=1e3, tau_f=0.8,
               tau_t=0.7, w0=1.0 / 3.0, phi_deg=0.0, storage=F64, check_interval=100,
               tm="resolved", h_tm=None, p_sc=1.0 / 3.0):
    """Workload parameters for the eye geometry.  Ra = g beta dT H^3 / (nu theta) and
    Da = K / H^2 with H the chamber depth and dT = T_iris - T_cornea = 1.  With
    tm="lumped" the meshwork has permeability K_tm = Da H^2 and thickness h_tm (default:
    the block width 4s) and drains to the Schlemm's-canal pressure p_sc."""
    H = geo.depth
    nu = viscosity_of(tau_f)
    th = diffusivity_of(tau_t, w0)
    p = Params(nx=nx, ny=ny, tau_f=tau_f, tau_t=tau_t, w0=w0, u_in_x=0.0, u_in_y=u_in,
               gbeta=Ra * nu * th / H ** 3, gravity_angle=math.radians(phi_deg),
               K=Da * H * H, storage=storage, check_interval=check_interval)
    if tm == "lumped":
        p.outlet_mode = OUTLET_LUMPED
        p.K_tm = Da * H * H
        p.h_tm = float(4 * geo.s) if h_tm is None else float(h_tm)
        p.p_sc = p_sc
    return p


def config0():
    """The 192x96 eye case: R = 80, alpha = 45 deg, u_in = 1e-4, Da = 1e-4, Ra = 1e3,
    tau_f = 0.8, tau_T = 0.7, gravity along -y, cornea T = 0, iris T = 1, T_init = 0.5."""
    mask, walls, geo = eye_mask(192, 96, 45.0, R=80.0, pupil_gap=2)
    p = eye_params(192, 96, geo)
    return p, mask, walls, geo


def sweep_instance(seed: int, nx: int, ny: int, *, tau_f=None, phi_deg=None, storage=F64,
                   check_interval=100, tm="resolved"):
    """One draw of the parameter sweep: alpha ~ U(25, 45) deg, u_in ~ U(0.5, 2) x 1e-4,
    Da ~ 10^U(-5, -3), Ra ~ 10^U(3, 5).  tau_f and phi default to 0.8 and 0 deg unless
    drawn (tau_f ~ U(0.55, 1.2), phi ~ U(0, 90) deg) when passed as 'draw'."""
    alpha = 25.0 + 20.0 * draw(seed, "alpha")
    u_in = (0.5 + 1.5 * draw(seed, "u_in")) * 1e-4
    Da = 10.0 ** (-5.0 + 2.0 * draw(seed, "log10_da"))
    Ra = 10.0 ** (3.0 + 2.0 * draw(seed, "log10_ra"))
    if tau_f == "draw":
        tau_f = 0.55 + 0.65 * draw(seed, "tau_f")
    elif tau_f is None:
        tau_f = 0.8
    if phi_deg == "draw":
        phi_deg = 90.0 * draw(seed, "phi")
    elif phi_deg is None:
        phi_deg = 0.0
    mask, walls, geo = eye_mask(nx, ny, alpha, tm=tm)
    p = eye_params(nx, ny, geo, u_in=u_in, Da=Da, Ra=Ra, tau_f=tau_f, phi_deg=phi_deg,
                   storage=storage, check_interval=check_interval, tm=tm)
    return p, mask, walls, geo


BATCH_SIZES = ((256, 128), (512, 256), (768, 384), (1024, 512))


def batch_size_of(seed: int):
    return BATCH_SIZES[min(3, int(4 * draw(seed, "size")))]


def interarrival(seed: int, rate: float) -> float:
    """Exponential inter-arrival time with mean 1/rate from U of the 'arrival' counter."""
    return -math.log(1.0 - draw(seed, "arrival")) / rate
