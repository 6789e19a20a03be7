"""FP64 CPU oracle of the coupled lattice Boltzmann model (arXiv:2102.12663, section 2.3).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports it.  The arithmetic lives in
`aq_oracle.c` (plain C, push form, FP64, built without FMA contraction); this module only
marshals numpy arrays through ctypes.

Pinned by the `-m "not gpu"` tests: equilibrium moment identities (eq. 7-9, 12-13),
forcing moments (eq. 17), exact mass conservation in closed boxes, shear-wave and
heat-mode decay rates (eq. 10, 14), plane Poiseuille (eq. 16), linear conduction (eq. 3),
the Darcy pressure drop (eq. 4), the Brinkman profile, mirror symmetry, the steady mass
balance, the wall-shear-stress momentum balance, invariance under a uniform shift of the
outlet and initial pressure (the outlet's p_out term), a closed box held at the inlet
temperature (the INLET thermal branch), and the deviation form against a literal
absolute-form statement of eq. 6-13 (tests/test_oracle_literal.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32),
                ("periodic_y", C.c_int32), ("check_interval", C.c_int32), ("outlet_mode", C.c_int32),
                ("bc_scheme", C.c_int32), ("pad_", C.c_int32),
                ("tau_f", C.c_double), ("tau_t", C.c_double), ("w0", C.c_double),
                ("u_in_x", C.c_double), ("u_in_y", C.c_double),
                ("p_ref", C.c_double), ("p_out", C.c_double), ("p_init", C.c_double),
                ("T_ref", C.c_double), ("T_init", C.c_double), ("T0", C.c_double),
                ("T_cornea", C.c_double), ("T_iris", C.c_double), ("T_inlet", C.c_double),
                ("gbeta", C.c_double), ("gravity_angle", C.c_double), ("K", C.c_double),
                ("K_tm", C.c_double), ("h_tm", C.c_double), ("p_sc", C.c_double)]


class OrObservables(C.Structure):
    _fields_ = [("step", C.c_int64)] + [(n, C.c_double) for n in (
        "iop_gauge", "p_mean_fluid", "q_in", "q_out", "wss_cornea_mean", "wss_cornea_max",
        "wss_iris_mean", "wss_iris_max", "resid_u", "resid_T", "u_max", "mass_flow",
        "mass_thermal")] + [("n_nonfinite", C.c_int64), ("u_seep", C.c_double)]

    def asdict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(OrParams), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_step.argtypes = [C.c_void_p, C.c_int64]
        L.or_step_count.argtypes = [C.c_void_p]
        L.or_step_count.restype = C.c_int64
        L.or_set_outlet.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        L.or_observables_get.argtypes = [C.c_void_p, C.POINTER(OrObservables)]
        L.or_observe.argtypes = [C.c_void_p, C.POINTER(OrObservables)]
        L.or_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.or_get_populations.argtypes = [C.c_void_p, dp, dp]
        L.or_set_populations.argtypes = [C.c_void_p, dp, dp]
        L.or_collide_node.argtypes = [C.POINTER(OrParams), C.c_int, dp, dp, dp, dp]
        L.or_equilibrium.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, C.c_double,
                                     C.c_double, dp, dp]
        L.or_moments.argtypes = [C.POINTER(OrParams), dp, dp, dp]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(p) -> OrParams:
    """Accept an aqinputs.Params (or any object/dict with the same field names)."""
    d = p if isinstance(p, dict) else p.asdict()
    op = OrParams()
    for name, _ in OrParams._fields_:
        if name != "pad_":
            setattr(op, name, d[name])
    return op


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().or_set_threads(int(n))


def max_threads() -> int:
    return lib().or_max_threads()


class Oracle:
    """One oracle lattice.  Populations are pre-collision, deviation form:
    h[q-1] = f_q - lambda_q p_ref (q = 1..8), g[q] = T_q - w^T_q T_ref (q = 0..4)."""

    def __init__(self, params, mask: np.ndarray, walls=None):
        self.params = params
        self._p = make_params(params)
        self.ny, self.nx = mask.shape
        assert self.nx == self._p.nx and self.ny == self._p.ny
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if walls is None or len(walls) == 0:
            node = np.zeros(1, np.int32); wid = np.zeros(1, np.int32)
            wnx = np.zeros(1); wny = np.zeros(1); nw = 0
            wq = -np.ones(8)
        else:
            node = np.ascontiguousarray(walls["node"], np.int32)
            wid = np.ascontiguousarray(walls["wall"], np.int32)
            wnx = np.ascontiguousarray(walls["nx"], np.float64)
            wny = np.ascontiguousarray(walls["ny"], np.float64)
            wq = (np.ascontiguousarray(walls["q"], np.float64) if "q" in walls.dtype.names
                  else -np.ones((len(walls), 8)))
            nw = len(walls)
        self._keep = (node, wid, wnx, wny, wq)
        self._s = lib().or_create(C.byref(self._p), self.mask.ctypes.data, nw, node.ctypes.data,
                                  wid.ctypes.data, wnx.ctypes.data, wny.ctypes.data, wq.ctypes.data)
        if not self._s:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        s = getattr(self, "_s", None)
        if s:
            lib().or_destroy(s)
            self._s = None

    def step(self, n: int):
        lib().or_step(self._s, int(n))
        return self

    def set_outlet(self, K_tm: float, h_tm: float, p_sc: float):
        """New lumped-meshwork constants; the seepage speed in effect is re-evaluated at
        once from the last check step's IOP (p_init before the first check)."""
        lib().or_set_outlet(self._s, K_tm, h_tm, p_sc)
        return self

    @property
    def steps(self) -> int:
        return lib().or_step_count(self._s)

    def observables(self) -> dict:
        o = OrObservables()
        lib().or_observables_get(self._s, C.byref(o))
        return o.asdict()

    def observe_now(self) -> dict:
        """The check-step observables of the current state, computed now."""
        o = OrObservables()
        lib().or_observe(self._s, C.byref(o))
        return o.asdict()

    def fields(self):
        """(p - p_ref, u_x, u_y, T) as [ny, nx] arrays, NaN at non-active nodes."""
        n = self.nx * self.ny
        out = [np.empty(n) for _ in range(4)]
        lib().or_fields(self._s, *[_dptr(a) for a in out])
        return [a.reshape(self.ny, self.nx) for a in out]

    def populations(self):
        n = self.nx * self.ny
        h = np.empty(8 * n)
        g = np.empty(5 * n)
        lib().or_get_populations(self._s, _dptr(h), _dptr(g))
        return h.reshape(8, self.ny, self.nx), g.reshape(5, self.ny, self.nx)

    def set_populations(self, h, g):
        h = np.ascontiguousarray(h, np.float64).reshape(-1)
        g = np.ascontiguousarray(g, np.float64).reshape(-1)
        lib().or_set_populations(self._s, _dptr(h), _dptr(g))


def collide_node(params, porous: bool, h8, g5):
    p = make_params(params)
    h8 = np.ascontiguousarray(h8, np.float64)
    g5 = np.ascontiguousarray(g5, np.float64)
    hs = np.empty(8)
    gs = np.empty(5)
    lib().or_collide_node(C.byref(p), int(porous), _dptr(h8), _dptr(g5), _dptr(hs), _dptr(gs))
    return hs, gs


def equilibrium(params, p, ux, uy, T):
    pp = make_params(params)
    h8 = np.empty(8)
    g5 = np.empty(5)
    lib().or_equilibrium(C.byref(pp), p, ux, uy, T, _dptr(h8), _dptr(g5))
    return h8, g5


def moments(params, h8, g5):
    pp = make_params(params)
    out = np.empty(4)
    lib().or_moments(C.byref(pp), _dptr(np.ascontiguousarray(h8, np.float64)),
                     _dptr(np.ascontiguousarray(g5, np.float64)), _dptr(out))
    return out
