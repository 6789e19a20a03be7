"""MI355X (gfx950) implementation of the coupled lattice Boltzmann model of aqueous-humour
dynamics of arXiv:2102.12663 (section 2.3): fused pull-stream/collide HIP kernels behind
the C-ABI of include/aqlbm.h.

This module only marshals arguments: every step of the method runs in the HIP library
`libaqlbm.so`.  PyTorch supplies the device arena and the HIP stream.  If the library is
missing, constructing a solver raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaqlbm.so")

AQ_OK, AQ_EINVAL, AQ_ENOMEM, AQ_EDEVICE, AQ_EDIVERGED, AQ_ENOTCONVERGED, AQ_EBUSY, AQ_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
AQ_RESULT_FLOOR = 1    # result status: F16S accepted at its rounding floor (IOP drift check passed)
F64, F32, F16S, F32X = 0, 1, 2, 3
FIELDS = {"p": 0, "ux": 1, "uy": 2, "T": 3, "pop_flow": 4, "pop_heat": 5}

# every symbol include/aqlbm.h declares
EXPORTS = ("aq_version", "aq_last_error", "aq_required_bytes", "aq_create", "aq_create_ext",
           "aq_destroy", "aq_step", "aq_run_to_steady", "aq_observe", "aq_read_field",
           "aq_write_populations", "aq_save", "aq_load", "aq_get_info", "aq_set_tile",
           "aq_time_step_kernel", "aq_run_intervals_timed", "aq_autotune_tile", "aq_set_fusion",
           "aq_time_fused_kernel", "aq_set_outlet",
           "aq_batch_create", "aq_batch_admit", "aq_batch_run", "aq_batch_poll", "aq_batch_read_field",
           "aq_batch_observe", "aq_batch_release", "aq_batch_get_info", "aq_batch_destroy",
           "aq_batch_set_outlet", "aq_batch_resume", "aq_diagnostics_bytes", "aq_diagnose",
           "aq_batch_diagnose", "aq_diagnose_noalloc", "aq_batch_run_timed", "aq_copy_bandwidth",
           "aq_set_fused_tile_rows", "aq_batch_set_fused_tile_rows")


class AqParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("storage", C.c_int32), ("check_interval", C.c_int32),
                ("fp16_exp_flow", C.c_int32), ("fp16_exp_thermal", C.c_int32),
                ("outlet_mode", C.c_int32), ("bc_scheme", C.c_int32), ("reserved1", C.c_int32)] + [
                    (n, C.c_double) for n in (
                    "tau_f", "tau_t", "w0", "u_in_x", "u_in_y", "p_ref", "p_out", "p_init",
                    "T_ref", "T_init", "T0", "T_cornea", "T_iris", "T_inlet", "gbeta",
                    "gravity_angle", "K", "K_tm", "h_tm", "p_sc")]


class AqWallNode(C.Structure):
    _fields_ = [("node", C.c_int32), ("wall", C.c_int32), ("n_x", C.c_double), ("n_y", C.c_double),
                ("q", C.c_double * 8)]


class AqObservables(C.Structure):
    _fields_ = [("step", C.c_int64)] + [(n, C.c_double) for n in (
        "iop_gauge", "p_mean_fluid", "q_in", "q_out", "wss_cornea_mean", "wss_cornea_max",
        "wss_iris_mean", "wss_iris_max", "resid_u", "resid_T", "u_max", "mass_flow",
        "mass_thermal")] + [("n_nonfinite", C.c_int64), ("u_seep", C.c_double)]

    def asdict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class AqDiagnostics(C.Structure):
    _fields_ = [("step", C.c_int64), ("vortex_intensity", C.c_double), ("u_max_fluid", C.c_double),
                ("psi_max", C.c_double), ("psi_min", C.c_double), ("psi_max_x", C.c_int32),
                ("psi_max_y", C.c_int32), ("psi_min_x", C.c_int32), ("psi_min_y", C.c_int32)]

    def asdict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class AqInfo(C.Structure):
    _fields_ = [("active_nodes", C.c_int64), ("fluid_nodes", C.c_int64), ("lattice_nodes", C.c_int64),
                ("nx", C.c_int32), ("ny", C.c_int32), ("pitch", C.c_int32), ("storage", C.c_int32),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("n_tiles", C.c_int32),
                ("check_interval", C.c_int32), ("fp16_exp_flow", C.c_int32),
                ("fp16_exp_thermal", C.c_int32), ("fusion", C.c_int32), ("graph_launches", C.c_int32),
                ("nt_store", C.c_int32), ("fused_tile_rows", C.c_int32),
                ("step", C.c_int64), ("device_bytes", C.c_size_t),
                ("bytes_per_node_update", C.c_double)]

    def asdict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class AqResult(C.Structure):
    _fields_ = [("request_id", C.c_int64), ("slot", C.c_int32), ("status", C.c_int32),
                ("storage", C.c_int32), ("fallback", C.c_int32), ("steps", C.c_int64),
                ("obs", AqObservables)]

    def asdict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "obs"}
        d["obs"] = self.obs.asdict()
        return d


class AqBatchInfo(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("running", C.c_int32), ("finished", C.c_int32),
                ("n_work", C.c_int32 * 4), ("active_nodes", C.c_int64), ("budget_bytes", C.c_size_t),
                ("used_bytes", C.c_size_t), ("largest_free_bytes", C.c_size_t), ("step", C.c_int64),
                ("fused_tile_rows", C.c_int32 * 4)]

    def asdict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n not in ("n_work", "fused_tile_rows")}
        d["n_work"] = list(self.n_work)
        d["fused_tile_rows"] = list(self.fused_tile_rows)
        return d


class AqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"aqlbm error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libaqlbm.so (raises if it has not been built).  torch, which provides the device
    memory and streams, brings up the HIP runtime first when a GPU is visible."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, sz, i32, i64, dp = C.c_void_p, C.c_size_t, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.aq_version.restype = C.c_char_p
    L.aq_last_error.restype = C.c_char_p
    L.aq_required_bytes.argtypes = [C.POINTER(AqParams), vp, C.POINTER(sz)]
    L.aq_create.argtypes = [C.POINTER(AqParams), vp, vp, i32, C.POINTER(vp)]
    L.aq_create_ext.argtypes = [C.POINTER(AqParams), vp, vp, i32, vp, sz, vp, C.POINTER(vp)]
    L.aq_destroy.argtypes = [vp]
    L.aq_step.argtypes = [vp, i64]
    L.aq_run_to_steady.argtypes = [vp, C.c_double, i64, C.POINTER(AqObservables)]
    L.aq_observe.argtypes = [vp, C.POINTER(AqObservables)]
    L.aq_read_field.argtypes = [vp, i32, i32, dp, sz]
    L.aq_write_populations.argtypes = [vp, dp, dp, sz]
    L.aq_save.argtypes = [vp, C.c_char_p]
    L.aq_load.argtypes = [vp, C.c_char_p]
    L.aq_get_info.argtypes = [vp, C.POINTER(AqInfo)]
    L.aq_set_tile.argtypes = [vp, i32, i32]
    L.aq_time_step_kernel.argtypes = [vp, i32, dp]
    L.aq_run_intervals_timed.argtypes = [vp, i32, dp, dp]
    ip = C.POINTER(i32)
    L.aq_set_fusion.argtypes = [vp, i32]
    L.aq_set_outlet.argtypes = [vp, C.c_double, C.c_double, C.c_double]
    L.aq_diagnostics_bytes.argtypes = [C.POINTER(AqParams), C.POINTER(sz)]
    L.aq_diagnose.argtypes = [vp, vp, sz, C.POINTER(AqDiagnostics)]
    L.aq_diagnose_noalloc.argtypes = [vp, C.POINTER(AqDiagnostics)]
    L.aq_batch_diagnose.argtypes = [vp, i32, vp, sz, C.POINTER(AqDiagnostics)]
    L.aq_batch_set_outlet.argtypes = [vp, i32, C.c_double, C.c_double, C.c_double]
    L.aq_batch_resume.argtypes = [vp, i32, C.c_double, i64]
    L.aq_time_fused_kernel.argtypes = [vp, i32, dp]
    L.aq_autotune_tile.argtypes = [vp, i32, i32, ip, ip, dp]
    L.aq_batch_create.argtypes = [sz, i32, i64, i32, i32, vp, C.POINTER(vp)]
    L.aq_batch_admit.argtypes = [vp, C.POINTER(AqParams), vp, vp, i32, i32, i32, C.c_double, C.c_double,
                                 i64, i64, i32, ip]
    L.aq_batch_run.argtypes = [vp, i32]
    L.aq_batch_run_timed.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i32)]
    L.aq_batch_poll.argtypes = [vp, C.POINTER(AqResult), i32, ip]
    L.aq_batch_read_field.argtypes = [vp, i32, i32, i32, dp, sz]
    L.aq_batch_observe.argtypes = [vp, i32, C.POINTER(AqObservables)]
    L.aq_batch_release.argtypes = [vp, i32]
    L.aq_batch_get_info.argtypes = [vp, C.POINTER(AqBatchInfo)]
    L.aq_batch_destroy.argtypes = [vp]
    L.aq_copy_bandwidth.argtypes = [sz, i32, C.POINTER(C.c_double)]
    L.aq_set_fused_tile_rows.argtypes = [vp, i32]
    L.aq_batch_set_fused_tile_rows.argtypes = [vp, i32]
    for name in EXPORTS:
        if name not in ("aq_version", "aq_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s (read + written bytes over time) of a plain device copy of nbytes, best of reps."""
    load_library()
    g = C.c_double()
    _check(_lib.aq_copy_bandwidth(nbytes, reps, C.byref(g)))
    return g.value


def _check(rc):
    if rc != AQ_OK:
        raise AqError(rc, _lib.aq_last_error().decode())
    return rc


def make_params(p) -> AqParams:
    """From an aqinputs.Params-like object or dict (periodic lattices are not supported
    by the HIP path)."""
    d = p if isinstance(p, dict) else p.asdict()
    if d.get("periodic_x") or d.get("periodic_y"):
        raise ValueError("the HIP path has no periodic boundaries")
    ap = AqParams()
    ap.struct_size = C.sizeof(AqParams)
    for name, _ in AqParams._fields_:
        if name in ("struct_size", "reserved0", "reserved1"):
            continue
        setattr(ap, name, d[name])
    return ap


def _walls(walls):
    if walls is None or len(walls) == 0:
        return None, 0, None
    arr = (AqWallNode * len(walls))()
    for i, w in enumerate(walls):
        arr[i].node, arr[i].wall, arr[i].n_x, arr[i].n_y = int(w["node"]), int(w["wall"]), float(w["nx"]), float(w["ny"])
        q = w["q"] if "q" in w.dtype.names else [-1.0] * 8
        for j in range(8):
            arr[i].q[j] = float(q[j])
    return C.cast(arr, C.c_void_p), len(walls), arr


class Solver:
    """One lattice on the GPU.  Device memory is a torch uint8 arena, work runs on a
    torch stream (default priority) owned by this object."""

    def __init__(self, params, mask, walls=None, device="cuda:0", stream=None):
        import torch
        L = load_library()
        self.params = params
        self._p = make_params(params)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = self.mask.shape
        if (self.nx, self.ny) != (self._p.nx, self._p.ny):
            raise ValueError("mask shape does not match nx, ny")
        nbytes = C.c_size_t()
        _check(L.aq_required_bytes(C.byref(self._p), self.mask.ctypes.data, C.byref(nbytes)))
        self.device = torch.device(device)
        self._arena = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self._arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        wptr, nw, self._warr = _walls(walls)
        h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        _check(L.aq_create_ext(C.byref(self._p), self.mask.ctypes.data, wptr, nw, C.c_void_p(aligned),
                               nbytes.value, C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.aq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- stepping
    def step(self, n: int):
        _check(_lib.aq_step(self._h, int(n)))
        return self

    def run_to_steady(self, tol: float, max_steps: int):
        o = AqObservables()
        rc = _lib.aq_run_to_steady(self._h, float(tol), int(max_steps), C.byref(o))
        if rc not in (AQ_OK, AQ_ENOTCONVERGED):
            _check(rc)
        return rc == AQ_OK, o.asdict()

    def synchronize(self):
        self._stream.synchronize()

    # --- outputs
    def observe(self) -> dict:
        o = AqObservables()
        _check(_lib.aq_observe(self._h, C.byref(o)))
        return o.asdict()

    def info(self) -> dict:
        i = AqInfo()
        _check(_lib.aq_get_info(self._h, C.byref(i)))
        return i.asdict()

    def read_field(self, name: str, q: int = 0) -> np.ndarray:
        out = np.empty(self.nx * self.ny)
        _check(_lib.aq_read_field(self._h, FIELDS[name], int(q),
                                  out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out.reshape(self.ny, self.nx)

    def fields(self):
        """(p - p_ref, u_x, u_y, T) like the oracle's fields()."""
        p = self.read_field("p") - self._p.p_ref
        return [p, self.read_field("ux"), self.read_field("uy"), self.read_field("T")]

    def populations(self):
        h = np.stack([self.read_field("pop_flow", q) for q in range(1, 9)])
        g = np.stack([self.read_field("pop_heat", q) for q in range(0, 5)])
        return h, g

    def write_populations(self, h, g):
        h = np.ascontiguousarray(h, np.float64).reshape(-1)
        g = np.ascontiguousarray(g, np.float64).reshape(-1)
        n = self.nx * self.ny
        assert h.size == 8 * n and g.size == 5 * n
        _check(_lib.aq_write_populations(self._h, h.ctypes.data_as(C.POINTER(C.c_double)),
                                         g.ctypes.data_as(C.POINTER(C.c_double)), n))

    # --- tuning and timing
    def set_tile(self, tx: int, ty: int):
        _check(_lib.aq_set_tile(self._h, int(tx), int(ty)))

    def diagnose(self) -> dict:
        """Vortex intensity, max |u| over FLUID nodes and the stream-function extrema with
        their nodes (aq_diagnose); the device workspace is allocated once and kept."""
        import torch
        nb = C.c_size_t()
        _check(_lib.aq_diagnostics_bytes(C.byref(self._p), C.byref(nb)))
        if getattr(self, "_diag_ws", None) is None or self._diag_ws.numel() < nb.value:
            torch.cuda.synchronize(self.device)
            self._diag_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
        d = AqDiagnostics()
        _check(_lib.aq_diagnose(self._h, C.c_void_p(self._diag_ws.data_ptr()), nb.value, C.byref(d)))
        return d.asdict()

    def diagnose_noalloc(self) -> dict:
        """The same diagnostics through aq_diagnose_noalloc: the library's fixed per-GPU
        workspace, no allocation (lattices up to 64 MiB of workspace)."""
        d = AqDiagnostics()
        _check(_lib.aq_diagnose_noalloc(self._h, C.byref(d)))
        return d.asdict()

    def set_outlet(self, K_tm: float, h_tm: float, p_sc: float):
        """Lumped meshwork: new permeability, thickness and canal pressure; the seepage
        speed in effect is re-evaluated at once from the last check step's IOP."""
        _check(_lib.aq_set_outlet(self._h, float(K_tm), float(h_tm), float(p_sc)))

    def set_fused_tile_rows(self, rows: int):
        _check(_lib.aq_set_fused_tile_rows(self._h, rows))

    def set_fusion(self, enable: bool):
        _check(_lib.aq_set_fusion(self._h, int(bool(enable))))

    def time_fused_kernel(self, n_launch: int) -> float:
        ms = C.c_double()
        _check(_lib.aq_time_fused_kernel(self._h, int(n_launch), C.byref(ms)))
        return ms.value

    def time_step_kernel(self, n_launch: int) -> float:
        ms = C.c_double()
        _check(_lib.aq_time_step_kernel(self._h, int(n_launch), C.byref(ms)))
        return ms.value

    def run_intervals_timed(self, n: int):
        tot, plain = C.c_double(), C.c_double()
        _check(_lib.aq_run_intervals_timed(self._h, int(n), C.byref(tot), C.byref(plain)))
        return tot.value, plain.value

    def autotune(self, n_launch: int = 20, only_256: bool = False):
        tx, ty, ms = C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.aq_autotune_tile(self._h, int(n_launch), int(only_256), C.byref(tx), C.byref(ty), C.byref(ms)))
        return tx.value, ty.value, ms.value

    def save(self, path: str):
        _check(_lib.aq_save(self._h, path.encode()))

    def load(self, path: str):
        _check(_lib.aq_load(self._h, path.encode()))


class Batch:
    """Continuously batched solves (include/aqlbm.h, aq_batch_*).  The batch allocates its
    instance arena once; work runs on a torch stream (default priority) owned here."""

    def __init__(self, budget_bytes: int, max_slots: int = 512, max_active_nodes: int = 0,
                 max_tiles: int = 1 << 20, check_interval: int = 100, device="cuda:0", stream=None):
        import torch
        load_library()
        self._stream = stream if stream is not None else torch.cuda.Stream(device=torch.device(device))
        h = C.c_void_p()
        _check(_lib.aq_batch_create(int(budget_bytes), int(max_slots), int(max_active_nodes), int(max_tiles),
                                    int(check_interval), C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self._h = h
        self._keep = {}
        self.shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.aq_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, params, mask, walls=None, tile=(64, 4), tol=1e-6, drift_tol=1e-3,
              max_steps=10 ** 7, request_id=0, keep=False):
        """Slot number, or None when the batch is full (AQ_EBUSY)."""
        p = make_params(params)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        wptr, nw, warr = _walls(walls)
        slot = C.c_int32()
        rc = _lib.aq_batch_admit(self._h, C.byref(p), mask.ctypes.data, wptr, nw, int(tile[0]), int(tile[1]),
                                 float(tol), float(drift_tol), int(max_steps), int(request_id), int(keep),
                                 C.byref(slot))
        if rc == AQ_EBUSY:
            return None
        _check(rc)
        self.shapes[slot.value] = mask.shape
        return slot.value

    def run(self, n_intervals: int = 1):
        _check(_lib.aq_batch_run(self._h, int(n_intervals)))

    def run_timed(self, n_intervals: int = 1):
        """aq_batch_run_timed: (total ms, ms in the two-step launches, number of them)."""
        tot, fused, nl = C.c_double(), C.c_double(), C.c_int32()
        _check(_lib.aq_batch_run_timed(self._h, int(n_intervals), C.byref(tot), C.byref(fused), C.byref(nl)))
        return tot.value, fused.value, nl.value

    def poll(self, cap: int = 4096):
        buf = (AqResult * cap)()
        n = C.c_int32()
        _check(_lib.aq_batch_poll(self._h, buf, int(cap), C.byref(n)))
        return [buf[i].asdict() for i in range(n.value)]

    def read_field(self, slot: int, name: str, q: int = 0):
        ny, nx = self.shapes[slot]
        out = np.empty(nx * ny)
        _check(_lib.aq_batch_read_field(self._h, int(slot), FIELDS[name], int(q),
                                        out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out.reshape(ny, nx)

    def observe(self, slot: int) -> dict:
        o = AqObservables()
        _check(_lib.aq_batch_observe(self._h, int(slot), C.byref(o)))
        return o.asdict()

    def diagnose(self, slot: int, params) -> dict:
        """aq_batch_diagnose; `params` are the instance's (for the workspace size)."""
        import torch
        nb = C.c_size_t()
        ap = make_params(params)
        _check(_lib.aq_diagnostics_bytes(C.byref(ap), C.byref(nb)))
        if getattr(self, "_diag_ws", None) is None or self._diag_ws.numel() < nb.value:
            torch.cuda.synchronize()
            self._diag_ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
        d = AqDiagnostics()
        _check(_lib.aq_batch_diagnose(self._h, int(slot), C.c_void_p(self._diag_ws.data_ptr()), nb.value,
                                      C.byref(d)))
        return d.asdict()

    def set_outlet(self, slot: int, K_tm: float, h_tm: float, p_sc: float):
        _check(_lib.aq_batch_set_outlet(self._h, int(slot), float(K_tm), float(h_tm), float(p_sc)))

    def resume(self, slot: int, tol: float, max_steps: int) -> bool:
        """Warm-start a finished kept instance; False when the batch has no room now."""
        rc = _lib.aq_batch_resume(self._h, int(slot), float(tol), int(max_steps))
        if rc == AQ_EBUSY:
            return False
        _check(rc)
        return True

    def release(self, slot: int):
        _check(_lib.aq_batch_release(self._h, int(slot)))

    def set_fused_tile_rows(self, rows: int):
        """Two-step tile rows of the F32 and F16S instances: 0 by size, 4 or 8
        (aq_batch_set_fused_tile_rows)."""
        _check(_lib.aq_batch_set_fused_tile_rows(self._h, int(rows)))

    def info(self) -> dict:
        i = AqBatchInfo()
        _check(_lib.aq_batch_get_info(self._h, C.byref(i)))
        return i.asdict()


def required_bytes(params, mask) -> int:
    """Device bytes one lattice needs (aq_required_bytes)."""
    load_library()
    p = make_params(params)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    n = C.c_size_t()
    _check(_lib.aq_required_bytes(C.byref(p), m.ctypes.data, C.byref(n)))
    return n.value


def version() -> str:
    return load_library().aq_version().decode()
