"""The C-ABI library loads on the CPU and exports every symbol include/aqlbm.h declares;
argument validation fails with AQ_EINVAL before any device work (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import aqinputs as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def aq():
    import paper_2102_12663_amd as aq
    if not os.path.exists(aq.LIB_PATH):
        pytest.fail("libaqlbm.so is not built (run __graft_entry__.build())")
    aq.load_library()
    return aq


def _declared():
    src = open(os.path.join(ROOT, "include", "aqlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aq_[a-z_0-9]+)\s*\(", src)))


def test_header_and_exports_agree(aq):
    declared = _declared()
    assert declared == sorted(aq.EXPORTS)
    lib = C.CDLL(aq.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert aq.version().startswith("aqlbm")


def test_struct_layouts_match_header(aq, tmp_path):
    """Every ctypes structure of the binding has the size and field offsets that a C
    compiler gives the header's structure (compiled and run here with gcc)."""
    structs = {"aq_params": aq.AqParams, "aq_wall_node": aq.AqWallNode, "aq_observables": aq.AqObservables,
               "aq_info": aq.AqInfo, "aq_result": aq.AqResult, "aq_batch_info": aq.AqBatchInfo,
               "aq_diagnostics": aq.AqDiagnostics}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aqlbm.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def _create(aq, p, mask, walls=None):
    ap = aq.make_params(p)
    h = C.c_void_p()
    wptr, nw, keep = aq._walls(walls)
    rc = aq._lib.aq_create(C.byref(ap), np.ascontiguousarray(mask, np.uint8).ctypes.data, wptr, nw, C.byref(h))
    return rc, aq._lib.aq_last_error().decode()


@pytest.mark.parametrize("change,msg", [
    ({"tau_f": 0.5}, "tau"),
    ({"tau_t": 0.3}, "tau"),
    ({"storage": 7}, "storage"),
    ({"check_interval": 7}, "check_interval"),
    ({"check_interval": 0}, "check_interval"),
    ({"K": 0.0}, "K"),
    ({"w0": 1.0}, "w0"),
    ({"outlet_mode": 2}, "outlet_mode"),
    ({"outlet_mode": 1, "K_tm": 0.0}, "lumped"),
    ({"outlet_mode": 1, "h_tm": -1.0}, "lumped"),
    ({"outlet_mode": 1, "p_sc": float("nan")}, "lumped"),
])
def test_invalid_parameters_rejected(aq, change, msg):
    p, mask, walls, geo = A.config0()
    d = p.asdict()
    d.update(change)
    rc, err = _create(aq, A.Params(**d), mask, walls)
    assert rc == aq.AQ_EINVAL and msg in err


def test_invalid_masks_rejected(aq):
    p, mask, walls, geo = A.config0()
    bad = mask.copy()
    bad[0, 10] = A.encode(A.FLUID)
    assert _create(aq, p, bad, walls)[0] == aq.AQ_EINVAL
    bad = mask.copy()
    bad[5, 5] = 7
    assert _create(aq, p, bad, walls)[0] == aq.AQ_EINVAL
    w = walls.copy()
    w["node"][[0, 1]] = w["node"][[1, 0]]
    assert _create(aq, p, mask, w)[0] == aq.AQ_EINVAL


def test_required_bytes(aq):
    p, mask, walls, geo = A.config0()
    ap = aq.make_params(p)
    n = C.c_size_t()
    assert aq._lib.aq_required_bytes(C.byref(ap), mask.ctypes.data, C.byref(n)) == 0
    # two population buffers of 13 arrays of at least nx*ny doubles
    assert n.value >= 2 * 13 * 192 * 96 * 8
    p.storage = A.F16S
    ap = aq.make_params(p)
    m = C.c_size_t()
    assert aq._lib.aq_required_bytes(C.byref(ap), mask.ctypes.data, C.byref(m)) == 0
    assert m.value < n.value


@pytest.mark.parametrize("nx,ny", [(32769, 32767), (16384, 32768)])
def test_f32_plane_limit(aq, nx, ny):
    """F32 kernels address populations with 32-bit byte offsets from a plane base, and a
    boundary pull reaches two planes beyond the node's own slot: a lattice whose three
    padded planes (ny x nx rounded up to 64 columns, 4 bytes each) pass 4 GiB is rejected
    in F32 storage, although it has no more than 2^30 nodes (the second size: one plane
    of 2 GiB)."""
    assert nx * ny <= 1 << 30
    mask = np.zeros((ny, nx), np.uint8)        # never touched: the size check comes first
    p = A.Params(nx=nx, ny=ny, storage=A.F32)
    rc, err = _create(aq, p, mask)
    assert rc == aq.AQ_EINVAL and "4 GiB" in err


@pytest.mark.parametrize("nbytes,reps", [(100, 1), (1 << 20, 0), ((1 << 20) + 8, 1)])
def test_copy_bandwidth_rejects_invalid_sizes(aq, nbytes, reps):
    """aq_copy_bandwidth checks its arguments before touching a device: sizes below 1 MiB
    or not a multiple of 16 bytes, and no repetitions, are AQ_EINVAL."""
    g = C.c_double(-1.0)
    assert aq._lib.aq_copy_bandwidth(nbytes, reps, C.byref(g)) == aq.AQ_EINVAL
    assert g.value == -1.0


def test_fused_tile_rows_rejected_without_a_solver(aq):
    """aq_set_fused_tile_rows checks its handle before anything else."""
    assert aq._lib.aq_set_fused_tile_rows(None, 4) == aq.AQ_EINVAL


def test_batch_fused_tile_rows_rejected_without_a_batch(aq):
    """aq_batch_set_fused_tile_rows checks its handle before anything else."""
    assert aq._lib.aq_batch_set_fused_tile_rows(None, 4) == aq.AQ_EINVAL
