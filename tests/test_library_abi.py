"""The C-ABI library loads on the CPU and exports every symbol include/aqlbm.h declares;
argument validation fails with AQ_EINVAL before any device work (no GPU needed)."""
import ctypes as C
import os
import re

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


def test_struct_sizes_match_header(aq):
    # aq_params: 8 int32 + 17 doubles; aq_wall_node: 2 int32 + 2 doubles
    assert C.sizeof(aq.AqParams) == 8 * 4 + 17 * 8
    assert C.sizeof(aq.AqWallNode) == 24
    assert C.sizeof(aq.AqObservables) == 8 + 13 * 8 + 8


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
