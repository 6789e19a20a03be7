"""Device vortex diagnostics (aq_diagnose; eq. 18, Table 3) against the numpy definitions
in oracle/diagnostics.py applied to the oracle's own state."""
import numpy as np
import pytest

import aqinputs as A
import oracle as O
from gpu_util import announce
from oracle import diagnostics as D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    return aq


def _compare(g, o):
    assert g["vortex_intensity"] == pytest.approx(o["vortex_intensity"], rel=1e-12)
    assert g["u_max_fluid"] == pytest.approx(o["u_max_fluid"], rel=1e-12)
    scale = max(abs(o["psi_max"]), abs(o["psi_min"]))
    assert abs(g["psi_max"] - o["psi_max"]) <= 1e-12 * scale
    assert abs(g["psi_min"] - o["psi_min"]) <= 1e-12 * scale
    assert (g["psi_max_x"], g["psi_max_y"]) == (o["psi_max_x"], o["psi_max_y"])
    assert (g["psi_min_x"], g["psi_min_y"]) == (o["psi_min_x"], o["psi_min_y"])


def _standing():
    mask, walls, geo = A.eye_mask(200, 100, 40.0)
    p = A.eye_params(200, 100, geo, Ra=2e3, Da=1e-3, phi_deg=90.0)
    return p, mask, walls


@pytest.mark.parametrize("case", ["config0", "standing"])
def test_diagnostics_match_oracle(aq, case):
    p, mask, walls = (A.config0()[:3] if case == "config0" else _standing())
    announce(f"[diagnostics] {case} {p.nx}x{p.ny}")
    s = aq.Solver(p, mask, walls)
    s.step(1000)
    o = O.Oracle(p, mask, walls).step(1000)
    dp, ux, uy, T = o.fields()
    g = s.diagnose()
    ref = D.diagnose(ux, uy, mask)
    announce(f"[diagnostics] gpu {g}")
    assert g["step"] == 1000
    _compare(g, ref)
    assert g == s.diagnose()          # deterministic, and the state is unchanged
    s.close()


def test_batch_diagnose_equals_solo(aq):
    p, mask, walls = _standing()
    b = aq.Batch(budget_bytes=512 << 20, max_slots=4)
    sl = b.admit(p, mask, walls, tile=(64, 4), tol=1e-14, max_steps=10 ** 6, keep=True)
    b.run(5)
    solo = aq.Solver(p, mask, walls)
    solo.set_tile(64, 4)
    solo.step(500)
    assert b.diagnose(sl, p) == solo.diagnose()
    solo.close()
    b.close()
