"""Meshwork-thickness calibration (section 3.1's healthy-eye procedure) on the GPU:
changing the lumped meshwork of a live solve matches the oracle doing the same, and the
batched calibration loop (warm restarts of resident solves) lands on the closed-form
thickness h* = target K A / (mu Q_in)."""
import numpy as np
import pytest

import aqinputs as A
import oracle as O
from gpu_util import announce, field_errors, obs_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    return aq


E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def _area(mask):
    cls, d = mask & 7, (mask >> 3) & 3
    area = 0.0
    for y, x in zip(*np.nonzero(A.active(mask))):
        for i in range(1, 9):
            yy, xx = y + E[i][1], x + E[i][0]
            if cls[yy, xx] == A.OUTLET:
                n = E[d[yy, xx] + 1]
                area += 6 * W[i] * (E[i][0] * n[0] + E[i][1] * n[1])
    return area


@pytest.mark.parametrize("first", [1000, 1037])
def test_set_outlet_matches_oracle(aq, first):
    """Thickness changed at a check step (1000) or between checks (1037): the read-out right
    after the change is unchanged, and 463 more steps match the oracle."""
    mask, walls, geo = A.eye_mask(192, 96, 45.0, R=80.0, pupil_gap=2, tm="lumped")
    p = A.eye_params(192, 96, geo, tm="lumped")
    p.p_init = p.p_sc + 1e-4
    announce(f"[calibration] set_outlet after {first} steps")
    s = aq.Solver(p, mask, walls)
    o = O.Oracle(p, mask, walls)
    s.step(first)
    o.step(first)
    before = s.fields()
    s.set_outlet(p.K_tm, 1.7 * p.h_tm, p.p_sc)
    o.set_outlet(p.K_tm, 1.7 * p.h_tm, p.p_sc)
    after = s.fields()
    assert all(np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0)) for x, y in zip(before, after))
    s.step(1500 - first)
    o.step(1500 - first)
    err = field_errors(s.fields(), o.fields(), mask, p.T_ref)
    assert all(v <= 1e-12 for v in err.values()), err
    bad = obs_close(s.observe(), o.observables(), 1e-11, keys=["iop_gauge", "q_out", "u_seep", "resid_u"])
    assert not bad, bad
    s.close()


def test_batched_calibration_reaches_closed_form(aq):
    from paper_2102_12663_amd import serve as S
    eyes, targets, h_star = [], [], []
    for alpha, u_in in ((45.0, 1e-4), (38.0, 1.5e-4), (30.0, 0.7e-4)):
        mask, walls, geo = A.eye_mask(128, 64, alpha, tm="lumped")
        p = A.eye_params(128, 64, geo, Ra=0.0, Da=1e-3, u_in=u_in, tm="lumped")
        nu = (2 * p.tau_f - 1) / 6
        area = _area(mask)
        q_in = u_in * (geo.inlet_cols[1] - geo.inlet_cols[0] + 1)
        rise0 = nu * p.h_tm * q_in / (p.K_tm * area)
        targets.append(1.25 * rise0)
        h_star.append(targets[-1] * p.K_tm * area / (nu * q_in))
        eyes.append((p, mask, walls))
    res = S.calibrate(eyes, targets, tol=1e-10, iop_rtol=1e-7, max_steps=400000)
    announce(f"[calibration] {({k: v for k, v in res.items() if k != 'records'})}")
    assert res["calibrated"] == 3
    for i, e in res["records"].items():
        assert e["rounds"] <= 3, e
        assert e["h"][-1] == pytest.approx(h_star[i], rel=1e-6), (e, h_star[i])


def test_resume_rules(aq):
    mask, walls, geo = A.eye_mask(96, 48, 45.0, R=40.0, pupil_gap=2, tm="lumped")
    p = A.eye_params(96, 48, geo, Ra=0.0, Da=1e-3, tm="lumped")
    b = aq.Batch(budget_bytes=256 << 20, max_slots=2)
    sl = b.admit(p, mask, walls, tol=1e-6, max_steps=10 ** 6, keep=True)
    with pytest.raises(aq.AqError):
        b.resume(sl, 1e-8, 1000)          # still running
    while not b.poll():
        b.run(5)
    assert b.resume(sl, 1e-8, 1000) is True
    assert b.info()["running"] == 1
    b.close()
