"""The seeded input generators: splitmix64, the eye-section mask and the wall list."""
import math

import numpy as np
import pytest

import aqinputs as A


def test_splitmix64_published_values():
    # first outputs of splitmix64 seeded with 0 (published reference sequence)
    assert A.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert A.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert A.splitmix64(0, 2) == 0x06C45D188009454F
    u = [A.uniform01(s, k) for s in range(50) for k in range(8)]
    assert 0.0 <= min(u) and max(u) < 1.0


@pytest.mark.parametrize("nx,ny,alpha", [(192, 96, 45.0), (256, 128, 25.0), (512, 256, 37.0),
                                         (768, 384, 44.0)])
def test_eye_mask_structure(nx, ny, alpha):
    R = 80.0 if nx == 192 else None
    mask, walls, geo = A.eye_mask(nx, ny, alpha, R=R)
    cls = mask & 7
    # frame never active, mirror symmetric, both porous blocks and outlets present
    act = A.active(mask)
    assert not act[0].any() and not act[-1].any() and not act[:, 0].any() and not act[:, -1].any()
    assert np.array_equal(mask, mask[:, ::-1])
    assert (cls == A.POROUS).sum() == 2 * 32 * geo.s * geo.s
    assert (cls == A.OUTLET).sum() == 2 * 8 * geo.s
    assert (cls == A.INLET).sum() >= 2
    # chamber angle and depth: the arc meets the floor's half-way line at angle alpha
    assert geo.depth == pytest.approx(geo.R * (1 - math.cos(math.radians(alpha))))
    assert geo.yc + geo.R == pytest.approx(geo.jf - 0.5 + geo.depth)
    # every inlet cell has fluid directly above it
    iy, ix = np.nonzero(cls == A.INLET)
    assert np.all(cls[iy + 1, ix] == A.FLUID)


def test_wall_list_brute_force():
    mask, walls, geo = A.eye_mask(192, 96, 45.0, R=80.0)
    ny, nx = mask.shape
    cls, wl = mask & 7, (mask >> 3) & 3
    want = {}
    for y in range(1, ny - 1):
        for x in range(1, nx - 1):
            if cls[y, x] != A.FLUID:
                continue
            ids = set()
            for ex, ey in [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]:
                if cls[y + ey, x + ex] == A.SOLID and wl[y + ey, x + ex] in (1, 2):
                    ids.add(int(wl[y + ey, x + ex]))
            if ids:
                want[y * nx + x] = 1 if 1 in ids else 2
    assert list(walls["node"]) == sorted(want)
    assert [want[k] for k in walls["node"]] == list(walls["wall"])
    assert np.allclose(np.hypot(walls["nx"], walls["ny"]), 1.0)
    # cornea normals point toward the circle's centre (into the chamber)
    c = walls["wall"] == A.WALL_CORNEA
    x = walls["node"][c] % nx
    y = walls["node"][c] // nx
    assert np.all((geo.xc - x) * walls["nx"][c] + (geo.yc - y) * walls["ny"][c] > 0)


def test_sweep_draws_in_range():
    for seed in range(20):
        p, mask, walls, geo = A.sweep_instance(seed, 256, 128, tau_f="draw", phi_deg="draw")
        assert 25.0 <= geo.alpha_deg <= 45.0
        assert 0.5e-4 <= p.u_in_y <= 2e-4
        assert 0.55 <= p.tau_f <= 1.2
        assert 0.0 <= p.gravity_angle <= math.pi / 2
        assert A.batch_size_of(seed) in A.BATCH_SIZES
