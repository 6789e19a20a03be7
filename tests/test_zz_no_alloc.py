"""aq_diagnose_noalloc (the library's fixed per-GPU workspace, no device allocation) against
aq_diagnose (a caller-provided workspace): the same kernels on the same state, so the
results must agree bit for bit.  Two calls in a row, the second on a smaller lattice, so
the second runs over what the first left in the shared array."""
import numpy as np
import pytest

import aqinputs as A
from gpu_util import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2102_12663_amd as aq
    aq.load_library()
    return aq


def _case(which):
    if which == "2048x1024":
        return A.sweep_instance(0, 2048, 1024)[:3]
    return A.config0()[:3]


@pytest.mark.parametrize("storage", [A.F64, A.F32])
def test_noalloc_matches_workspace_form_twice(aq, storage):
    for which in ("2048x1024", "192x96"):
        p, mask, walls = _case(which)
        p = A.Params(**{**p.asdict(), "storage": storage})
        s = aq.Solver(p, mask, walls)
        s.step(600)
        announce(f"[noalloc] {which} storage={storage}")
        got = s.diagnose_noalloc()
        want = s.diagnose()
        again = s.diagnose_noalloc()
        s.close()
        assert got == want, (which, got, want)
        assert again == want
        assert got["vortex_intensity"] > 0 and np.isfinite(got["psi_max"])


def test_noalloc_rejects_a_lattice_beyond_its_workspace(aq):
    """A lattice whose diagnostics need more than the fixed 64 MiB is refused before any
    launch, with a message naming the limit; the allocating form still serves it."""
    nx, ny = 3000, 1600                      # 2 x 4.8 M doubles of velocity alone: 77 MB
    mask = A.box_mask(nx, ny)
    p = A.Params(nx=nx, ny=ny, storage=A.F16S, check_interval=100, gbeta=1e-6)
    s = aq.Solver(p, mask, A.no_walls())
    s.step(2)
    with pytest.raises(Exception) as e:
        s.diagnose_noalloc()
    assert "fixed diagnostics workspace" in str(e.value)
    d = s.diagnose()
    s.close()
    assert np.isfinite(d["u_max_fluid"])
