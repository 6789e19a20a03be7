"""Shared helpers for the GPU parity tests (HIP library vs the FP64 oracle)."""
import sys

import numpy as np

import aqinputs as A

FIELD_NAMES = ("dp", "ux", "uy", "T")


def field_errors(gpu_fields, ora_fields, mask, T_ref):
    """Normwise error per field over active nodes: max|gpu - oracle| / max|oracle|,
    with T measured from T_ref."""
    act = A.active(mask)
    out = {}
    for name, G, O in zip(FIELD_NAMES, gpu_fields, ora_fields):
        g, o = G[act], O[act]
        if name == "T":
            g, o = g - T_ref, o - T_ref
        scale = np.max(np.abs(o))
        out[name] = float(np.max(np.abs(g - o)) / scale) if scale > 0 else float(np.max(np.abs(g - o)))
    return out


def obs_close(a, b, rel, keys=None, floor=1e-300):
    """Relative agreement of observables (dicts), with an absolute floor per key."""
    bad = {}
    for k in keys or [k for k in a if k not in ("step", "n_nonfinite")]:
        x, y = a[k], b[k]
        den = max(abs(x), abs(y), floor)
        if abs(x - y) > rel * den:
            bad[k] = (x, y)
    return bad


def announce(msg):
    print(msg, flush=True)
    sys.stdout.flush()
