"""Helpers shared by the GPU tests: run the library and the oracle on the
same seeded inputs and compare (max-norm relative error per field)."""
import sys

import numpy as np

from oracle import rlb as orlb
from paper_1301_3423_amd import rlb

FIELDS = ("n", "eps", "U0", "U1", "U2", "U3", "P")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def split(out):
    d = dict(n=out["n"], eps=out["eps"], P=out["P"])
    for k in range(4):
        d["U%d" % k] = out["U"][k]
    return d


def field_errors(gpu, ref):
    """max_x |F_gpu - F_ref| / scale(F) for every field.  The scale of n,
    eps, P and U^0 is max_x |F_ref|; the spatial components U^1..U^3 share
    one scale, the largest |U^j_ref| over x and j, because a component that
    vanishes in the continuum (the transverse flow of a shock tube, a pure
    lattice artefact here) would otherwise turn rounding into a large ratio;
    that scale is at least 1e-3 max|U^0_ref|, so a state at rest (spatial
    components pure rounding on both sides) is measured against the
    4-velocity's size."""
    g, r = split(gpu), split(ref)
    vscale = max(max(np.max(np.abs(r["U%d" % j])) for j in (1, 2, 3)), 1e-3 * np.max(np.abs(r["U0"])))
    out = {}
    for k in FIELDS:
        scale = vscale if k in ("U1", "U2", "U3") else np.max(np.abs(r[k]))
        out[k] = float(np.max(np.abs(g[k] - r[k])) / scale) if scale > 0 else float(np.max(np.abs(g[k])))
    return out


def run_pair(lat, shape, fields, steps, precision="fp64", **relax):
    """Initialise both sides with the same fields, advance `steps`, read."""
    nx, ny, nz = shape
    note("case shape=%s steps=%d precision=%s relax=%s" % (shape, steps, precision, relax))
    s = rlb.Solver(nx, ny, nz, precision=precision, **relax)
    s.init_fields(*fields)
    s.step(steps)
    gpu = s.read_fields()
    flags, t = s.status()
    o = orlb.Solver(nx, ny, nz, lat=lat, **relax)
    o.init_fields(*fields)
    o.step(steps)
    ref = o.read_fields()
    return gpu, ref, flags, t, s, o
