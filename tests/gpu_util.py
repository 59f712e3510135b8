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
    """max_x |F_gpu - F_ref| / scale(F).  For n, eps and P the scale is
    max_x |F_ref|.  The 4-velocity is compared as a 4-vector: every
    component U^0..U^3 against max_{x,mu} |U^mu_ref| (which is max U^0 >= 1),
    because a spatial component can vanish (a state at rest, the transverse
    flow of a shock tube, a decayed flow) and a per-component ratio would
    then measure rounding against nothing."""
    g, r = split(gpu), split(ref)
    uscale = max(np.max(np.abs(r["U%d" % j])) for j in range(4))
    out = {}
    for k in FIELDS:
        scale = uscale if k.startswith("U") else np.max(np.abs(r[k]))
        out[k] = float(np.max(np.abs(g[k] - r[k])) / scale)
    comp = component_errors(gpu, ref)
    note("  U errors, 4-vector scale / own scale: %s" % "  ".join(
        "U%d %.2e / %.2e" % (j, out["U%d" % j], comp["U%d" % j]) for j in range(4)))
    return out


def component_errors(gpu, ref):
    """The per-component form of the velocity error: max_x |U^j_gpu - U^j_ref|
    / max_x |U^j_ref| for each j separately (infinite where the reference
    component is zero everywhere).  Reported beside the 4-vector form; how
    much of it plain rounding explains on the long runs is measured in
    test_oracle_conditioning.py."""
    g, r = split(gpu), split(ref)
    out = {}
    for j in range(4):
        k = "U%d" % j
        scale = np.max(np.abs(r[k]))
        diff = np.max(np.abs(g[k] - r[k]))
        out[k] = float(diff / scale) if scale > 0 else (0.0 if diff == 0 else float("inf"))
    return out


def run_pair(lat, shape, fields, steps, precision="fp64", order=3, **relax):
    """Initialise both sides with the same fields, advance `steps`, read.
    `lat` is the oracle lattice of model `order`."""
    nx, ny, nz = shape
    note("case order=%d shape=%s steps=%d precision=%s relax=%s" % (order, shape, steps, precision, relax))
    s = rlb.Solver(nx, ny, nz, precision=precision, order=order, **relax)
    s.init_fields(*fields)
    s.step(steps)
    gpu = s.read_fields()
    flags, t = s.status()
    o = orlb.Solver(nx, ny, nz, lat=lat, order=order, **relax)
    o.init_fields(*fields)
    o.step(steps)
    ref = o.read_fields()
    return gpu, ref, flags, t, s, o
