"""Long runs against stored oracle fields (tests/golden/
oracle_long_runs.npz, written by make_oracle_runs.py from the oracle
only): 2000 steps of boxes and tubes of both models, 1000 steps of a channel
and a closed tube with walls.  The error of the float64 path stays at
rounding level and the mixed path within its tolerance over the length of
the runs; errors are taken over the fluid cells."""
import os

import numpy as np
import pytest

from gpu_util import field_errors, note
from paper_1301_3423_amd import rlb

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = np.load(os.path.join(HERE, "golden", "oracle_long_runs.npz"))

import importlib.util  # noqa: E402

_spec = importlib.util.spec_from_file_location("make_oracle_runs", os.path.join(HERE, "golden", "make_oracle_runs.py"))
_mk = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(_mk)

TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(_mk.RUNS))
def test_long_run(name, precision):
    shape, recipe, relax, checkpoints, order, walls = _mk.RUNS[name]
    note("long run %s %s %s order %d walls %s" % (name, shape, precision, order, walls))
    s = rlb.Solver(*shape, precision=precision, order=order, **relax)
    solid = _mk.solid_of(shape, walls)
    if solid is not None:
        s.set_walls(solid)
    fluid = np.ones(np.prod(shape), dtype=bool) if solid is None else ~solid.ravel()
    s.init_fields(*_mk.fields_of(shape, recipe))
    for cp in checkpoints:
        s.step(cp - s.status()[1])
        got = s.read_fields()
        ref = {k: GOLD["%s_t%d_%s" % (name, cp, k)] for k in ("n", "eps", "U", "P")}
        sel = lambda d: {k: (v[:, fluid] if k == "U" else v[fluid]) for k, v in d.items() if k in ("n", "eps", "U", "P")}
        err = field_errors(sel(got), sel(ref))
        note("  t=%d max err %.2e (%s)" % (cp, max(err.values()), max(err, key=err.get)))
        assert s.status()[0] == 0
        assert max(err.values()) <= TOL[precision], (cp, err)
