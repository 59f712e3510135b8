"""The whole 512-tube batch workload (inputs.tube_batch(512, seed 4): lengths
200-4000, temperature ratios 1.1-2, eta/s in {0.01, ..., 0.5}), 500 steps in
one persistent launch -- the launch the benchmark times -- against the
oracle's fields of every tube (golden/oracle_tube_batch.npz, written by
make_tube_batch.py from the oracle alone) on 28-32 sampled cells per tube,
each relative to the largest value of its field over the whole tube (the
4-velocity as a 4-vector).  Tubes the oracle flags non-physical must be
flagged on the GPU and only those.  The float64 bar of a tube is 1e-12, or
three times the spread between two float64 formulations of the oracle
(Table I projection, Appendix B closed form) where that is larger; mixed
precision is held to 1e-5."""
import os

import numpy as np
import pytest

from gpu_util import note
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "oracle_tube_batch.npz")
STEPS = 500


@pytest.mark.skipif(not os.path.exists(GOLD), reason="oracle fields of the tube batch not generated")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_tube_of_the_batch_matches_the_oracle(precision):
    spec = inputs.tube_batch(512, 4)
    ref = np.load(GOLD)
    b = rlb.Batch([dict(n=t["N"], eta_s=t["eta_s"]) for t in spec], precision=precision)
    for j, t in enumerate(spec):
        b.init_tube(j, *inputs.shock_tube(t["N"], t["T_left"], t["T_right"]))
    note("batch %s: 512 tubes, %d steps in one launch" % (precision, STEPS))
    b.step(STEPS)
    worst, checked, flagged = 0.0, 0, 0
    for j in range(len(spec)):
        flags, t = b.status(j)
        assert t == STEPS
        oflags = int(ref["t%d_flags" % j])
        assert bool(flags) == bool(oflags), (j, flags, oflags)
        if oflags:
            flagged += 1
            continue
        got = b.read_tube(j)
        cells = ref["t%d_cells" % j]
        scale = ref["t%d_scale" % j]
        err = max(np.max(np.abs(got["n"][cells] - ref["t%d_n" % j])) / scale[0],
                  np.max(np.abs(got["eps"][cells] - ref["t%d_eps" % j])) / scale[1],
                  np.max(np.abs(got["U"][:, cells] - ref["t%d_U" % j])) / scale[2])
        bar = 1e-5 if precision == "mixed" else max(1e-12, 3.0 * float(np.max(ref["t%d_spread" % j])))
        assert err <= bar, (j, spec[j], err, bar)
        worst = max(worst, err / bar)
        checked += 1
    note("%d tubes within their bar (largest error / bar %.2f), %d flagged as on the oracle"
         % (checked, worst, flagged))
