"""Writes oracle_long_runs.npz: fields of long oracle runs used by
test_gpu_long_runs.py.  Calls only the oracle and the seeded input
generator.  Run from the repository root:

    python tests/golden/make_oracle_runs.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import rlb  # noqa: E402
from paper_1301_3423_amd import inputs  # noqa: E402

# name: (shape, field recipe, relaxation, checkpoints)
RUNS = {
    "box": ((16, 12, 10), ("box", 0.6, 3), dict(eta_s=0.5), (500, 2000)),
    "tube": ((1, 1, 400), ("tube", 0.5), dict(eta_s=0.1), (500, 2000)),
}


def fields_of(shape, recipe):
    if recipe[0] == "box":
        return inputs.random_box(*shape, recipe[1], seed=recipe[2])
    return inputs.shock_tube(shape[2], 1.0, recipe[1])


def main():
    lat = oracle.load_lattice()
    out = {}
    for name, (shape, recipe, relax, checkpoints) in RUNS.items():
        s = rlb.Solver(*shape, lat=lat, **relax)
        s.init_fields(*fields_of(shape, recipe))
        for cp in checkpoints:
            s.step(cp - s.t)
            r = s.read_fields()
            for k in ("n", "eps", "U", "P"):
                out["%s_t%d_%s" % (name, cp, k)] = r[k]
            out["%s_t%d_flags" % (name, cp)] = np.array(r["flags"])
            print(name, cp, "flags", r["flags"], flush=True)
    np.savez_compressed(os.path.join(HERE, "oracle_long_runs.npz"), **out)


if __name__ == "__main__":
    main()
