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

from oracle import rlb  # noqa: E402
from oracle.lattice import model_lattice  # noqa: E402
from paper_1301_3423_amd import inputs  # noqa: E402

# name: (shape, field recipe, relaxation, checkpoints, model order, walls)
RUNS = {
    "box": ((16, 12, 10), ("box", 0.6, 3), dict(eta_s=0.5), (500, 2000), 3, None),
    "tube": ((1, 1, 400), ("tube", 0.5), dict(eta_s=0.1), (500, 2000), 3, None),
    "box_order2": ((16, 12, 10), ("box", 0.6, 3), dict(eta_s=0.5), (500, 2000), 2, None),
    "tube_order2": ((1, 1, 400), ("tube", 0.5), dict(eta_s=0.1), (500, 2000), 2, None),
    # a channel: solid slabs of 6 cells at both y ends, flow along x
    "channel": ((8, 24, 6), ("box", 0.3, 4), dict(eta_s=0.2), (250, 1000), 3, ("slabs", 1, 6)),
    # a closed shock tube: solid slabs of 6 cells at both z ends
    "closed_tube": ((1, 1, 300), ("tube", 0.5), dict(eta_s=0.1), (250, 1000), 3, ("slabs", 0, 6)),
}


def fields_of(shape, recipe):
    if recipe[0] == "box":
        return inputs.random_box(*shape, recipe[1], seed=recipe[2])
    return inputs.shock_tube(shape[2], 1.0, recipe[1])


def solid_of(shape, walls):
    """Solid mask [nz, ny, nx] of a wall recipe (None: no walls); axis 0 is z,
    1 is y of the mask array."""
    if walls is None:
        return None
    nx, ny, nz = shape
    kind, axis, thick = walls
    assert kind == "slabs"
    m = np.zeros((nz, ny, nx), dtype=bool)
    idx = [slice(None)] * 3
    idx[axis] = slice(0, thick)
    m[tuple(idx)] = True
    idx[axis] = slice(m.shape[axis] - thick, m.shape[axis])
    m[tuple(idx)] = True
    return m


def main():
    out = {}
    for name, (shape, recipe, relax, checkpoints, order, walls) in RUNS.items():
        s = rlb.Solver(*shape, lat=model_lattice(order), order=order, solid=solid_of(shape, walls), **relax)
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
