"""Writes oracle_tube_batch.npz: the oracle's fields of every tube of the
512-tube batch workload (inputs.tube_batch(512, seed 4), 500 steps), on a
seeded sample of cells per tube, for test_gpu_tube_batch.py.  Calls only the
oracle and the seeded input generators.  Run from the repository root:

    python tests/golden/make_tube_batch.py [workers]

(about 2.7 CPU-hours per formulation; one process per worker, one thread
each).  Per tube it stores the flags, the largest |n|, |eps| and |U^mu| over
all cells (the scales of the max-norm relative errors), n, eps and U on the
sampled cells, and, for tubes that stay physical, the spread between the
Table I projection and the closed form of Appendix B (Eq. equi3rd, as
transcribed in tests/appendix_equilibrium.py), run from the same initial
state: how closely float64 arithmetic fixes each tube's fields at all."""
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, REPO)
sys.path.insert(0, os.path.dirname(HERE))

STEPS = 500
NSAMPLE = 32


def sample_cells(N, j):
    """The two ends, the two cells at the initial step, and seeded others."""
    rng = np.random.default_rng(1000 + j)
    fixed = [0, N // 2 - 1, N // 2, N - 1]
    rest = rng.choice(N, size=min(N, NSAMPLE) - len(fixed), replace=False)
    return np.unique(np.concatenate([fixed, rest]))[:NSAMPLE]


def run_one(j, formulations=2):
    """Tube j of the batch on the oracle; formulations=1 skips the
    closed-form run (no spread)."""
    from threadpoolctl import threadpool_limits
    from oracle import rlb
    from oracle.equilibrium import Equilibrium
    from oracle.lattice import model_lattice
    from paper_1301_3423_amd import inputs
    from appendix_equilibrium import equi3rd

    class ClosedForm(Equilibrium):
        def __call__(self, n, T, U):
            out = np.empty((len(n), self.lat.Q))
            Uc = (U[:, 0], U[:, 1], U[:, 2], U[:, 3])
            for i in range(self.lat.Q):
                out[:, i] = equi3rd(n, T, Uc, tuple(self.lat.p[i]), self.lat.w[i])
            return out

    t = inputs.tube_batch(512, 4)[j]
    t0 = time.time()
    with threadpool_limits(limits=1):
        runs = []
        for closed in (False, True)[:formulations]:
            o = rlb.Solver(1, 1, t["N"], lat=model_lattice(3), eta_s=t["eta_s"])
            if closed:
                o.eq = ClosedForm(o.lat, 30)
            o.init_fields(*inputs.shock_tube(t["N"], t["T_left"], t["T_right"]))
            o.step(STEPS)
            runs.append(o.read_fields())
            if runs[0]["flags"]:
                break
    r = runs[0]
    cells = sample_cells(t["N"], j)
    out = {"cells": cells, "flags": int(r["flags"]),
           "scale": np.array([np.max(np.abs(r["n"])), np.max(np.abs(r["eps"])), np.max(np.abs(r["U"]))]),
           "n": r["n"][cells], "eps": r["eps"][cells], "U": r["U"][:, cells], "spread": np.full(3, np.nan)}
    if len(runs) == 2:
        out["spread"] = np.array([np.max(np.abs(runs[1][k] - r[k])) / np.max(np.abs(r[k])) for k in ("n", "eps", "U")])
    return j, out, time.time() - t0


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    from paper_1301_3423_amd import inputs
    spec = inputs.tube_batch(512, 4)
    order = sorted(range(len(spec)), key=lambda j: -spec[j]["N"])   # longest first
    res = {}
    t0 = time.time()
    with get_context("spawn").Pool(workers) as pool:
        for j, out, dt in pool.imap_unordered(run_one, order):
            res[j] = out
            print("tube %3d N=%4d eta/s=%.2f flags %d spread %s (%.0f s, %d/512 after %.0f s)" % (
                j, spec[j]["N"], spec[j]["eta_s"], out["flags"], np.array2string(out["spread"], precision=2),
                dt, len(res), time.time() - t0), flush=True)
    z = {}
    for j in range(len(spec)):
        for k, v in res[j].items():
            z["t%d_%s" % (j, k)] = v
    np.savez_compressed(os.path.join(HERE, "oracle_tube_batch.npz"), **z)


if __name__ == "__main__":
    main()
