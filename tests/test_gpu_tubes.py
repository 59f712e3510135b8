"""Batched shock tubes (one persistent launch) against the FP64 oracle and
against the single-box path, through the C ABI."""
import numpy as np
import pytest

from gpu_util import field_errors, note
from oracle import rlb as orlb
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}

# ragged lengths: a single cell, lengths below the displacement range,
# partial passes of 128 cells, several passes
TUBES = [
    dict(n=1, tau=0.8),
    dict(n=5, eta_s=0.1),
    dict(n=13, tau=1.1),
    dict(n=200, eta_s=0.1),
    dict(n=257, eta_s=0.5),
    dict(n=700, tau=0.9),
]
STEPS = [3, 7, 0, 40, 25, 12]          # tube 2 stays untouched


def _fields(n, r):
    if n < 2:
        return [np.array([1.0]), np.array([3.0]), np.zeros(1), np.zeros(1), np.array([0.2])]
    return inputs.shock_tube(n, 1.0, 1.0 / r)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_oracle(lat, precision):
    b = rlb.Batch(TUBES, precision=precision)
    ratios = [1.3, 1.5, 1.2, 2.0, 1.25, 1.7]
    fields = [_fields(t["n"], r) for t, r in zip(TUBES, ratios)]
    for j, f in enumerate(fields):
        b.init_tube(j, *f)
    note("batch %s: %d tubes, steps %s" % (precision, len(TUBES), STEPS))
    b.step(STEPS)
    for j, t in enumerate(TUBES):
        relax = {k: t[k] for k in ("tau", "eta_s") if k in t}
        o = orlb.Solver(1, 1, t["n"], lat=lat, **relax)
        o.init_fields(*fields[j])
        o.step(STEPS[j])
        ref = o.read_fields()
        got = b.read_tube(j)
        err = field_errors(got, ref)
        flags, tt = b.status(j)
        note("tube %d n=%d steps=%d max err %.2e flags %d" % (j, t["n"], STEPS[j], max(err.values()), flags))
        assert flags == 0 and tt == STEPS[j]
        assert max(err.values()) <= TOL[precision], (j, err)


def test_batch_two_launches_equal_one(lat):
    """Advancing 10 + 15 steps equals 25 steps (state carried between launches)."""
    tubes = [dict(n=300, eta_s=0.2), dict(n=77, tau=0.95)]
    f = [inputs.shock_tube(300, 1.0, 0.6), inputs.shock_tube(77, 1.0, 0.8)]
    a = rlb.Batch(tubes, precision="fp64")
    c = rlb.Batch(tubes, precision="fp64")
    for j in range(2):
        a.init_tube(j, *f[j])
        c.init_tube(j, *f[j])
    a.step(25)
    c.step([10, 10])
    c.step([15, 15])
    for j in range(2):
        ra, rc = a.read_tube(j), c.read_tube(j)
        for k in ("n", "eps", "U", "P"):
            assert np.array_equal(ra[k], rc[k])


def test_batch_equals_box_path(lat):
    """The same tube as a 1 x 1 x n box through rlb_step."""
    n = 333
    f = inputs.shock_tube(n, 1.0, 0.55)
    b = rlb.Batch([dict(n=n, eta_s=0.1)], precision="fp64")
    b.init_tube(0, *f)
    b.step(30)
    s = rlb.Solver(1, 1, n, precision="fp64", eta_s=0.1)
    s.init_fields(*f)
    s.step(30)
    err = field_errors(b.read_tube(0), s.read_fields())
    assert max(err.values()) < 1e-13, err


def test_failure_stays_in_its_tube():
    import torch
    tubes = [dict(n=64, tau=1.0), dict(n=64, tau=1.0)]
    b = rlb.Batch(tubes, precision="mixed")
    good = inputs.shock_tube(64, 1.0, 0.7)
    b.init_tube(0, *good)
    # tube 1: a negative density, injected through the device path
    bad = [np.asarray(a, dtype=np.float64).copy() for a in good]
    bad[0][10] = -1.0
    with pytest.raises(rlb.RLBError) as e:
        b.init_tube(1, *bad)
    assert e.value.code == rlb.ENONPHYS
    d = [torch.tensor(a, device="cuda") for a in bad]
    rlb.check(rlb.lib().rlb_batch_init(b._h, 1, *[rlb.ctypes.c_void_p(t.data_ptr()) for t in d], 1))
    torch.cuda.synchronize()
    b.step([5, 5])
    f0, _ = b.status(0)
    f1, _ = b.status(1)
    assert f0 == 0
    assert f1 & rlb.FLAG_NONPHYSICAL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_many_chunks_and_steps_match_oracle(lat, precision):
    """Tubes of many wavefront chunks (4000 cells: 63 chunks of 64 cells in
    float32, 125 of 32 in float64) and a ragged one, advanced 60 steps in one
    launch: the wavefronts work through (step, chunk) items in order, each
    waiting only for its neighbouring chunks, across step boundaries."""
    tubes = [dict(n=4000, eta_s=0.2), dict(n=1999, tau=0.85), dict(n=65, eta_s=0.05)]
    fields = [inputs.shock_tube(4000, 1.0, 0.55), inputs.shock_tube(1999, 1.0, 0.7),
              inputs.shock_tube(65, 1.0, 0.9)]
    steps = [60, 45, 60]
    b = rlb.Batch(tubes, precision=precision)
    for j, f in enumerate(fields):
        b.init_tube(j, *f)
    note("batch %s: tubes %s, steps %s" % (precision, [t["n"] for t in tubes], steps))
    b.step(steps)
    for j, t in enumerate(tubes):
        relax = {k: t[k] for k in ("tau", "eta_s") if k in t}
        o = orlb.Solver(1, 1, t["n"], lat=lat, **relax)
        o.init_fields(*fields[j])
        o.step(steps[j])
        err = field_errors(b.read_tube(j), o.read_fields())
        flags, tt = b.status(j)
        note("tube n=%d: max err %.2e flags %d" % (t["n"], max(err.values()), flags))
        assert flags == 0 and tt == steps[j]
        assert max(err.values()) <= TOL[precision], (t["n"], err)


def test_tube_beyond_the_dataflow_flags_takes_the_barrier_kernel():
    """A float64 tube of more chunks than a workgroup's flags hold (786,433
    cells) runs in the barrier form of the kernel, in the same call as a
    short tube that runs in the dataflow form; both equal the box path."""
    n_big, n_small = 786433, 300
    f_big = inputs.shock_tube(n_big, 1.0, 0.6)
    f_small = inputs.shock_tube(n_small, 1.0, 0.8)
    b = rlb.Batch([dict(n=n_big, eta_s=0.1), dict(n=n_small, eta_s=0.1)], precision="fp64")
    b.init_tube(0, *f_big)
    b.init_tube(1, *f_small)
    note("batch fp64: a %d-cell tube (barrier kernel) and a %d-cell tube, 3 steps" % (n_big, n_small))
    b.step(3)
    for j, (n, f) in enumerate(((n_big, f_big), (n_small, f_small))):
        s = rlb.Solver(1, 1, n, precision="fp64", eta_s=0.1)
        s.init_fields(*f)
        s.step(3)
        err = field_errors(b.read_tube(j), s.read_fields())
        assert b.status(j) == (0, 3)
        assert max(err.values()) < 1e-13, (n, err)


def test_stalled_wait_is_flagged_and_the_launch_ends(monkeypatch):
    """The kernel's waits for neighbouring chunks are bounded.  With the bound
    lowered to one poll (RLB_TUBE_SPIN_LIMIT=1, read by rlb_batch_step), the
    waits that do not succeed at once give up: the launch still ends and the
    tube reports RLB_FLAG_STALL (its fields are then not to be trusted).
    Without the variable the same run is clean."""
    f = inputs.shock_tube(100, 1.0, 0.8)      # two float32 chunks: wavefronts wait across steps
    monkeypatch.setenv("RLB_TUBE_SPIN_LIMIT", "1")
    b = rlb.Batch([dict(n=100, tau=0.9)], precision="mixed")
    b.init_tube(0, *f)
    b.step(50)
    flags, t = b.status(0)
    assert t == 50 and flags & rlb.FLAG_STALL
    monkeypatch.delenv("RLB_TUBE_SPIN_LIMIT")
    c = rlb.Batch([dict(n=100, tau=0.9)], precision="mixed")
    c.init_tube(0, *f)
    c.step(50)
    assert c.status(0) == (0, 50)
