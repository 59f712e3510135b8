"""The second-order model of Appendix A (66 points, R = 3) on the GPU,
through the C ABI, against the FP64 oracle: boxes on every kernel path,
shock tubes in one persistent launch, the serving path, and checkpoints.

Bar as for the third-order model: max-norm relative error per field
<= 1e-12 (FP64 path) and <= 1e-5 (mixed path)."""
import numpy as np
import pytest

from gpu_util import field_errors, note, run_pair
from oracle import rlb as orlb
from oracle.lattice import model_lattice
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}

# Perturbing the oracle's populations by 1e-15 moves its fields by less
# than 2e-15 after these step counts (well-conditioned cases).
CASES = [
    ((13, 11, 7), 0.5, 12, dict(eta_s=0.2)),     # ragged tail of the last block
    ((5, 4, 3), 0.4, 6, dict(eta_s=0.1)),        # every axis < 7: wrap beyond the edge
    ((9, 1, 17), 0.5, 4, dict(tau=1.3)),         # a degenerate axis of size 1
    ((1, 1, 1), 0.3, 3, dict(tau=0.7)),          # a single cell
    ((40, 36, 33), 0.5, 10, dict(eta_s=0.2)),    # 47520 cells
    ((64, 3, 5), 0.5, 6, dict(eta_s=0.2)),       # rows of 64: one lane per cell (float32)
    ((128, 12, 9), 0.5, 6, dict(tau=0.8)),
]


@pytest.fixture(scope="module")
def lat2():
    return model_lattice(2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,vmax,steps,relax", CASES)
def test_box_parity(lat2, shape, vmax, steps, relax, precision):
    fields = inputs.random_box(*shape, vmax, seed=sum(shape))
    gpu, ref, flags, t, _, _ = run_pair(lat2, shape, fields, steps, precision, order=2, **relax)
    err = field_errors(gpu, ref)
    note("errors %s" % {k: "%.2e" % v for k, v in err.items()})
    assert flags == 0 and t == steps
    assert max(err.values()) <= TOL[precision], err


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shock_tube_config(lat2, precision):
    fields = inputs.shock_tube(200, 1.0, 0.8)
    gpu, ref, flags, t, _, _ = run_pair(lat2, (1, 1, 200), fields, 200, precision, order=2, eta_s=0.1)
    err = field_errors(gpu, ref)
    note("errors %s" % {k: "%.2e" % v for k, v in err.items()})
    assert flags == 0
    assert max(err.values()) <= TOL[precision], err


def test_conservation_and_lattice(lat2):
    fields = inputs.random_box(20, 18, 16, 0.5, seed=2)
    s = rlb.Solver(20, 18, 16, precision="fp64", eta_s=0.2, order=2)
    s.init_fields(*fields)
    c0 = s.conserved()
    o = orlb.Solver(20, 18, 16, lat=lat2, eta_s=0.2, order=2)
    o.init_fields(*fields)
    assert np.max(np.abs(c0 - o.conserved())) < 1e-13 * abs(c0[1])
    s.step(100)
    c1 = s.conserved()
    note("conservation drift %s" % ((c1 - c0) / c0[1]))
    assert np.max(np.abs(c1 - c0)) < 1e-13 * abs(c0[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tube_batch(lat2, precision):
    tubes = [dict(n=1, tau=0.8), dict(n=5, eta_s=0.1), dict(n=200, eta_s=0.1), dict(n=257, tau=0.9),
             dict(n=600, eta_s=0.3)]
    steps = [3, 7, 40, 0, 12]
    b = rlb.Batch(tubes, precision=precision, order=2)
    fields = []
    for j, t in enumerate(tubes):
        n = t["n"]
        f = ([np.array([1.0]), np.array([3.0]), np.zeros(1), np.zeros(1), np.array([0.2])] if n < 2
             else inputs.shock_tube(n, 1.0, 0.7))
        fields.append(f)
        b.init_tube(j, *f)
    b.step(steps)
    for j, t in enumerate(tubes):
        relax = {k: t[k] for k in ("tau", "eta_s") if k in t}
        o = orlb.Solver(1, 1, t["n"], lat=lat2, order=2, **relax)
        o.init_fields(*fields[j])
        o.step(steps[j])
        err = field_errors(b.read_tube(j), o.read_fields())
        flags, tt = b.status(j)
        note("tube %d n=%d steps=%d max err %.2e" % (j, t["n"], steps[j], max(err.values())))
        assert flags == 0 and tt == steps[j]
        assert max(err.values()) <= TOL[precision], (j, err)


def test_server_mixes_models(lat2):
    """Tubes and boxes of both models and both precisions in one server:
    every result matches its own model's oracle."""
    from oracle.lattice import model_lattice as ml
    items = [("tube", (1, 1, 300), "fp64", 30, dict(eta_s=0.1), 2),
             ("tube", (1, 1, 300), "fp64", 30, dict(eta_s=0.1), 3),
             ("tube", (1, 1, 129), "mixed", 21, dict(tau=0.9), 2),
             ("box", (12, 10, 9), "fp64", 14, dict(eta_s=0.2), 2),
             ("box", (64, 4, 3), "mixed", 9, dict(tau=1.0), 2),
             ("box", (9, 8, 7), "mixed", 10, dict(eta_s=0.3), 3)]
    sv = rlb.Server(1 << 30, chunk_steps=8, max_tubes=16)

    def fields(kind, shape):
        return inputs.shock_tube(shape[2], 1.0, 0.7) if kind == "tube" else inputs.random_box(*shape, 0.5, seed=5)
    ids = [sv.submit(k, sh, pr, st, fields(k, sh), order=od, **rx) for (k, sh, pr, st, rx, od) in items]
    done = {c["id"]: c for c in sv.drain(timeout_s=300)}
    sv.close()
    for rid, (kind, shape, prec, steps, rx, od) in zip(ids, items):
        got = done[rid]
        o = orlb.Solver(*shape, lat=ml(od), order=od, **rx)
        o.init_fields(*fields(kind, shape))
        o.step(steps)
        err = field_errors(got["fields"], o.read_fields())
        note("%s %s %s order %d: max err %.2e" % (kind, shape, prec, od, max(err.values())))
        assert got["rc"] == 0 and got["flags"] == 0
        assert max(err.values()) <= TOL[prec], (kind, shape, prec, od, err)
    # the two fp64 tubes differ only in the model: their results differ
    a, b = done[ids[0]]["fields"], done[ids[1]]["fields"]
    assert np.max(np.abs(a["n"] - b["n"])) > 1e-6


def test_checkpoint_carries_the_model(tmp_path):
    fields = inputs.random_box(12, 10, 9, 0.5, seed=4)
    a = rlb.Solver(12, 10, 9, precision="fp64", eta_s=0.1, order=2)
    a.init_fields(*fields)
    a.step(4)
    a.save(tmp_path / "ck2.bin")
    c = rlb.Solver(12, 10, 9, precision="fp64", eta_s=0.1, order=2)
    c.load(tmp_path / "ck2.bin")
    ra, rc = a.read_fields(), c.read_fields()
    for k in ("n", "eps", "U", "P"):
        assert np.array_equal(ra[k], rc[k])
    third = rlb.Solver(12, 10, 9, precision="fp64", eta_s=0.1, order=3)
    with pytest.raises(rlb.RLBError) as e:
        third.load(tmp_path / "ck2.bin")
    assert e.value.code == rlb.EINVAL
