"""The in-place AA streaming pattern against the two-buffer (AB) pull.

Both patterns run the same per-cell arithmetic on the same values, so after
every step the macroscopic fields of an AA solver equal those of an AB
solver bit for bit, after even steps (natural AA layout) and after odd steps
(swapped layout).  A read-after-write race in the in-place update, or a
wrong slot in either half-step, would break that equality.  The oracle is
checked directly as well, to the usual parity bar."""
import os
import tempfile

import numpy as np
import pytest

from gpu_util import field_errors, note
from oracle import rlb as orlb
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}

SHAPES = [
    (13, 11, 7),     # ragged tail of the two-lane kernel
    (5, 4, 3),       # every axis below the largest displacement: wrap beyond the edge
    (9, 1, 17),      # a degenerate axis
    (64, 3, 5),      # whole-wavefront rows (float32 one-lane kernel), small y and z;
                     # the odd step rotates its stores through LDS (four rows a block)
    (128, 12, 9),
    (256, 2, 3),     # one row a block
    (64, 1, 1),      # one row: the block's other wavefronts only join its barriers
    (192, 2, 3),     # rows across blocks: the odd step stores at x + theta directly
    (96, 3, 4),      # float32 on the two-lane kernel with rows of whole wavefronts
    (32, 5, 3),      # four rows a two-lane block
    (32, 1, 1),      # one wavefront of cells in a block of four
]


def _same(a, b):
    for k in ("n", "eps", "P"):
        if not np.array_equal(a[k], b[k]):
            return False
    return np.array_equal(a["U"], b["U"])


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES)
def test_aa_equals_ab_every_step(shape, precision, order):
    note("case AA vs AB order=%d shape=%s precision=%s" % (order, shape, precision))
    fields = inputs.random_box(*shape, 0.5, seed=sum(shape) + order)
    ab = rlb.Solver(*shape, precision=precision, eta_s=0.2, order=order, pattern="ab")
    aa = rlb.Solver(*shape, precision=precision, eta_s=0.2, order=order, pattern="aa")
    ab.init_fields(*fields)
    aa.init_fields(*fields)
    assert _same(ab.read_fields(), aa.read_fields())
    for t in range(1, 6):
        ab.step(1)
        aa.step(1)
        assert _same(ab.read_fields(), aa.read_fields()), "step %d" % t
    assert aa.status() == (0, 5)
    c_ab, c_aa = ab.conserved(), aa.conserved()
    assert np.max(np.abs(c_ab - c_aa)) < 1e-13 * abs(c_ab[1])


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("steps", [7, 8])
def test_aa_matches_oracle(lat, lat2, order, precision, steps):
    shape = (40, 36, 33)   # 47520 cells: many blocks, ragged tail
    note("case AA vs oracle order=%d precision=%s steps=%d" % (order, precision, steps))
    fields = inputs.random_box(*shape, 0.5, seed=41)
    s = rlb.Solver(*shape, precision=precision, eta_s=0.2, order=order, pattern="aa")
    s.init_fields(*fields)
    s.step(steps)
    gpu = s.read_fields()
    o = orlb.Solver(*shape, lat=lat if order == 3 else lat2, order=order, eta_s=0.2)
    o.init_fields(*fields)
    o.step(steps)
    err = field_errors(gpu, o.read_fields())
    note("errors %s" % {k: "%.2e" % v for k, v in err.items()})
    assert s.status() == (0, steps)
    assert max(err.values()) <= TOL[precision], err


def test_aa_conserves_on_device():
    fields = inputs.random_box(20, 18, 16, 0.5, seed=2)
    s = rlb.Solver(20, 18, 16, precision="fp64", eta_s=0.2, pattern="aa")
    s.init_fields(*fields)
    c0 = s.conserved()
    for steps in (1, 1, 97):      # odd t, even t, odd t
        s.step(steps)
        c1 = s.conserved()
        assert np.max(np.abs(c1 - c0)) < 1e-13 * abs(c0[1]), (s.status(), c1 - c0)


@pytest.mark.parametrize("split", [3, 4])
def test_aa_checkpoint_resumes_bitwise(split):
    shape = (24, 16, 10)
    fields = inputs.random_box(*shape, 0.5, seed=5)
    ref = rlb.Solver(*shape, precision="fp64", tau=0.9, pattern="aa")
    ref.init_fields(*fields)
    ref.step(7)
    a = rlb.Solver(*shape, precision="fp64", tau=0.9, pattern="aa")
    a.init_fields(*fields)
    a.step(split)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "aa.ckpt")
        a.save(path)
        b = rlb.Solver(*shape, precision="fp64", tau=0.9, pattern="aa")
        b.load(path)
        assert b.status() == (0, split)
        b.step(7 - split)
        assert _same(b.read_fields(), ref.read_fields())
        # a checkpoint of the other pattern is refused
        c = rlb.Solver(*shape, precision="fp64", tau=0.9, pattern="ab")
        with pytest.raises(rlb.RLBError):
            c.load(path)


def test_aa_refuses_walls():
    s = rlb.Solver(16, 16, 8, precision="fp64", tau=1.0, pattern="aa")
    solid = np.zeros((8, 16, 16), bool)
    solid[:, :6] = True
    with pytest.raises(rlb.RLBError):
        s.set_walls(solid)


def test_aa_halves_the_footprint():
    """At 256^3 the AA state is one population buffer plus staging."""
    for prec, b in (("fp64", 8), ("mixed", 4)):
        ab = rlb.state_bytes(256, 256, 256, prec, 3, "ab")
        aa = rlb.state_bytes(256, 256, 256, prec, 3, "aa")
        cells = 256 ** 3
        assert aa - 128 * cells * b - 56 * cells < 1 << 20
        assert ab - 2 * 128 * cells * b < 1 << 20


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_aa_equals_ab_at_256cube(precision):
    """The benchmark's box and launch configuration: after an odd and an even
    number of steps the AA fields equal the AB fields bit for bit (the AB
    path is pinned to the oracle at this size on sampled cells)."""
    import torch
    shape = (256, 256, 256)
    note("case AA vs AB 256^3 precision=%s" % precision)
    fields = inputs.random_box(*shape, 0.6, seed=3)
    ab = rlb.Solver(*shape, precision=precision, eta_s=0.5, pattern="ab")
    ab.init_fields(*fields)
    ref = []
    for steps in (3, 1):
        ab.step(steps)
        ref.append(ab.read_fields())
    del ab
    torch.cuda.empty_cache()
    aa = rlb.Solver(*shape, precision=precision, eta_s=0.5, pattern="aa")
    aa.init_fields(*fields)
    for steps, r in zip((3, 1), ref):
        aa.step(steps)
        assert _same(aa.read_fields(), r), "t=%d" % aa.status()[1]
    assert aa.status() == (0, 4)


def largest_aa_edge(precision, reserve_per_cell=40, frac=0.92):
    """Largest multiple of 64 whose AA box (plus its device input fields)
    fits in the free memory of the current device, within the library's
    size cap."""
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    per_cell = rlb.state_bytes(64, 64, 64, precision, 3, "aa") / 64 ** 3 + reserve_per_cell
    edge = int((frac * free / per_cell) ** (1.0 / 3.0)) // 64 * 64
    while edge > 64 and rlb.state_bytes(edge, edge, edge, precision, 3, "aa") == 0:
        edge -= 64
    return edge


def test_aa_largest_box_matches_oracle_on_sampled_cells(lat):
    """The largest float64 box one GPU holds with the AA pattern (576^3 on
    288 GB, where the two-buffer layout would need 391 GB): after two steps
    sampled cells, corners included, agree with the oracle run on the
    periodic 25^3 window of the initial fields around each of them."""
    import torch
    K, W = 2, 25
    edge = largest_aa_edge("fp64")
    shape = (edge, edge, edge)
    note("case AA largest box %d^3 fp64 (AA %.1f GB, AB would need %.1f GB)" % (
        edge, rlb.state_bytes(*shape, "fp64", 3, "aa") / 1e9, rlb.state_bytes(*shape, "fp64", 3, "ab") / 1e9))
    fields, norms = inputs.random_box_device(*shape, 0.6, 3)
    torch.cuda.empty_cache()
    s = rlb.Solver(*shape, precision="fp64", eta_s=0.5, pattern="aa")
    s.init_fields(*fields)
    s.release_inputs()
    del fields
    torch.cuda.empty_cache()
    s.step(K)
    out = s.read_fields()
    assert s.status() == (0, K)
    del s
    rng = np.random.default_rng(edge)
    pts = [(0, 0, 0), (edge - 1, edge - 1, edge - 1), (edge // 2, 0, edge - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, edge, 3)) for _ in range(2)]
    mid = 6 * K * (W * W + W + 1)
    for c in pts:
        idx = [np.arange(ci - 6 * K, ci + 6 * K + 1) % edge for ci in c]
        win = inputs.field_window(3, shape, norms, idx)
        o = orlb.Solver(W, W, W, lat=lat, eta_s=0.5)
        o.init_fields(*win)
        o.step(K)
        ref = o.read_fields()
        flat = (c[0] * edge + c[1]) * edge + c[2]
        U0 = ref["U"][0, mid]
        errs = [abs(out[k][flat] - ref[k][mid]) / ref[k][mid] for k in ("n", "eps", "P")]
        errs += [abs(out["U"][j, flat] - ref["U"][j, mid]) / U0 for j in range(4)]
        assert max(errs) <= 1e-12, (c, errs)


def test_aa_reinit_at_odd_t_and_device_read():
    """init_fields at an odd t starts again from the natural layout (t = 0),
    and reading into device tensors gives the host read's values."""
    shape = (24, 16, 10)
    f1 = inputs.random_box(*shape, 0.5, seed=6)
    f2 = inputs.random_box(*shape, 0.4, seed=7)
    a = rlb.Solver(*shape, precision="fp64", eta_s=0.2, pattern="aa")
    a.init_fields(*f1)
    a.step(3)
    a.init_fields(*f2)
    assert a.status() == (0, 0)
    a.step(5)
    b = rlb.Solver(*shape, precision="fp64", eta_s=0.2, pattern="aa")
    b.init_fields(*f2)
    b.step(5)
    host = a.read_fields()
    assert _same(host, b.read_fields())
    dev = a.read_fields(on_device=True)
    for k in ("n", "eps", "P", "U"):
        assert np.array_equal(dev[k].cpu().numpy(), host[k])
