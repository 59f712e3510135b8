"""Solid walls (link-wise bounce-back) on the GPU, through the C ABI,
against the FP64 oracle with the same mask: porous boxes on every kernel
path, a channel, a closed shock tube, conservation and the rest state.

Bar as for periodic boxes: max-norm relative error per field over the fluid
cells <= 1e-12 (FP64 path), <= 1e-5 (mixed path)."""
import numpy as np
import pytest

from gpu_util import field_errors, note
from oracle import rlb as orlb
from oracle.lattice import model_lattice
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def _porous(shape, frac, seed):
    return np.random.default_rng(seed).uniform(size=shape) < frac


def _channel(shape, axis, thick):
    s = np.zeros(shape, dtype=bool)
    idx = [slice(None)] * 3
    idx[axis] = slice(0, thick)
    s[tuple(idx)] = True
    idx[axis] = slice(shape[axis] - thick, shape[axis])
    s[tuple(idx)] = True
    return s


def _fluid_errors(gpu, ref, solid):
    fl = ~solid.ravel()
    g = dict(n=gpu["n"][fl], eps=gpu["eps"][fl], P=gpu["P"][fl], U=gpu["U"][:, fl])
    r = dict(n=ref["n"][fl], eps=ref["eps"][fl], P=ref["P"][fl], U=ref["U"][:, fl])
    return field_errors(g, r)


CASES = [
    # shape (nx, ny, nz), mask, v_max, steps, relaxation
    ((13, 11, 7), ("porous", 0.2, 1), 0.4, 6, dict(eta_s=0.2)),      # pair kernels, ragged tail
    ((64, 48, 3), ("channel", 1, 6), 0.3, 5, dict(eta_s=0.1)),       # row kernel (float32), channel in y
    ((1, 1, 160), ("channel", 0, 6), 0.0, 30, dict(eta_s=0.1)),      # closed shock tube (walls in z)
    ((9, 8, 10), ("porous", 0.35, 2), 0.3, 4, dict(tau=0.9)),
]


def _mask(shape, spec):
    nx, ny, nz = shape
    if spec[0] == "porous":
        return _porous((nz, ny, nx), spec[1], spec[2])
    return _channel((nz, ny, nx), {0: 0, 1: 1, 2: 2}[spec[1]], spec[2])


def _fields(shape, vmax):
    nx, ny, nz = shape
    if vmax == 0.0:
        return inputs.shock_tube(nz, 1.0, 0.6)
    return inputs.random_box(nx, ny, nz, vmax, seed=sum(shape))


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,spec,vmax,steps,relax", CASES)
def test_walls_parity(shape, spec, vmax, steps, relax, precision, order):
    nx, ny, nz = shape
    solid = _mask(shape, spec)
    fields = _fields(shape, vmax)
    note("walls order %d %s %s %s steps %d" % (order, precision, shape, spec, steps))
    s = rlb.Solver(nx, ny, nz, precision=precision, order=order, **relax)
    s.set_walls(solid)
    s.init_fields(*fields)
    s.step(steps)
    gpu = s.read_fields()
    flags, _ = s.status()
    o = orlb.Solver(nx, ny, nz, lat=model_lattice(order), order=order, solid=solid, **relax)
    o.init_fields(*fields)
    o.step(steps)
    ref = o.read_fields()
    err = _fluid_errors(gpu, ref, solid)
    note("errors %s" % {k: "%.2e" % v for k, v in err.items()})
    assert flags == 0
    assert np.all(gpu["n"][solid.ravel()] == 0)
    assert max(err.values()) <= TOL[precision], err


@pytest.mark.parametrize("order", [3, 2])
def test_walls_conserve_N0_and_T00_on_device(order):
    nx, ny, nz = 20, 18, 16
    solid = _porous((nz, ny, nx), 0.15, 3)
    fields = inputs.random_box(nx, ny, nz, 0.4, seed=9)
    s = rlb.Solver(nx, ny, nz, precision="fp64", eta_s=0.2, order=order)
    s.set_walls(solid)
    s.init_fields(*fields)
    c0 = s.conserved()
    o = orlb.Solver(nx, ny, nz, lat=model_lattice(order), order=order, solid=solid, eta_s=0.2)
    o.init_fields(*fields)
    assert np.max(np.abs(c0 - o.conserved())) < 1e-13 * abs(c0[1])
    s.step(60)
    c1 = s.conserved()
    note("walls order %d: N0 drift %.2e, T00 drift %.2e, T0x change %.2e" % (
        order, (c1[0] - c0[0]) / c0[0], (c1[1] - c0[1]) / c0[1], (c1[2] - c0[2]) / c0[1]))
    assert abs(c1[0] - c0[0]) < 1e-13 * abs(c0[0])
    assert abs(c1[1] - c0[1]) < 1e-13 * abs(c0[1])
    assert np.max(np.abs(c1[2:] - c0[2:])) > 1e-4 * abs(c0[1])


def test_rest_state_stays_and_walls_can_be_removed():
    nx, ny, nz = 64, 8, 6
    solid = _porous((nz, ny, nx), 0.3, 4)
    C = nx * ny * nz
    rest = [np.full(C, 1.1), np.full(C, 3 * 1.1 * 0.95), np.zeros(C), np.zeros(C), np.zeros(C)]
    for prec in ("fp64", "mixed"):
        s = rlb.Solver(nx, ny, nz, precision=prec, eta_s=0.3)
        s.set_walls(solid)
        s.init_fields(*rest)
        s.step(10)
        out = s.read_fields()
        fl = ~solid.ravel()
        assert np.max(np.abs(out["n"][fl] - 1.1)) < (1e-13 if prec == "fp64" else 1e-6)
        assert np.max(np.abs(out["U"][1:, fl])) < (1e-13 if prec == "fp64" else 1e-6)
    # removing the walls gives back the periodic solver
    fields = inputs.random_box(nx, ny, nz, 0.3, seed=5)
    a = rlb.Solver(nx, ny, nz, precision="fp64", eta_s=0.2)
    b = rlb.Solver(nx, ny, nz, precision="fp64", eta_s=0.2)
    b.set_walls(solid)
    b.set_walls(None)
    for x in (a, b):
        x.init_fields(*fields)
        x.step(4)
    ra, rb = a.read_fields(), b.read_fields()
    for k in ("n", "eps", "U", "P"):
        assert np.array_equal(ra[k], rb[k])


def test_walls_checkpoint_requires_the_same_walls(tmp_path):
    nx, ny, nz = 12, 10, 9
    solid = _porous((nz, ny, nx), 0.2, 6)
    fields = inputs.random_box(nx, ny, nz, 0.4, seed=4)
    a = rlb.Solver(nx, ny, nz, precision="fp64", eta_s=0.1)
    a.set_walls(solid)
    a.init_fields(*fields)
    a.step(3)
    a.save(tmp_path / "w.bin")
    a.step(3)
    b = rlb.Solver(nx, ny, nz, precision="fp64", eta_s=0.1)
    with pytest.raises(rlb.RLBError):
        b.load(tmp_path / "w.bin")                 # no walls set
    b.set_walls(solid)
    b.load(tmp_path / "w.bin")
    b.step(3)
    ra, rb = a.read_fields(), b.read_fields()
    for k in ("n", "eps", "U", "P"):
        assert np.array_equal(ra[k], rb[k])


def test_walls_reject_bad_masks():
    s = rlb.Solver(4, 4, 4, precision="fp64", tau=1.0)
    with pytest.raises(rlb.RLBError) as e:
        s.set_walls(np.ones((4, 4, 4)))
    assert e.value.code == rlb.EINVAL
    with pytest.raises(ValueError):
        s.set_walls(np.zeros(10))
