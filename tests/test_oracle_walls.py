"""Pins of the oracle's solid walls: link-wise bounce-back, which the
paper enables by requiring inversion-paired weights (Sec. II C).  A
population whose source cell is solid is replaced by the post-collision
population of the inverse direction at the receiving cell."""
import numpy as np
import pytest

import bruteforce
from oracle import rlb
from oracle.lattice import model_lattice
from paper_1301_3423_amd import inputs


def _porous(shape, frac, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(size=shape) < frac


def _slab_walls(shape, axis, thick):
    s = np.zeros(shape, dtype=bool)
    idx = [slice(None)] * 3
    idx[axis] = slice(0, thick)
    s[tuple(idx)] = True
    idx[axis] = slice(shape[axis] - thick, shape[axis])
    s[tuple(idx)] = True
    return s


@pytest.mark.parametrize("order", [3, 2])
def test_rest_state_with_walls_is_stationary(order):
    """At rest f_i^eq = f_inv(i)^eq (equal weights on pairs), so reflecting
    a population changes nothing: any geometry keeps a fluid at rest."""
    nx, ny, nz = 6, 5, 7
    solid = _porous((nz, ny, nx), 0.3, 1)
    s = rlb.Solver(nx, ny, nz, eta_s=0.2, order=order, solid=solid)
    C = s.C
    s.init_fields(np.full(C, 1.3), np.full(C, 3 * 1.3 * 0.9), np.zeros(C), np.zeros(C), np.zeros(C))
    f0 = s.f.copy()
    s.step(5)
    assert np.max(np.abs(s.f - f0)) < 1e-14 * np.max(np.abs(f0))
    assert s.flags == 0


@pytest.mark.parametrize("order", [3, 2])
def test_walls_keep_N0_and_T00_but_take_momentum(order):
    """Streaming with bounce-back permutes post-collision populations among
    fluid slots, each on its own shell: the totals of N^0 and T^{00} stay
    to rounding; the walls exchange momentum, so T^{0i} changes."""
    nx, ny, nz = 8, 7, 9
    solid = _porous((nz, ny, nx), 0.2, 2)
    s = rlb.Solver(nx, ny, nz, eta_s=0.2, order=order, solid=solid)
    s.init_fields(*inputs.random_box(nx, ny, nz, 0.4, 3))
    c0 = s.conserved()
    s.step(30)
    c1 = s.conserved()
    assert s.flags == 0
    assert abs(c1[0] - c0[0]) < 1e-13 * abs(c0[0])
    assert abs(c1[1] - c0[1]) < 1e-13 * abs(c0[1])
    assert np.max(np.abs(c1[2:] - c0[2:])) > 1e-4 * abs(c0[1])


def test_reflecting_the_same_direction_would_not_conserve():
    """A planted mistake (bounce-back into i instead of inv(i)) breaks the
    N^0 budget, so the test above can tell the two apart."""
    lat = model_lattice(3)
    nx, ny, nz = 6, 6, 6
    solid = _porous((nz, ny, nx), 0.2, 4)
    s = rlb.Solver(nx, ny, nz, eta_s=0.2, solid=solid)
    s.init_fields(*inputs.random_box(nx, ny, nz, 0.4, 5))
    c0 = s.conserved()
    saved = lat.inv
    try:
        s.lat.inv = np.arange(s.lat.Q)
        s.step(3)
    finally:
        s.lat.inv = saved
    assert abs(s.conserved()[0] - c0[0]) > 1e-6 * abs(c0[0])


def test_far_from_walls_the_flow_is_the_periodic_one():
    """Populations move at most 6 cells per step, so after t steps cells
    farther than 6 t from a wall see the same history as without walls."""
    nz, t = 400, 20
    fields = inputs.shock_tube(nz, 1.0, 0.6)
    solid = np.zeros((nz, 1, 1), dtype=bool)
    solid[:6] = True
    solid[-6:] = True
    a = rlb.Solver(1, 1, nz, eta_s=0.1, solid=solid)
    b = rlb.Solver(1, 1, nz, eta_s=0.1)
    a.init_fields(*fields)
    b.init_fields(*fields)
    a.step(t)
    b.step(t)
    lo, hi = 6 + 6 * t, nz - 6 - 6 * t
    assert np.max(np.abs(a.f[:, lo:hi] - b.f[:, lo:hi])) < 1e-14 * np.max(np.abs(b.f))
    # and near the walls it is not
    assert np.max(np.abs(a.f[:, 6:12] - b.f[:, 6:12])) > 1e-6


def test_channel_flow_is_slowed_by_the_walls():
    """A uniform flow along a channel between two walls at rest: a no-slip
    boundary layer grows from the walls (about one displacement per step)
    while the momentum falls every step; the centre of the channel is not
    reached before the layer gets there."""
    nx, ny, nz = 4, 48, 3
    solid = _slab_walls((nz, ny, nx), 1, 6)
    s = rlb.Solver(nx, ny, nz, eta_s=0.1, solid=solid)
    C = s.C
    s.init_fields(np.ones(C), np.full(C, 3.0), np.full(C, 0.2), np.zeros(C), np.zeros(C))
    px = [s.conserved()[2]]
    for k in range(4):
        s.step(1)
        px.append(s.conserved()[2])
        r = s.read_fields()
        vx = (r["U"][1] / np.where(r["U"][0] > 0, r["U"][0], 1)).reshape(nz, ny, nx)[1, :, 2]
        assert vx[6] < 0.15 * 0.2 and vx[ny - 7] < 0.15 * 0.2        # next to the walls
        if 6 * (k + 1) < ny // 2 - 6:                                  # the centre: not reached yet
            assert abs(vx[ny // 2] - 0.2) < 1e-12
    assert all(b < a for a, b in zip(px, px[1:]))
    assert np.all(r["n"].reshape(nz, ny, nx)[:, :6] == 0)              # solid cells report nothing


@pytest.mark.parametrize("order", [3, 2])
def test_bruteforce_agrees_with_oracle_with_walls(order):
    nx, ny, nz = 4, 3, 5
    solid = _porous((nz, ny, nx), 0.25, 6)
    s = rlb.Solver(nx, ny, nz, eta_s=0.1, order=order, solid=solid)
    s.init_fields(*inputs.random_box(nx, ny, nz, 0.4, 7))
    f = s.f.copy()
    for _ in range(3):
        f = bruteforce.step(s.lat, f, (nz, ny, nx), eta_s=0.1, order=order, solid=solid)
    s.step(3)
    assert np.max(np.abs(f - s.f)) < 1e-12 * np.max(np.abs(f))
