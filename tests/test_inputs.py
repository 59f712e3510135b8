"""The seeded input generators agree with each other: the device version of
random_box (run here on the CPU through torch) and the window evaluator
reproduce random_box to rounding."""
import numpy as np

from paper_1301_3423_amd import inputs


def test_device_generator_and_window_match_random_box():
    shape = (24, 20, 16)
    ref = inputs.random_box(*shape, 0.6, 7)
    dev, norms = inputs.random_box_device(*shape, 0.6, 7, device="cpu")
    for a, b in zip(ref, dev):
        assert np.max(np.abs(a - b.numpy())) < 1e-13
    v = np.sqrt(sum(b.numpy() ** 2 for b in dev[2:]))
    assert abs(v.max() - 0.6) < 1e-14
    idx = (np.arange(-3, 9) % 16, np.arange(-4, 5) % 20, np.arange(20, 27) % 24)
    win = inputs.field_window(7, shape, norms, idx)
    for a, b in zip(ref, win):
        assert np.max(np.abs(a[np.ix_(*idx)] - b)) < 1e-13


def test_boosted_box_composes_velocities_relativistically():
    """boosted_box is random_box seen from a frame moving with -boost: per
    cell the Lorentz factors multiply as gamma = gamma_b gamma_v (1 + b.v)
    (the time component of the boosted 4-velocity), a velocity along the
    boost adds as (b + v)/(1 + b v), and every speed stays below 1."""
    shape, b = (12, 10, 8), np.array([0.1, 0.2, 0.2])
    n0, e0, vx0, vy0, vz0 = inputs.random_box(*shape, 0.3, 2)
    n, e, vx, vy, vz = inputs.boosted_box(*shape, 0.3, 2, b)
    assert np.array_equal(n, n0) and np.array_equal(e, e0)
    g = lambda u2: 1.0 / np.sqrt(1.0 - u2)
    v2 = vx * vx + vy * vy + vz * vz
    assert v2.max() < (0.3 + 0.3) ** 2
    lhs = g(v2)
    rhs = g(b @ b) * g(vx0 ** 2 + vy0 ** 2 + vz0 ** 2) * (1.0 + b[0] * vx0 + b[1] * vy0 + b[2] * vz0)
    assert np.max(np.abs(lhs / rhs - 1.0)) < 1e-14
    # collinear: a boost along z on a box moving along z only
    one = np.ones((1, 1, 1))
    import unittest.mock as um
    with um.patch.object(inputs, "random_box", lambda *a, **k: (one, 3 * one, 0 * one, 0 * one, 0.5 * one)):
        _, _, ux, uy, uz = inputs.boosted_box(1, 1, 1, 0.5, 0, (0.0, 0.0, 0.4))
    assert abs(uz[0, 0, 0] - 0.9 / 1.2) < 1e-15 and ux[0, 0, 0] == 0 and uy[0, 0, 0] == 0
