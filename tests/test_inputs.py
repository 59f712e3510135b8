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
