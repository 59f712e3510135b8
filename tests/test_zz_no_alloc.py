"""rlb_conserved_noalloc, the entry point for callers that cannot allocate
device memory, against rlb_conserved through the C ABI: the same kernels in
the same order on a fixed scratch array, so the totals must agree bit for
bit, also on a second call with a smaller box (the array then holds the
first call's larger set of partial sums)."""
import ctypes

import numpy as np
import pytest

from gpu_util import note
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu


def _totals(fn, s):
    out = (ctypes.c_double * 5)()
    rc = fn(s._h, out)
    return rc, np.array(out[:])


@pytest.mark.parametrize("precision,pattern,order", [("fp64", "ab", 3), ("mixed", "aa", 3), ("mixed", "ab", 2)])
def test_noalloc_equals_conserved_on_two_calls(precision, pattern, order):
    L = rlb.lib()
    for shape in [(48, 40, 36), (9, 8, 7)]:
        note("no-alloc conserved: %s %s order %d shape %s" % (precision, pattern, order, shape))
        s = rlb.Solver(*shape, precision=precision, eta_s=0.2, pattern=pattern, order=order)
        s.init_fields(*inputs.random_box(*shape, 0.5, seed=1))
        s.step(3)                       # odd t: the AA buffer is in its swapped state
        rc0, ref = _totals(L.rlb_conserved, s)
        rc1, got = _totals(L.rlb_conserved_noalloc, s)
        assert rc0 == rlb.OK and rc1 == rlb.OK
        assert np.array_equal(got, ref), (got, ref)
        # and the state is left as it was: the next step's totals agree too
        s.step(1)
        assert np.array_equal(_totals(L.rlb_conserved_noalloc, s)[1], _totals(L.rlb_conserved, s)[1])


def test_noalloc_refuses_walls_and_boxes_beyond_its_scratch():
    L = rlb.lib()
    note("no-alloc conserved: refusals")
    s = rlb.Solver(8, 24, 6, precision="mixed", eta_s=0.2)
    solid = np.zeros((6, 24, 8), dtype=bool)
    solid[:, :6] = True
    s.set_walls(solid)
    s.init_fields(*inputs.random_box(8, 24, 6, 0.3, seed=4))
    assert _totals(L.rlb_conserved_noalloc, s)[0] == rlb.EINVAL
    assert b"walls" in L.rlb_last_error()
    # 64 x 64 x 8193 cells: one block of partial sums more than the scratch
    # holds; refused before anything is launched (the box is never initialised)
    big = rlb.Solver(64, 64, 8193, precision="mixed", eta_s=0.2, pattern="aa")
    assert _totals(L.rlb_conserved_noalloc, big)[0] == rlb.EINVAL
    assert b"scratch" in L.rlb_last_error()
    del big
