"""The C-ABI library loads and exports what include/rlb.h declares; host-only
calls (no device work) behave as documented.  Runs without a GPU."""
import os
import re

import numpy as np
import pytest

from paper_1301_3423_amd import rlb

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(REPO, "include", "rlb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rlb_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(rlb.EXPORTS) == _declared()


def test_header_constants_match_the_binding():
    """Every #define RLB_<NAME> value of include/rlb.h equals the binding's <NAME>."""
    src = open(os.path.join(REPO, "include", "rlb.h")).read()
    found = dict(re.findall(r"#define RLB_([A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", src))
    found.pop("H", None)
    assert len(found) >= 20
    for name, value in found.items():
        assert getattr(rlb, name) == int(value), name


def test_library_exports_every_declared_symbol():
    L = rlb.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_lattice_info_matches_table(lat):
    info = rlb.lattice_info()
    assert info["q"] == lat.Q == 128 and info["r2"] == 41 and info["nshell"] == 4
    assert np.array_equal(info["theta"], lat.theta)
    assert np.array_equal(info["p0"], lat.p0)
    assert np.array_equal(info["w"], lat.w)
    assert np.array_equal(info["inv"], lat.inv)
    assert np.array_equal(info["shell"], lat.shell)
    import hashlib
    path = os.path.join(REPO, "paper_1301_3423_amd", "lattice", "d3q128.txt")
    assert info["sha256"] == hashlib.sha256(open(path, "rb").read()).hexdigest()


def test_second_order_lattice_info_matches_table():
    import hashlib
    from oracle.lattice import model_lattice
    lat2 = model_lattice(2)
    info = rlb.lattice_info(rlb.ORDER2)
    assert info["q"] == lat2.Q == 66 and info["r2"] == 9 and info["nshell"] == 3
    for k in ("theta", "p0", "w", "inv", "shell"):
        assert np.array_equal(info[k], getattr(lat2, k)), k
    path = os.path.join(REPO, "paper_1301_3423_amd", "lattice", "d3q66.txt")
    assert info["sha256"] == hashlib.sha256(open(path, "rb").read()).hexdigest()
    # order 0 is the default, the third-order model
    assert rlb.lattice_info(0)["q"] == 128
    import ctypes
    lat = rlb.Lattice()
    assert rlb.lib().rlb_lattice_info(4, ctypes.byref(lat)) == rlb.EINVAL


@pytest.mark.parametrize("order,q", [(3, 128), (2, 66)])
def test_state_bytes(order, q):
    b64 = rlb.state_bytes(16, 16, 16, "fp64", order)
    b32 = rlb.state_bytes(16, 16, 16, "mixed", order)
    cells = 16 ** 3
    assert b64 >= 2 * q * cells * 8 and b32 >= 2 * q * cells * 4
    assert b64 - 2 * q * cells * 8 < 2 * q * 64 * 8 + 8192
    assert rlb.state_bytes(0, 4, 4) == 0
    assert rlb.lib().rlb_state_bytes(4, 4, 4, 7, order, 0) == 0
    assert rlb.lib().rlb_state_bytes(4, 4, 4, 0, 1, 0) == 0       # no first-order model
    assert rlb.lib().rlb_state_bytes(4, 4, 4, 0, order, 2) == 0   # no third pattern
    # boxes up to 2^28 - 2^16 cells: 640^3 is accepted, 2^28 cells are not
    assert rlb.state_bytes(640, 640, 640, "fp64", order, "aa") > 0
    assert rlb.state_bytes(1024, 512, 512, "mixed", order) == 0


@pytest.mark.parametrize("order,q", [(3, 128), (2, 66)])
def test_state_bytes_aa_holds_one_buffer(order, q):
    """AA: one population buffer plus 7 doubles of staging per cell."""
    cells = 24 * 20 * 16
    for prec, b in (("fp64", 8), ("mixed", 4)):
        ab = rlb.state_bytes(24, 20, 16, prec, order, "ab")
        aa = rlb.state_bytes(24, 20, 16, prec, order, "aa")
        assert aa >= q * cells * b + 7 * 8 * cells
        assert aa - (q * cells * b + 7 * 8 * cells) < q * 64 * b + 8192
        assert abs((ab - aa) - (q * cells * b - 7 * 8 * cells)) < q * 64 * b + 256


def test_batch_and_request_bytes_follow_the_model():
    tubes = [dict(n=100, tau=1.0), dict(n=37, eta_s=0.1)]
    b3 = rlb.batch_bytes(tubes, "fp64", 3)
    b2 = rlb.batch_bytes(tubes, "fp64", 2)
    assert 0 < b2 < b3
    assert rlb.batch_bytes(tubes, "fp64", 5) == 0
    assert 0 < rlb.request_bytes("tube", (1, 1, 64), "mixed", 2) < rlb.request_bytes("tube", (1, 1, 64), "mixed", 3)
    assert rlb.request_bytes("box", (8, 8, 8), "fp64", 9) == 0


def test_strerror_names_codes():
    L = rlb.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.rlb_strerror(code).decode() != "unknown error"
    assert L.rlb_strerror(-99).decode() == "unknown error"


def test_create_rejects_bad_arguments():
    import ctypes
    L = rlb.lib()
    h = ctypes.c_void_p()
    cfg = rlb.Config(8, 8, 8, rlb.FP64, rlb.TAU_FIXED, 0.4, 0.0)      # tau <= 1/2
    fake = ctypes.c_void_p(1 << 20)                                    # never dereferenced
    assert L.rlb_create(ctypes.byref(h), ctypes.byref(cfg), fake, 1 << 40, None) == rlb.EINVAL
    cfg = rlb.Config(8, 8, 8, rlb.FP64, rlb.TAU_FIXED, 1.0, 0.0)
    assert L.rlb_create(ctypes.byref(h), ctypes.byref(cfg), fake, 1024, None) == rlb.ENOMEM
    assert b"needs" in L.rlb_last_error()
    cfg = rlb.Config(8, 8, 8, 5, rlb.TAU_FIXED, 1.0, 0.0)
    assert L.rlb_create(ctypes.byref(h), ctypes.byref(cfg), fake, 1 << 40, None) == rlb.EINVAL
    cfg = rlb.Config(8, 8, 8, rlb.FP64, rlb.TAU_ETA_S, 0.0, -1.0)
    assert L.rlb_create(ctypes.byref(h), ctypes.byref(cfg), fake, 1 << 40, None) == rlb.EINVAL
    cfg = rlb.Config(8, 8, 8, rlb.FP64, rlb.TAU_FIXED, 1.0, 0.0, 1)   # order 1 does not exist
    assert L.rlb_create(ctypes.byref(h), ctypes.byref(cfg), fake, 1 << 40, None) == rlb.EINVAL
    assert b"order" in L.rlb_last_error()
    cfg = rlb.Config(8, 8, 8, rlb.FP64, rlb.TAU_FIXED, 1.0, 0.0, 3, 2)   # pattern 2 does not exist
    assert L.rlb_create(ctypes.byref(h), ctypes.byref(cfg), fake, 1 << 40, None) == rlb.EINVAL
    assert b"pattern" in L.rlb_last_error()
    assert L.rlb_step(None, 1) == rlb.EINVAL


@pytest.mark.parametrize("order", [3, 2])
def test_walls_bytes_counts_bounce_back_links(order):
    """rlb_walls_bytes: the mask (rounded to 256 B) plus 12 B per
    (solid cell, population) pair whose target cell is fluid, counted here
    independently from the table."""
    import ctypes
    from oracle.lattice import model_lattice
    lat = model_lattice(order)
    nx, ny, nz = 7, 5, 9
    rng = np.random.default_rng(order)
    solid = (rng.uniform(size=(nz, ny, nx)) < 0.3).astype(np.uint8)
    n = 0
    for z, y, x in zip(*np.nonzero(solid)):
        for tx, ty, tz in lat.theta:
            if not solid[(z + tz) % nz, (y + ty) % ny, (x + tx) % nx]:
                n += 1
    def a256(v):
        return (v + 255) // 256 * 256
    got = rlb.lib().rlb_walls_bytes(order, nx, ny, nz, ctypes.c_void_p(solid.ctypes.data))
    assert got == a256(nx * ny * nz) + a256(12 * n)
    full = np.ones((nz, ny, nx), dtype=np.uint8)
    assert rlb.lib().rlb_walls_bytes(order, nx, ny, nz, ctypes.c_void_p(full.ctypes.data)) == 0
    assert rlb.lib().rlb_walls_bytes(order, nx, ny, nz, None) == 0
    assert rlb.lib().rlb_walls_bytes(5, nx, ny, nz, ctypes.c_void_p(solid.ctypes.data)) == 0


def test_stream_probe_library_loads_and_rejects_bad_arguments():
    """The benchmark's streaming probe (not part of the method) is built
    beside the library; its argument checks run before any device call."""
    import ctypes
    from paper_1301_3423_amd import build as _b
    if not os.path.exists(_b.PROBE_OUT):
        pytest.skip("libstream_probe.so not built")
    f = ctypes.CDLL(_b.PROBE_OUT).stream_probe_ms
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    assert f(0, 4, 64, 16, 16, None, 0, 1, None) == -1.0      # no bytes
    assert f(0, 4, 64, 16, 16, None, 24, 1, None) == -1.0     # not a multiple of 16
    assert f(0, 3, 64, 16, 16, None, 32, 1, None) == -1.0     # unroll not 1, 2, 4 or 8
    assert f(4, 4, 64, 16, 16, None, 32, 1, None) == -1.0     # no such kind
    assert f(2, 4, 64, 16, None, None, 32, 1, None) == -1.0   # read without a sink
    assert f(0, 4, 64, None, 16, None, 32, 1, None) == -1.0   # copy without a source
