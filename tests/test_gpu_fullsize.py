"""Parity at the benchmark sizes, in the launch configuration bench.py
times, on sampled cells the oracle can compute one by one: after k steps a
cell depends only on cells within 6k (the largest displacement is 6), so the
oracle runs a periodic window of the initial fields of edge 12k + 1 + 2r
centred on a sample, and the (2r + 1)^3 cells around its centre are exact.
Samples include the box corners (the periodic wrap) and a cube across the
x boundary between storage tiles."""
import numpy as np
import pytest

from gpu_util import note
from oracle import rlb as orlb
from paper_1301_3423_amd import inputs, rlb

pytestmark = pytest.mark.gpu

K = 2                      # steps
RIN = 3                    # half edge of the exact cube compared around a sample
H = 6 * K + RIN            # half edge of the oracle window
W = 2 * H + 1              # window edge


def _window(a, c):
    """Periodic window of edge W centred on cell c = (z, y, x)."""
    idx = [np.arange(ci - H, ci + H + 1) % n for ci, n in zip(c, a.shape)]
    return a[np.ix_(*idx)]


def _samples(edge, rng, count=6):
    pts = [(0, 0, 0), (edge - 1, edge - 1, edge - 1), (edge // 2, 0, edge - 1), (edge // 3, 1, 64)]
    while len(pts) < count:
        pts.append(tuple(int(v) for v in rng.integers(0, edge, 3)))
    return pts


@pytest.mark.parametrize("edge,precision,vmax,eta_s,seed,order", [
    (128, "fp64", 0.5, 0.2, 2, 3),     # the 128^3 float64 configuration
    (256, "fp64", 0.6, 0.5, 3, 3),     # 256^3 float64 (timed next to the mixed one)
    (256, "mixed", 0.6, 0.5, 3, 3),    # the 256^3 mixed configuration
    (256, "fp64", 0.6, 0.5, 3, 2),     # the same boxes with the second-order model
    (256, "mixed", 0.6, 0.5, 3, 2),    # (displacements <= 3: the window is wider than needed)
])
def test_sampled_cells_at_full_size(lat, edge, precision, vmax, eta_s, seed, order):
    from oracle.lattice import model_lattice
    if order == 2:
        lat = model_lattice(2)
    note("full size %d^3 %s order %d, %d steps, %d^3 cells around each sample" % (edge, precision, order, K, 2 * RIN + 1))
    fields = inputs.random_box(edge, edge, edge, vmax, seed)
    s = rlb.Solver(edge, edge, edge, precision=precision, eta_s=eta_s, order=order)
    s.init_fields(*fields)
    s.step(K)
    out = s.read_fields()
    flags, _ = s.status()
    assert flags == 0
    del s
    tol = 1e-12 if precision == "fp64" else 1e-5
    rng = np.random.default_rng(edge)
    worst = 0.0
    inner = np.arange(H - RIN, H + RIN + 1)
    pts = _samples(edge, rng)
    for c in pts:
        win = [_window(a, c) for a in fields]
        o = orlb.Solver(W, W, W, lat=lat, eta_s=eta_s, order=order)
        o.init_fields(*win)
        o.step(K)
        ref = o.read_fields()
        # the exact cube: window cells H - RIN .. H + RIN on each axis, the
        # box cells c - RIN .. c + RIN (periodic)
        mids = np.ravel(inner[:, None, None] * W * W + inner[None, :, None] * W + inner[None, None, :])
        gz, gy, gx = [np.arange(ci - RIN, ci + RIN + 1) % edge for ci in c]
        flat = np.ravel(gz[:, None, None] * edge * edge + gy[None, :, None] * edge + gx[None, None, :])
        U0 = ref["U"][0, mids]
        errs = [np.max(np.abs(out[k][flat] - ref[k][mids]) / ref[k][mids]) for k in ("n", "eps", "P")] + \
               [np.max(np.abs(out["U"][j, flat] - ref["U"][j, mids]) / U0) for j in range(4)]
        worst = max(worst, max(errs))
        assert max(errs) <= tol, (c, errs)
    note("worst relative error over %d cells: %.2e" % (len(pts) * (2 * RIN + 1) ** 3, worst))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("order", [3, 2])
def test_shear_wave_decays_at_the_kinetic_viscosity(precision, order):
    """A property that holds at any size: a small shear wave v_x = A sin(kz)
    decays at nu = (tau - 1/2) R^2 / 5 cells^2/step (the Anderson-Witting
    viscosity, pinned on the oracle in test_oracle_viscosity.py), here on a
    64 x 4 x 128 box through the kernels bench.py times (the row kernel for
    mixed precision)."""
    nx, ny, nz, tau = 64, 4, 128, 0.8
    z = np.arange(nz)
    mode = np.sin(2 * np.pi * z / nz)
    C = nx * ny * nz
    vx = np.broadcast_to((1e-3 * mode)[:, None, None], (nz, ny, nx)).ravel()
    s = rlb.Solver(nx, ny, nz, precision=precision, tau=tau, order=order)
    s.init_fields(np.ones(C), np.full(C, 3.0), vx, np.zeros(C), np.zeros(C))
    t, a = [], []
    for _ in range(10):
        s.step(5)
        r = s.read_fields()
        v = (r["U"][1] / r["U"][0]).reshape(nz, ny, nx).mean(axis=(1, 2))
        t.append(s.status()[1])
        a.append(np.dot(v, mode) * 2 / nz)
    t, a = np.array(t), np.array(a)
    sel = t >= 20
    rate = -np.polyfit(t[sel], np.log(np.abs(a[sel])), 1)[0]
    R = {3: np.sqrt(41.0), 2: 3.0}[order]
    ratio = rate / (2 * np.pi / nz) ** 2 / ((tau - 0.5) * R * R / 5)
    note("order %d %s: nu / nu_AW = %.4f" % (order, precision, ratio))
    assert abs(ratio - 1) < 0.02, ratio
