"""Seeded synthetic initial fields (n, eps, v) shaped like the paper's
workloads.  This module holds no part of the scheme's arithmetic: it only
draws fields; the library and the test oracle both take them as input.

All fields are float64 arrays of shape (nz, ny, nx), x fastest.  Numerical
units follow Sec. III of the paper: at rest n = T^3 and P = n T = T^4, so
eps = 3 n T = 3 T^4.

random_box   smooth random flow: for each component (vx, vy, vz, theta)
             eight Fourier modes with integer wave vectors in [-4, 4]^3
             (redrawn when zero), amplitudes U(0.5, 1) and phases U(0, 2 pi);
             v is scaled so that max |v| = v_max exactly and
             T = 1 + 0.1 g_theta / max |g_theta|.
boosted_box  random_box with a uniform velocity composed onto it
             relativistically: a flow with net momentum, which a periodic
             box keeps for ever.
shock_tube   the Riemann problem of Sec. III: at rest, T = T_L for
             z < nz/2 and T_R otherwise.
tube_batch   the parameters of many shock tubes: lengths, temperature
             ratios and eta/s drawn from a seeded generator.
serve_requests  a stream of solve requests for the serving benchmark: 70 %
             shock tubes (N ~ U{200..8000}, 100..2000 steps, T_L/T_R ~
             U(1.1, 2)), 30 % periodic boxes (edge ~ U{32..128}, |v| <= 0.6,
             200..1000 steps), eta/s ~ U(0.01, 0.5), float64 or mixed
             precision with equal odds.
"""
import numpy as np


def _modes(rng, nmodes=8):
    out = []
    for _ in range(nmodes):
        k = rng.integers(-4, 5, 3)
        while not np.any(k):
            k = rng.integers(-4, 5, 3)
        a = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        out.append((k, a, ph))
    return out


def _field(modes, nx, ny, nz):
    """sum_j a_j cos(2 pi k_j . (x/nx, y/ny, z/nz) + phi_j) on the cell
    indices: the real part of a sum of separable complex exponentials,
    formed as one (z y) x j by j x x product."""
    ex = lambda k, n: np.exp(2j * np.pi * k * np.arange(n) / n)
    A = np.stack([(a * np.exp(1j * ph) * ex(k[2], nz))[:, None] * ex(k[1], ny)[None, :]
                  for k, a, ph in modes], axis=-1).reshape(nz * ny, len(modes))
    B = np.stack([ex(k[0], nx) for k, a, ph in modes], axis=0)
    return (A @ B).real.reshape(nz, ny, nx)


def box_modes(seed):
    """The Fourier modes of random_box for this seed: (vx, vy, vz, theta)."""
    rng = np.random.default_rng(seed)
    return tuple(_modes(rng) for _ in range(4))


def random_box(nx, ny, nz, v_max, seed):
    """Returns n, eps, vx, vy, vz for a periodic box."""
    mvx, mvy, mvz, mth = box_modes(seed)
    gx, gy, gz, gth = (_field(m, nx, ny, nz) for m in (mvx, mvy, mvz, mth))
    norm = np.sqrt(gx * gx + gy * gy + gz * gz).max()
    s = v_max / norm if norm > 0 else 0.0
    vx, vy, vz = gx * s, gy * s, gz * s
    gmax = np.abs(gth).max()
    T = 1.0 + 0.1 * gth / (gmax if gmax > 0 else 1.0)
    n = T ** 3
    eps = 3.0 * T ** 4
    return n, eps, vx, vy, vz


def boosted_box(nx, ny, nz, v_max, seed, boost):
    """random_box(nx, ny, nz, v_max, seed) seen from a frame moving with the
    uniform velocity -boost: each cell's velocity v becomes the relativistic
    sum boost (+) v = [v / g + b + g/(1 + g) (b.v) b] / (1 + b.v), g the
    Lorentz factor of b; n and eps (rest-frame scalars) are unchanged.
    |boost| + v_max < 1 keeps every speed below 1 with margin."""
    n, eps, vx, vy, vz = random_box(nx, ny, nz, v_max, seed)
    b = np.asarray(boost, dtype=np.float64)
    g = 1.0 / np.sqrt(1.0 - b @ b)
    bv = b[0] * vx + b[1] * vy + b[2] * vz
    c = g / (1.0 + g) * bv
    den = 1.0 + bv
    return (n, eps, (vx / g + b[0] + c * b[0]) / den, (vy / g + b[1] + c * b[1]) / den,
            (vz / g + b[2] + c * b[2]) / den)


def shock_tube(nz, T_left=1.0, T_right=0.8, nx=1, ny=1):
    """Returns n, eps, vx, vy, vz for a tube at rest with a temperature step."""
    z = np.arange(nz)
    T1 = np.where(z < nz // 2, T_left, T_right).astype(np.float64)
    T = np.broadcast_to(T1[:, None, None], (nz, ny, nx)).copy()
    n = T ** 3
    eps = 3.0 * T ** 4
    zero = np.zeros_like(T)
    return n, eps, zero, zero.copy(), zero.copy()


ETA_S_CHOICES = (0.01, 0.05, 0.1, 0.2, 0.5)


def tube_batch(ntubes, seed, n_min=200, n_max=4000):
    """Per tube (drawn in this order): length N, temperature ratio r
    (T_L = 1, T_R = 1/r) and eta/s."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(ntubes):
        N = int(rng.integers(n_min, n_max + 1))
        r = float(rng.uniform(1.1, 2.0))
        es = float(rng.choice(ETA_S_CHOICES))
        out.append(dict(N=N, T_left=1.0, T_right=1.0 / r, eta_s=es))
    return out


def serve_requests(nreq, seed=5):
    """Request descriptions (no fields): dicts with kind, shape, precision,
    steps, eta_s and the field recipe."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nreq):
        tube = rng.uniform() < 0.7
        if tube:
            N = int(rng.integers(200, 8001))
            steps = int(rng.integers(100, 2001))
            ratio = float(rng.uniform(1.1, 2.0))
            req = dict(kind="tube", shape=(1, 1, N), steps=steps, T_right=1.0 / ratio)
        else:
            e = int(rng.integers(32, 129))
            steps = int(rng.integers(200, 1001))
            req = dict(kind="box", shape=(e, e, e), steps=steps, v_max=0.6)
        req["eta_s"] = float(rng.uniform(0.01, 0.5))
        req["precision"] = "fp64" if rng.uniform() < 0.5 else "mixed"
        out.append(req)
    return out


def request_fields(req, cache=None):
    """Initial fields of a request; boxes of one edge share one field (seed =
    edge), cached in `cache` if given."""
    if req["kind"] == "tube":
        return shock_tube(req["shape"][2], 1.0, req["T_right"])
    e = req["shape"][0]
    if cache is not None and e in cache:
        return cache[e]
    f = random_box(e, e, e, req["v_max"], seed=e)
    if cache is not None:
        cache[e] = f
    return f


def _field_torch(modes, nx, ny, nz, device):
    """_field evaluated on a device with torch (complex128)."""
    import torch
    def ex(k, n):
        return torch.exp(2j * np.pi * k * torch.arange(n, device=device, dtype=torch.float64) / n)
    A = torch.stack([(complex(a * np.exp(1j * ph)) * ex(int(k[2]), nz))[:, None] * ex(int(k[1]), ny)[None, :]
                     for k, a, ph in modes], dim=-1).reshape(nz * ny, len(modes))
    B = torch.stack([ex(int(k[0]), nx) for k, a, ph in modes], dim=0)
    return (A @ B).real.contiguous().reshape(nz, ny, nx)


def random_box_device(nx, ny, nz, v_max, seed, device="cuda"):
    """random_box generated on a device (same modes, same formulas; equal to
    random_box up to rounding), for boxes too large to build on the host.
    Returns the five float64 tensors and the two normalisations used,
    (v_max / max |g_v|, max |g_theta|), so that field_window can rebuild any
    part of the same fields on the host."""
    import torch
    mvx, mvy, mvz, mth = box_modes(seed)
    gx, gy, gz = (_field_torch(m, nx, ny, nz, device) for m in (mvx, mvy, mvz))
    norm = float(torch.sqrt(gx * gx + gy * gy + gz * gz).max())
    sv = v_max / norm if norm > 0 else 0.0
    gx.mul_(sv), gy.mul_(sv), gz.mul_(sv)
    gth = _field_torch(mth, nx, ny, nz, device)
    gmax = float(gth.abs().max())
    T = gth.mul_(0.1 / (gmax if gmax > 0 else 1.0)).add_(1.0)
    n = T ** 3
    eps = 3.0 * T ** 4
    del T
    return (n, eps, gx, gy, gz), (sv, gmax)


def field_window(seed, shape, norms, idx):
    """n, eps, vx, vy, vz of random_box_device's fields on the cells
    idx = (z, y, x) (index arrays, combined as an open grid), evaluated
    directly from the modes on the host."""
    nx, ny, nz = shape
    sv, gmax = norms
    z, y, x = np.ix_(*idx)
    def g(modes):
        return sum(a * np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
                   for k, a, ph in modes)
    mvx, mvy, mvz, mth = box_modes(seed)
    vx, vy, vz = g(mvx) * sv, g(mvy) * sv, g(mvz) * sv
    T = 1.0 + 0.1 * g(mth) / (gmax if gmax > 0 else 1.0)
    return T ** 3, 3.0 * T ** 4, vx, vy, vz
