"""Pins of the Landau-Lifshitz solve (Eq. eigenproblem)."""
import numpy as np

from oracle import landau
from oracle.equilibrium import ETA


def _constructed(rng, m, vmax=0.95, pi_frac=0.3):
    """T = (4 eps/3) U U - (eps/3) eta + Pi with Pi symmetric, traceless
    and orthogonal to U, so that (eps, U) is an exact eigenpair."""
    out, Us, eps = [], [], []
    for _ in range(m):
        v = rng.normal(size=3)
        v *= vmax * rng.uniform() / np.linalg.norm(v)
        g = 1 / np.sqrt(1 - v @ v)
        U = g * np.array([1, *v])
        e = rng.uniform(0.5, 3)
        # projector onto the rest space of U
        Ul = ETA @ U
        Delta = ETA - np.outer(U, U)                      # Delta^{mu nu}
        Dm = Delta @ ETA                                  # Delta^mu_nu
        A = rng.normal(size=(4, 4))
        A = A + A.T
        Pi = Dm @ A @ Dm.T                                # orthogonal to U
        tr = np.trace(Pi @ ETA)                           # Pi^mu_mu
        Pi = Pi - tr / 3 * Delta                          # traceless
        Pi *= pi_frac * (e / 3) / np.abs(Pi).max()
        Tm = 4 * e / 3 * np.outer(U, U) - e / 3 * ETA + Pi
        assert np.allclose(Tm @ Ul, e * U)
        out.append(Tm)
        Us.append(U)
        eps.append(e)
    return np.array(out), np.array(Us), np.array(eps)


def test_recovers_constructed_eigenpairs():
    rng = np.random.default_rng(1)
    Tm, U, eps = _constructed(rng, 500)
    e, u, it, ok = landau.solve(Tm)
    assert ok.all()
    assert np.max(np.abs(e - eps) / eps) < 1e-12
    assert np.max(np.abs(u - U) / U[:, :1]) < 1e-11
    resid = np.einsum("cij,cj->ci", Tm, u @ ETA) - e[:, None] * u
    assert np.max(np.abs(resid) / Tm[:, 0, 0][:, None]) < 1e-13
    assert it.max() < 60


def test_matches_lapack_eig():
    rng = np.random.default_rng(2)
    Tm, U, eps = _constructed(rng, 50, pi_frac=0.5)
    e, u, _, ok = landau.solve(Tm)
    for c in range(50):
        w, V = np.linalg.eig(Tm[c] @ ETA)
        # timelike eigenvector: U.U > 0
        k = [j for j in range(4) if (V[:, j].real @ ETA @ V[:, j].real) > 0]
        assert len(k) == 1
        vv = V[:, k[0]].real
        vv = vv / np.sqrt(vv @ ETA @ vv) * np.sign(vv[0])
        assert abs(w[k[0]].real - e[c]) < 1e-12 * e[c]
        assert np.max(np.abs(vv - u[c])) < 1e-10 * u[c, 0]


def test_ideal_fluid_at_rest():
    Tm = np.array([np.diag([3.0, 1.0, 1.0, 1.0])])
    e, u, it, ok = landau.solve(Tm)
    assert ok[0] and abs(e[0] - 3.0) < 1e-15 and np.allclose(u[0], [1, 0, 0, 0], atol=0)
