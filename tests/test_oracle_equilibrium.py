"""Pins of the oracle's equilibrium (Eqs. MJ:eq, coeff, disc1,
moments:dis1-3, and Appendix B)."""
import numpy as np
import pytest

from appendix_equilibrium import equi2nd, equi3rd
from oracle import equilibrium as eqm
from oracle.equilibrium import Equilibrium, ETA


def _random_states(rng, m, vmax=0.9, tmin=0.5, tmax=1.5):
    v = rng.normal(size=(m, 3))
    v *= (vmax * rng.uniform(0, 1, m) ** (1 / 3) / np.linalg.norm(v, axis=1))[:, None]
    g = 1 / np.sqrt(1 - np.sum(v * v, axis=1))
    U = np.concatenate([g[:, None], g[:, None] * v], axis=1)
    T = rng.uniform(tmin, tmax, m)
    n = rng.uniform(0.5, 2.0, m)
    return n, T, U


def _mj_numeric(n, T, U, nth=96, nph=192):
    """Moments of A exp(-p.U/T) by quadrature: the radial integral is
    exact, int p^(k+1) exp(-a p) dp = (k+1)!/a^(k+2) with
    a = (U0 - nhat.U)/T, and the angles use Gauss-Legendre x uniform."""
    A = n / (8 * np.pi * T**3)                          # so that N^0 = n at rest
    x, wx = np.polynomial.legendre.leggauss(nth)
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    X, PH = np.meshgrid(x, ph, indexing="ij")
    S = np.sqrt(1 - X**2)
    nh = np.stack([np.ones_like(X), S * np.cos(PH), S * np.sin(PH), X], axis=0)   # (1, nhat)
    wang = (wx[:, None] * np.ones_like(PH)) * (2 * np.pi / nph)
    a = (U[0] - (nh[1] * U[1] + nh[2] * U[2] + nh[3] * U[3])) / T
    from math import factorial

    def radial(k):
        return factorial(k + 1) / a ** (k + 2)
    Z = A * np.sum(wang * radial(0))
    N = np.array([A * np.sum(wang * radial(1) * nh[m]) for m in range(4)])
    Tm = np.array([[A * np.sum(wang * radial(2) * nh[m] * nh[k]) for k in range(4)] for m in range(4)])
    P = np.array([[[A * np.sum(wang * radial(3) * nh[m] * nh[k] * nh[l]) for l in range(4)]
                   for k in range(4)] for m in range(4)])
    return Z, N, Tm, P


def test_mj_moments_against_quadrature():
    rng = np.random.default_rng(11)
    n, T, U = _random_states(rng, 4, vmax=0.6)
    Z, N, Tm, P = eqm.mj_moments(n, T, U)
    for c in range(4):
        z, nn, tt, pp = _mj_numeric(n[c], T[c], U[c])
        assert abs(Z[c] - z) < 1e-11 * abs(z)
        assert np.max(np.abs(N[c] - nn)) < 1e-11 * np.max(np.abs(nn))
        assert np.max(np.abs(Tm[c] - tt)) < 1e-11 * np.max(np.abs(tt))
        assert np.max(np.abs(P[c] - pp)) < 1e-11 * np.max(np.abs(pp))


def test_discrete_moments_reproduce_closed_forms(lat):
    """Eqs. moments:dis1-3: the first three moments of f_eq on the lattice
    are those of the continuous distribution."""
    rng = np.random.default_rng(3)
    n, T, U = _random_states(rng, 200)
    eq = Equilibrium(lat)
    f = eq(n, T, U)                                      # [c, Q]
    N = f @ lat.p
    Tm = np.einsum("ci,im,in->cmn", f, lat.p, lat.p)
    P = np.einsum("ci,im,in,il->cmnl", f, lat.p, lat.p, lat.p)
    _, N0, T0, P0 = eqm.mj_moments(n, T, U)
    def rel(a, b):
        return np.max(np.abs(a - b).reshape(len(n), -1).max(axis=1)
                      / np.abs(b).reshape(len(n), -1).max(axis=1))
    assert rel(N, N0) < 1e-12
    assert rel(Tm, T0) < 1e-12
    assert rel(P, P0) < 1e-12
    # and the printed forms of T and P directly (Sec. II C)
    for c in range(5):
        u = U[c]
        Tp = -n[c] * T[c] * ETA + 4 * n[c] * T[c] * np.outer(u, u)
        assert np.max(np.abs(Tm[c] - Tp)) < 1e-12 * np.abs(Tp).max()


def test_rest_frame_reference_state_is_the_weight(lat):
    """At U = (1,0,0,0) and T = 1 the Maxwell-Juttner distribution is the
    weight function itself when n = 2 (4 pi A = 1), so f_i^eq = w_i."""
    eq = Equilibrium(lat)
    f = eq(np.array([2.0]), np.array([1.0]), np.array([[1.0, 0, 0, 0]]))[0]
    assert np.max(np.abs(f - lat.w)) < 1e-15


def test_equilibrium_matches_appendix_third_order(lat):
    rng = np.random.default_rng(5)
    n, T, U = _random_states(rng, 100)
    f = Equilibrium(lat)(n, T, U)
    for c in range(len(n)):
        g = equi3rd(n[c], T[c], U[c], lat.p.T, lat.w)
        assert np.max(np.abs(f[c] - g)) < 1e-12 * np.max(np.abs(g)), c


def test_second_order_equilibrium_matches_appendix(lat):
    """Keeping J_0..J_13 gives Eq. equi2nd (evaluated here on the
    third-order points; the formula holds pointwise)."""
    rng = np.random.default_rng(6)
    n, T, U = _random_states(rng, 50)
    f = Equilibrium(lat, kmax=14)(n, T, U)
    for c in range(len(n)):
        g = equi2nd(n[c], T[c], U[c], lat.p.T, lat.w)
        assert np.max(np.abs(f[c] - g)) < 1e-12 * np.max(np.abs(g)), c


def test_equilibrium_is_linear_in_n(lat):
    rng = np.random.default_rng(8)
    n, T, U = _random_states(rng, 10)
    eq = Equilibrium(lat)
    a, b = eq(3 * n, T, U), 3 * eq(n, T, U)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_rest_equilibrium_positive_only_between_0745_and_220(lat):
    """At rest the third-order equilibrium depends on a point only through
    its shell energy, and it is positive on every shell only for
    0.745 < T < 2.20 (a property of the four Laguerre energies and the
    projection, the same for any weight vertex; the paper's remark that
    large reference temperatures are unstable rests on it)."""
    eq = Equilibrium(lat)
    U = np.array([[1.0, 0, 0, 0]])
    def min_ratio(T):
        return float((eq(np.array([1.0]), np.array([T]), U)[0] / lat.w).min())
    for T in (0.75, 1.0, 1.5, 2.2):
        assert min_ratio(T) > 0, T
    for T in (0.745, 2.21):
        assert min_ratio(T) < 0, T
    # the ratio depends on the shell only
    f = eq(np.array([1.3]), np.array([0.9]), U)[0] / lat.w
    for l in range(4):
        r = f[lat.shell == l]
        assert np.ptp(r) < 1e-13 * np.max(np.abs(r)), l
