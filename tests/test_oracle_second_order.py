"""Pins of the second-order model of Appendix A in the oracle: its lattice
(R = 3, three energy shells, 66 of 90 candidate points), its equilibrium
(Table I up to J_13, Eq. equi2nd) and its time step."""
import itertools
import os

import numpy as np
import pytest
import sympy as sp

import bruteforce
from appendix_equilibrium import equi2nd
from exact_moments import monomials, weight_integral
from oracle import basis, rlb
from oracle import equilibrium as eqm
from oracle.equilibrium import Equilibrium
from oracle.lattice import model_lattice
from paper_1301_3423_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lat2():
    return model_lattice(2)


def _paper_numbers():
    out = {}
    for line in open(os.path.join(GOLD, "paper_numbers.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, rest = line.split(None, 1)
        out[key] = rest.strip()
    return out


def _printed_directions_2nd():
    pats = [tuple(int(x) for x in p.split()) for p in _paper_numbers()["dirs_2nd"].split("|")]
    out = set()
    for pat in pats:
        for s in itertools.product((1, -1), repeat=3):
            out.add(tuple(a * b for a, b in zip(pat, s)))
    return out


def test_printed_directions_are_all_solutions_for_R3():
    """Appendix A lists the directions of |theta|^2 = 9; they are all 30
    integer solutions, and 3 shells x 30 directions give the 90 candidates."""
    printed = _printed_directions_2nd()
    sols = {d for d in itertools.product(range(-4, 5), repeat=3) if sum(x * x for x in d) == 9}
    assert printed == sols and len(sols) == 30
    assert 3 * len(sols) == int(_paper_numbers()["candidates_2nd"])


def test_table_points_directions_and_pairing(lat2):
    assert lat2.Q == int(_paper_numbers()["points_2nd"]) == 66
    assert lat2.R2 == 9 and lat2.R == 3.0
    sols = _printed_directions_2nd()
    for t in lat2.theta:
        assert tuple(t) in sols
    assert len({(s, tuple(t)) for s, t in zip(lat2.shell, lat2.theta)}) == lat2.Q
    for i in range(lat2.Q):
        j = lat2.inv[i]
        assert j == i ^ 1
        assert np.array_equal(lat2.theta[j], -lat2.theta[i])
        assert lat2.w[j] == lat2.w[i] and lat2.shell[j] == lat2.shell[i]
    assert np.all(lat2.w > 0)
    assert abs(lat2.w.sum() - 1.0) < 1e-15


def test_energies_are_zeros_of_the_printed_R3(lat2):
    """p0_l are the zeros of R^(3) = p (p - 6)^2 / 12 - 2 (Appendix A),
    printed as 0.936, 3.305, 7.759."""
    p = sp.symbols("p")
    R3 = sp.Rational(1, 12) * p * (p - 6) ** 2 - 2
    roots = sorted(float(r) for r in sp.Poly(R3, p).nroots(n=30))
    printed = [float(x) for x in _paper_numbers()["p0_2nd"].split()]
    shells = sorted(set(lat2.p0))
    assert len(shells) == 3
    for s, r, pr in zip(shells, roots, printed):
        assert abs(s - r) <= 4e-16 * r
        assert abs(s - pr) < 5e-4 * pr
    # R^(3) is the radial third-order polynomial of Table I (J_14)
    assert sp.expand(basis.TABLE_I[14].subs(basis.p0, p) - R3) == 0


def test_momentum_reconstruction(lat2):
    m2 = lat2.p[:, 0] ** 2 - np.sum(lat2.p[:, 1:] ** 2, axis=1)
    assert np.max(np.abs(m2) / lat2.p[:, 0] ** 2) < 1e-15


def test_exact_to_fifth_degree_not_sixth(lat2):
    """The discrete sums reproduce the weighted integrals of every monomial
    of degree <= 5, and fail for some of degree 6."""
    def resid(deg_list):
        out = []
        for (a, b, c, d) in deg_list:
            exact = float(weight_integral(a, b, c, d))
            num = float(np.sum(lat2.w * lat2.p[:, 0] ** a * lat2.p[:, 1] ** b * lat2.p[:, 2] ** c
                               * lat2.p[:, 3] ** d))
            out.append(abs(num - exact) / float(weight_integral(a + b + c + d, 0, 0, 0)))
        return np.array(out)
    assert resid(monomials(5)).max() < 2e-14
    six = [m for m in monomials(6) if sum(m) == 6]
    assert resid(six).max() > 1e-6


def test_discrete_orthonormality_up_to_second_order(lat2):
    """Eq. ortho:qua for the polynomials the model keeps (J_0..J_13); the
    third-order polynomials are not orthonormal on this lattice."""
    J = basis.evaluate(lat2.p)
    G = (J * lat2.w[None, :]) @ J.T
    assert np.max(np.abs(G[:14, :14] - np.eye(14))) < 5e-14
    assert np.max(np.abs(G[14:, 14:] - np.eye(16))) > 1e-3


def _random_states(rng, m, vmax=0.8):
    v = rng.normal(size=(m, 3))
    v *= (vmax * rng.uniform(0, 1, m) ** (1 / 3) / np.linalg.norm(v, axis=1))[:, None]
    g = 1 / np.sqrt(1 - np.sum(v * v, axis=1))
    U = np.concatenate([g[:, None], g[:, None] * v], axis=1)
    return rng.uniform(0.5, 2.0, m), rng.uniform(0.5, 1.5, m), U


def test_equilibrium_is_the_appendix_formula(lat2):
    """Eq. equi2nd, restated term by term, at the 66 points."""
    rng = np.random.default_rng(21)
    n, T, U = _random_states(rng, 60)
    f = Equilibrium(lat2, kmax=14)(n, T, U)
    for c in range(len(n)):
        g = equi2nd(n[c], T[c], U[c], lat2.p.T, lat2.w)
        assert np.max(np.abs(f[c] - g)) < 1e-12 * np.max(np.abs(g)), c


def test_equilibrium_reproduces_N_and_T_but_not_P(lat2):
    """The model recovers the moments up to the energy-momentum tensor
    (Fig. 2 caption: up to the second-order moment) and, as Appendix A
    states, not the third-order moment."""
    rng = np.random.default_rng(22)
    n, T, U = _random_states(rng, 100)
    f = Equilibrium(lat2, kmax=14)(n, T, U)
    N = f @ lat2.p
    Tm = np.einsum("ci,im,in->cmn", f, lat2.p, lat2.p)
    P = np.einsum("ci,im,in,il->cmnl", f, lat2.p, lat2.p, lat2.p)
    _, N0, T0, P0 = eqm.mj_moments(n, T, U)
    def rel(a, b):
        return (np.abs(a - b).reshape(len(n), -1).max(axis=1)
                / np.abs(b).reshape(len(n), -1).max(axis=1))
    assert rel(N, N0).max() < 1e-12
    assert rel(Tm, T0).max() < 1e-12
    assert rel(P, P0).max() > 1e-3


def test_rest_state_is_the_weight(lat2):
    f = Equilibrium(lat2, kmax=14)(np.array([2.0]), np.array([1.0]), np.array([[1.0, 0, 0, 0]]))[0]
    assert np.max(np.abs(f - lat2.w)) < 1e-15


def test_relaxation_time_from_the_fitted_viscosity(lat2):
    """eta_2nd = (1/7) P (tau - 1/2) / R with P = n T (Appendix A) and
    s = 4n - n ln(n/T^3): solving for tau at a few states."""
    n = np.array([1.0, 0.7, 2.0])
    T = np.array([1.0, 0.8, 1.3])
    eta_s = 0.05
    tau = rlb.relaxation_time(lat2, n, T, eta_s=eta_s, order=2)
    s = 4 * n - n * np.log(n / T**3)
    eta = (1.0 / 7.0) * n * T * (tau - 0.5) / lat2.R
    assert np.max(np.abs(eta / s - eta_s)) < 1e-15
    # a different model coefficient than the third-order one
    tau3 = rlb.relaxation_time(lat2, n, T, eta_s=eta_s, order=3)
    assert np.all(np.abs((tau - 0.5) / (tau3 - 0.5) - 14.0 / 3.0) < 1e-13)


def test_solver_selects_the_second_order_model():
    s = rlb.Solver(2, 2, 2, tau=1.0, order=2)
    assert s.lat.Q == 66 and s.eq.kmax == 14
    with pytest.raises(ValueError):
        rlb.Solver(2, 2, 2, tau=1.0, order=4)


def test_collision_conserves_N0_and_T0nu(lat2):
    rng = np.random.default_rng(23)
    s = rlb.Solver(5, 4, 3, eta_s=0.1, order=2)
    s.init_fields(*inputs.random_box(5, 4, 3, 0.6, 1))
    f2 = s.f.reshape(lat2.Q, -1) * (1 + 0.2 * rng.uniform(-1, 1, (lat2.Q, s.C)))
    fs, _ = rlb.collide(lat2, s.eq, f2, tau=0.8, order=2)
    p = lat2.p
    for mom in (p[:, 0], p[:, 0] * p[:, 0], p[:, 0] * p[:, 1], p[:, 0] * p[:, 2], p[:, 0] * p[:, 3]):
        scale = (p[:, 0] ** 2) @ np.abs(f2)
        assert np.max(np.abs(mom @ fs - mom @ f2) / scale) < 1e-14
    assert np.max(np.abs(p[:, 1] @ fs - p[:, 1] @ f2)) > 1e-6


def test_global_conservation_and_stationary_boost():
    s = rlb.Solver(6, 5, 7, eta_s=0.2, order=2)
    s.init_fields(*inputs.random_box(6, 5, 7, 0.5, 2))
    c0 = s.conserved()
    s.step(40)
    assert np.max(np.abs(s.conserved() - c0)) / abs(c0[1]) < 1e-13
    assert s.flags == 0
    u = rlb.Solver(3, 4, 5, eta_s=0.2, order=2)
    C = u.C
    u.init_fields(np.full(C, 1.3), np.full(C, 3.51), np.full(C, 0.3), np.full(C, -0.4), np.full(C, 0.5))
    f0 = u.f.copy()
    u.step(3)
    assert np.max(np.abs(u.f - f0)) < 3e-14 * np.max(np.abs(f0))


@pytest.mark.parametrize("shape,kw", [((1, 1, 11), dict(eta_s=0.05)),
                                      ((2, 3, 4), dict(tau=0.7)),
                                      ((3, 3, 3), dict(eta_s=0.3))])
def test_bruteforce_agrees_with_oracle(shape, kw):
    nx, ny, nz = shape
    s = rlb.Solver(nx, ny, nz, order=2, **kw)
    s.init_fields(*inputs.random_box(nx, ny, nz, 0.5, 7))
    f = s.f.copy()
    for _ in range(3):
        f = bruteforce.step(s.lat, f, (nz, ny, nx), order=2, **kw)
    s.step(3)
    assert np.max(np.abs(f - s.f)) < 1e-12 * np.max(np.abs(f))


def test_models_differ_on_the_same_flow():
    """Same initial fields, same eta/s: the two models give different
    fields after a few steps (the second-order model is not a relabelled
    third-order one), but the same conserved totals."""
    fields = inputs.random_box(4, 4, 4, 0.4, 3)
    a = rlb.Solver(4, 4, 4, eta_s=0.1, order=3)
    b = rlb.Solver(4, 4, 4, eta_s=0.1, order=2)
    a.init_fields(*fields)
    b.init_fields(*fields)
    assert np.max(np.abs(a.conserved() - b.conserved())) < 1e-12 * abs(a.conserved()[1])
    a.step(4)
    b.step(4)
    ra, rb = a.read_fields(), b.read_fields()
    assert np.max(np.abs(ra["n"] - rb["n"])) > 1e-6
