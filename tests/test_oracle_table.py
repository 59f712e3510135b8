"""Pins of the quadrature table against what the paper fixes (Sec. II C,
Eqs. dio, mrecon2, eqs:eqs, ortho:qua)."""
import itertools
import os

import numpy as np
import pytest
import sympy as sp

from exact_moments import monomials, weight_integral

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_numbers():
    out = {}
    for line in open(os.path.join(GOLD, "paper_numbers.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, rest = line.split(None, 1)
        out[key] = rest.strip()
    return out


def _printed_directions():
    pats = [tuple(int(x) for x in l.split()) for l in open(os.path.join(GOLD, "paper_directions.txt"))
            if l.strip() and not l.startswith("#")]
    out = set()
    for pat in pats:
        for s in itertools.product((1, -1), repeat=3):
            out.add(tuple(a * b for a, b in zip(pat, s)))
    return out


def test_printed_directions_are_all_diophantine_solutions():
    printed = _printed_directions()
    sols = {d for d in itertools.product(range(-7, 8), repeat=3) if sum(x * x for x in d) == 41}
    assert len(sols) == 96
    assert printed == sols


def test_candidate_and_point_counts(lat):
    nums = _paper_numbers()
    assert 4 * 96 == int(nums["candidates_3rd"])
    assert lat.Q == int(nums["points_3rd"])
    assert len({(s, tuple(t)) for s, t in zip(lat.shell, lat.theta)}) == lat.Q


def test_energies_are_zeros_of_printed_radial_polynomial(lat):
    p = sp.symbols("p")
    R4 = (120 + p * (-240 + p * (120 + (p - 20) * p)))
    roots = sorted(float(r) for r in sp.Poly(R4, p).nroots(n=30))
    printed = [float(x) for x in _paper_numbers()["p0_3rd"].split()]
    shells = sorted(set(lat.p0))
    assert len(shells) == 4
    for s, r, pr in zip(shells, roots, printed):
        assert abs(s - r) <= 4e-16 * r
        # printed to 3-4 significant digits
        assert abs(s - pr) < 5e-3 * pr


def test_directions_and_pairing(lat):
    sols = _printed_directions()
    for t in lat.theta:
        assert tuple(t) in sols
    for i in range(lat.Q):
        j = lat.inv[i]
        assert j == i ^ 1
        assert np.array_equal(lat.theta[j], -lat.theta[i])
        assert lat.shell[j] == lat.shell[i]
        assert lat.w[j] == lat.w[i]                      # Eq. eqs:eqs, pairing
    assert np.all(lat.w > 0)                             # Eq. eqs:eqs, w >= 0 (retained points)
    assert abs(lat.w.sum() - 1.0) < 1e-15


def test_momentum_reconstruction(lat):
    # Eq. mrecon2: p = p0 (1, theta / R); p is light-like
    m2 = lat.p[:, 0] ** 2 - np.sum(lat.p[:, 1:] ** 2, axis=1)
    assert np.max(np.abs(m2) / lat.p[:, 0] ** 2) < 1e-15


@pytest.mark.parametrize("maxdeg", [6])
def test_exactness_up_to_sixth_order(lat, maxdeg):
    """Eqs. eqs:eqs: the discrete sums reproduce the weighted integrals of
    every monomial of degree <= 6 (orthonormality products up to degree 6,
    and the 4th, 5th and 6th moments)."""
    worst = 0.0
    for (a, b, c, d) in monomials(maxdeg):
        exact = float(weight_integral(a, b, c, d))
        num = float(np.sum(lat.w * lat.p[:, 0] ** a * lat.p[:, 1] ** b * lat.p[:, 2] ** c
                           * lat.p[:, 3] ** d))
        scale = float(weight_integral(a + b + c + d, 0, 0, 0))
        worst = max(worst, abs(num - exact) / scale)
    assert worst < 2e-14, worst


def test_seventh_order_is_not_exact(lat):
    """The rule is not exact beyond what the paper asks for: some degree-7
    angular moment fails (so the degree-6 check above is not vacuous)."""
    bad = 0
    for (a, b, c, d) in monomials(7):
        if a + b + c + d != 7:
            continue
        exact = float(weight_integral(a, b, c, d))
        num = float(np.sum(lat.w * lat.p[:, 0] ** a * lat.p[:, 1] ** b * lat.p[:, 2] ** c
                           * lat.p[:, 3] ** d))
        if abs(num - exact) > 1e-6 * float(weight_integral(7, 0, 0, 0)):
            bad += 1
    assert bad > 0


def test_discrete_orthonormality_of_table_I(lat):
    """Eq. ortho:qua: sum_i w_i J_l(p_i) J_k(p_i) = delta_lk."""
    from oracle import basis
    J = basis.evaluate(lat.p)
    G = (J * lat.w[None, :]) @ J.T
    assert np.max(np.abs(G - np.eye(30))) < 5e-13


def test_library_initialiser_matches_table(lat):
    """The C initialiser compiled into the library holds the same numbers."""
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1301_3423_amd", "lattice", "d3q128.inc")
    rows = [l.strip().strip("{},").split(",") for l in open(inc) if l.startswith("{")]
    assert len(rows) == lat.Q
    for i, r in enumerate(rows):
        tx, ty, tz, sh = (int(x) for x in r[:4])
        assert (tx, ty, tz) == tuple(lat.theta[i]) and sh == lat.shell[i]
        assert float.fromhex(r[4].strip()) == lat.p0[i]
        assert float.fromhex(r[5].strip()) == lat.w[i]
