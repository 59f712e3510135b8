"""Pin of the oracle's eta/s -> tau map to the relaxation times the paper
prints.

Sec. III (Numerical Validation) runs its Riemann problem at eta/s = 0.5 with
temperatures 1.0 and 0.5 in numerical units (n = T^3 there: the printed
pressures are P = T^4) and states that the third-order model then needs
relaxation times of about 20 to 40.  The oracle's map
    tau = 1/2 + (3 R / (2 T)) (eta/s) (4 - ln(n / T^3))
comes from the shear viscosity eta = (2/3) n T (tau - 1/2) / R of the same
section and the entropy density s = 4 n - n ln(n / n_eq) with n_eq = T^3.
Those two relations leave room for misreadings (R multiplying or dividing,
the 2/3 on either side, n_eq with the gluon degeneracy d_G / pi^2); the
printed range tells them apart, and each misreading, planted in the oracle,
must fail the pin."""
import copy
import os

import numpy as np
import pytest

from oracle import rlb

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_numbers():
    out = {}
    for line in open(os.path.join(GOLD, "paper_numbers.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, rest = line.split(None, 1)
        out[key] = rest.split()
    return out


def _numbers(key):
    return np.array([float(x) for x in _paper_numbers()[key]])


def _riemann_taus(lat, order=3):
    """tau of the oracle at the two initial states of the Sec. III Riemann
    problem, eta/s = 0.5."""
    T = _numbers("riemann_T")
    n = T ** 3
    return rlb.relaxation_time(lat, n, T, eta_s=0.5, order=order)


def _in_printed_range(taus):
    lo, hi = _numbers("tau_range_eta_s_0.5")
    # the range is approximate: allow 5 % beyond either printed end
    return bool(np.all(taus >= 0.95 * lo) and np.all(taus <= 1.05 * hi))


def test_numerical_units_have_n_equal_T_cubed():
    """The printed pressures of the Riemann problem (1.0 at T = 1.0, 0.062 at
    T = 0.5) are P = T^4, i.e. n = T^3 with P = n T: the density at which
    the entropy's log term vanishes when n_eq = T^3."""
    P = _numbers("riemann_P")
    T = _numbers("riemann_T")
    assert np.allclose(T ** 4, P, rtol=0.01)


def test_oracle_tau_is_in_the_printed_range(lat):
    taus = _riemann_taus(lat)
    assert _in_printed_range(taus), taus
    # and the two ends are the two temperatures: tau scales as 1/T at n = T^3
    assert abs((taus[1] - 0.5) / (taus[0] - 0.5) - 2.0) < 1e-12


def _planted(lat, monkeypatch, kind):
    """The oracle with one misreading of the viscosity relations planted."""
    bad = copy.copy(lat)
    if kind == "divide_by_R":
        # eta = (2/3) n T (tau - 1/2) * R, i.e. tau - 1/2 carries 1/R
        bad.R = 1.0 / lat.R
    elif kind == "no_R":
        bad.R = 1.0
    elif kind == "no_two_thirds":
        # eta = n T (tau - 1/2) / R
        monkeypatch.setitem(rlb.VISCOSITY_C, 3, 1.0)
    elif kind == "two_thirds_inverted":
        monkeypatch.setitem(rlb.VISCOSITY_C, 3, 2.0 / 3.0)
    elif kind == "n_eq_with_degeneracy":
        # n_eq = d_G T^3 / pi^2 in the units where n = T^3: ln(n/n_eq) = ln(pi^2/16)
        orig = rlb.relaxation_time

        def tau_deg(lat_, n, T, tau=None, eta_s=None, order=3):
            return orig(lat_, n * np.pi ** 2 / 16.0, T, tau, eta_s, order)

        return lambda: tau_deg(lat, *_riemann_state(), eta_s=0.5)
    else:
        raise ValueError(kind)
    return lambda: rlb.relaxation_time(bad, *_riemann_state(), eta_s=0.5, order=3)


def _riemann_state():
    T = _numbers("riemann_T")
    return T ** 3, T


@pytest.mark.parametrize("kind", ["divide_by_R", "no_R", "no_two_thirds", "two_thirds_inverted",
                                  "n_eq_with_degeneracy"])
def test_misreadings_fail_the_pin(lat, monkeypatch, kind):
    taus = _planted(lat, monkeypatch, kind)()
    assert not _in_printed_range(taus), (kind, taus)

