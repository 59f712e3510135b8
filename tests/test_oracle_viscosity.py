"""The shear viscosity of the scheme, measured on the oracle from the decay
of a small transverse shear wave, against kinetic theory and against the
paper's numbers.

A wave v_x = A sin(k z) in a fluid at rest decays as exp(-nu k^2 t) with
nu = eta / (eps + P).  For the Anderson-Witting model of a massless gas
Chapman-Enskog gives eta = (4/5) P tau_R (textbook value); the lattice step
replaces tau_R by (tau - 1/2) delta t, and a population crosses R cells per
step, so in lattice units (cells, steps) nu = (tau - 1/2) R^2 / 5 for both
models.

The paper's relations eta = (2/3) n T (tau - 1/2) / R (Sec. III, third
order) and eta_2nd ~ (1/7) P (tau - 1/2) / R (Appendix A, a numerical fit)
fix the ratio of the two models' viscosities at equal tau in physical time
(delta t = R delta x / c): [(1/7)/3] / [(2/3)/sqrt(41)] = 0.457, which the
measured ratio must reproduce to within the accuracy of a fit."""
import numpy as np
import pytest

from oracle import rlb


def _nu(order, tau, L=64, steps=50, skip=20):
    z = np.arange(L)
    s = rlb.Solver(1, 1, L, tau=tau, order=order)
    mode = np.sin(2 * np.pi * z / L)
    s.init_fields(np.ones(L), np.full(L, 3.0), 1e-3 * mode, np.zeros(L), np.zeros(L))
    t, a = [], []
    for _ in range(steps):
        s.step(1)
        r = s.read_fields()
        t.append(s.t)
        a.append(np.dot(r["U"][1] / r["U"][0], mode) * 2 / L)
    t, a = np.array(t), np.array(a)
    sel = t >= skip
    rate = -np.polyfit(t[sel], np.log(np.abs(a[sel])), 1)[0]
    return rate / (2 * np.pi / L) ** 2, s.lat.R


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("tau", [0.6, 0.8])
def test_shear_viscosity_is_the_anderson_witting_value(order, tau):
    """Third order within 0.5 %; the second-order model, whose equilibrium
    misses the third moment that enters the viscous stress, within 1 %
    (measured 0.6-0.7 % above, at any wavelength)."""
    nu, R = _nu(order, tau)
    ratio = nu / ((tau - 0.5) * R * R / 5)
    assert abs(ratio - 1) < (5e-3 if order == 3 else 1e-2), ratio


def test_viscosity_grows_linearly_from_tau_one_half():
    """nu is proportional to tau - 1/2 (the lattice correction of tau)."""
    nus = [_nu(3, tau)[0] for tau in (0.55, 0.7)]
    assert abs(nus[1] / nus[0] - 0.2 / 0.05) < 0.02 * 4


def test_second_to_third_order_viscosity_ratio_matches_the_paper_fit():
    """At equal tau and in physical time (one step is R delta x / c, so
    nu_phys = nu_lattice / R for a fixed delta x)."""
    nu3, R3 = _nu(3, 0.8)
    nu2, R2 = _nu(2, 0.8)
    measured = (nu2 / R2) / (nu3 / R3)
    paper = ((1 / 7) / 3) / ((2 / 3) / np.sqrt(41))
    assert abs(measured / paper - 1) < 0.05, (measured, paper)
    # and the relaxation times the library derives from eta/s keep that ratio:
    # tau - 1/2 scales with VISC R, i.e. (7 * 3) / (1.5 * sqrt(41))
    lat3, lat2 = rlb.model_lattice(3), rlb.model_lattice(2)
    n, T = np.array([1.0]), np.array([1.0])
    t3 = rlb.relaxation_time(lat3, n, T, eta_s=0.1, order=3)[0] - 0.5
    t2 = rlb.relaxation_time(lat2, n, T, eta_s=0.1, order=2)[0] - 0.5
    assert abs(t2 / t3 - (7 * 3) / (1.5 * np.sqrt(41))) < 1e-12
