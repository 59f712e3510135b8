"""Sound waves on the oracle: the equation of state P = eps/3 of the
ultra-relativistic gas fixes the speed of sound at c/sqrt(3), and a
conformal fluid (no bulk viscosity) damps sound at (2/3) nu k^2 with
nu = eta/(eps + P).  In lattice units a population crosses R cells per
step (c = R cells/step) and nu = (tau - 1/2) R^2 / 5 (test_oracle_viscosity).
A small standing wave delta P ~ cos(kz) is fitted with a damped cosine."""
import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import rlb


def _fit(order, tau, L=128):
    z = np.arange(L)
    s = rlb.Solver(1, 1, L, tau=tau, order=order)
    mode = np.cos(2 * np.pi * z / L)
    T = 1 + 1e-3 * mode
    s.init_fields(T**3, 3 * T**4, np.zeros(L), np.zeros(L), np.zeros(L))
    R = s.lat.R
    k = 2 * np.pi / L
    w0 = k * R / np.sqrt(3)
    t, a = [], []
    for _ in range(int(3 * 2 * np.pi / w0)):
        s.step(1)
        r = s.read_fields()
        t.append(s.t)
        a.append(np.dot(r["P"] - r["P"].mean(), mode) * 2 / L)
    t, a = np.array(t, float), np.array(a)
    popt, _ = curve_fit(lambda t, A, g, w, p: A * np.exp(-g * t) * np.cos(w * t + p), t, a,
                        p0=(a[0], 0.0, w0, 0.0))
    return popt[2] / k / R, popt[1] / (k * k * (tau - 0.5) * R * R / 5)


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_speed_and_damping_of_sound(order, tau):
    cs_over_c, damping = _fit(order, tau)
    assert abs(cs_over_c * np.sqrt(3) - 1) < 3e-3, cs_over_c
    assert abs(damping - 2 / 3) < 0.03, damping
