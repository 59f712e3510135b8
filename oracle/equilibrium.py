"""Maxwell-Juttner moments and the discrete equilibrium (Sec. II B-C).

Metric: eta = diag(+1, -1, -1, -1); U^mu = gamma (1, v); natural units.

The continuous equilibrium f^MJ = A exp(-p.U/T) (Eq. MJ:eq) enters only
through its moments with the measure d^3p/p0:
    Z          = int f d^3p/p0          = n / (2 T)
    N^mu       = int f p^mu             = n U^mu
    T^{mu nu}  = int f p^mu p^nu        = -n T eta + 4 n T U U
    P^{mu nu l}= int f p^mu p^nu p^l    = -4 n T^2 (eta U + eta U + eta U) + 24 n T^2 U U U
N, T and P are printed with Eqs. moments:dis1-3.  Z is not printed; it
follows from Eq. MJ:eq in the rest frame (int A e^{-p/T} p dp dOmega =
4 pi A T^2 while n = 8 pi A T^3) and is a Lorentz scalar.

Projection (Eq. coeff): a_k = int f^MJ J_k d^3p/p0.  Each J_k is a
polynomial of degree <= 3, so a_k is the same linear combination of the
moment components above.

Discrete equilibrium (Eq. disc1): f_i^eq = w_i sum_k a_k J_k(p_i).
"""
import numpy as np

from . import basis

ETA = np.diag([1.0, -1.0, -1.0, -1.0])


def mj_moments(n, T, U):
    """Z[c], N[c,4], Tm[c,4,4], P[c,4,4,4] for arrays n[c], T[c], U[c,4]."""
    n = np.asarray(n, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    Z = n / (2.0 * T)
    N = n[:, None] * U
    UU = U[:, :, None] * U[:, None, :]
    Tm = (n * T)[:, None, None] * (4.0 * UU - ETA[None])
    UUU = UU[:, :, :, None] * U[:, None, None, :]
    etaU = (ETA[None, :, :, None] * U[:, None, None, :]
            + ETA[None, :, None, :] * U[:, None, :, None]
            + ETA[None, None, :, :] * U[:, :, None, None])
    P = (4.0 * n * T * T)[:, None, None, None] * (6.0 * UUU - etaU)
    return Z, N, Tm, P


def moment_component(Z, N, Tm, P, exps):
    """The MJ moment of the monomial p0^a0 px^ax py^ay pz^az: the component
    of the rank-(a0+ax+ay+az) moment tensor with that index multiset."""
    idx = [0] * exps[0] + [1] * exps[1] + [2] * exps[2] + [3] * exps[3]
    if len(idx) == 0:
        return Z
    if len(idx) == 1:
        return N[:, idx[0]]
    if len(idx) == 2:
        return Tm[:, idx[0], idx[1]]
    if len(idx) == 3:
        return P[:, idx[0], idx[1], idx[2]]
    raise ValueError("degree > 3")


def projections(n, T, U, kmax=30):
    """a_k(n, T, U) for k < kmax (Eq. coeff); returns [c, kmax]."""
    Z, N, Tm, P = mj_moments(n, T, U)
    a = np.zeros((len(Z), kmax))
    for k in range(kmax):
        for exps, c in basis.terms(k):
            a[:, k] += c * moment_component(Z, N, Tm, P, exps)
    return a


class Equilibrium:
    """Discrete equilibrium on a lattice (Eq. disc1), with J_k(p_i)
    evaluated once.  kmax = 30 is the third-order model; kmax = 14 keeps the
    polynomials up to second order (Appendix A's model, whose equilibrium
    Appendix B prints as Eq. equi2nd)."""

    def __init__(self, lat, kmax=30):
        self.lat = lat
        self.kmax = kmax
        self.J = basis.evaluate(lat.p, kmax)          # [kmax, Q]

    def __call__(self, n, T, U):
        """f_eq[c, Q] for arrays n[c], T[c], U[c,4]."""
        a = projections(n, T, U, self.kmax)           # [c, kmax]
        return (a @ self.J) * self.lat.w[None, :]
