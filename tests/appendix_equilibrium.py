"""The closed-form discrete equilibria printed in Appendix B of the paper
(Eq. equi3rd for the third-order model, Eq. equi2nd for the second-order
one), restated term by term.  Tests use them as an independent pin of the
oracle, which builds the same equilibrium by projecting on Table I.

p = (p0, px, py, pz) are the contravariant components of the lattice
4-momentum p_i, U = (U0, Ux, Uy, Uz) the contravariant 4-velocity; both
formulas have Uz^2 and pz^2 eliminated by the mass-shell relations.
"""


def equi3rd(n, T, U, p, w):
    U0, Ux, Uy, Uz = U
    p0, px, py, pz = p
    pu = px * Ux + py * Uy + pz * Uz
    A = p0**3 * (T * U0 - 1) * (T**2 * (4 * U0**2 - 3 * (Ux**2 + Uy**2 + 1)) - 2 * T * U0 + 1)
    B = -p0**2 * (
        T**3 * (-2 * U0**2 * (3 * px * Ux + 3 * py * Uy + 2 * pz * Uz)
                + (Ux**2 + Uy**2 + 1) * (3 * px * Ux + 3 * py * Uy + pz * Uz)
                + 36 * U0**3 - 6 * U0 * (3 * Ux**2 + 3 * Uy**2 + 4))
        + 3 * T**2 * (2 * U0 * pu - 22 * U0**2 + 7 * (Ux**2 + Uy**2) + 9)
        - 3 * T * (pu - 14 * U0) - 15)
    C = -3 * p0 * (
        T**3 * (U0**3 * (px**2 + py**2 - 24)
                - U0 * (px**2 * (2 * Ux**2 + Uy**2 + 1)
                        + 2 * px * Ux * (py * Uy + pz * Uz)
                        + py * (py * Ux**2 + 2 * py * Uy**2 + py + 2 * pz * Uy * Uz)
                        - 12)
                + 12 * U0**2 * pu - 2 * pu)
        + T**2 * (px**2 * (-U0**2 + 2 * Ux**2 + Uy**2 + 1)
                  + 2 * px * Ux * (py * Uy + pz * Uz - 11 * U0)
                  + py**2 * (-U0**2 + Ux**2 + 2 * Uy**2 + 1)
                  + 2 * py * Uy * (pz * Uz - 11 * U0)
                  - 22 * pz * U0 * Uz + 56 * U0**2 - 14)
        + 2 * T * (6 * pu - 25 * U0) + 20)
    D = T * (
        px**3 * T**2 * Ux * (-3 * U0**2 + 4 * Ux**2 + 3 * Uy**2 + 3)
        + px**2 * T * (3 * (U0**2 - 2 * Ux**2 - Uy**2 - 1) * (-py * T * Uy + 6 * T * U0 - 7)
                       + pz * T * Uz * (-U0**2 + 4 * Ux**2 + Uy**2 + 1))
        + 3 * px * Ux * (T * (T * (py**2 * (-U0**2 + Ux**2 + 2 * Uy**2 + 1)
                                   + 2 * py * Uy * (pz * Uz - 6 * U0)
                                   - 12 * pz * U0 * Uz + 24 * U0**2 - 4)
                              + 14 * py * Uy + 14 * pz * Uz - 48 * U0) + 30)
        + py**3 * T**2 * Uy * (-3 * U0**2 + 3 * Ux**2 + 4 * Uy**2 + 3)
        + py**2 * T * (pz * T * Uz * (-U0**2 + Ux**2 + 4 * Uy**2 + 1)
                       + 3 * (6 * T * U0 - 7) * (U0**2 - Ux**2 - 2 * Uy**2 - 1))
        + 6 * py * Uy * (T * (2 * T * (-3 * pz * U0 * Uz + 6 * U0**2 - 1) + 7 * pz * Uz - 24 * U0) + 15)
        + 6 * pz * Uz * (2 * T**2 * (6 * U0**2 - 1) - 24 * T * U0 + 15)
        - 24 * U0 * (T**2 * (2 * U0**2 - 1) - 5 * T * U0 + 5))
    E = -30 * (T**2 - 2)
    return n * w / (12 * T) * (A + B + C + D + E)


def equi2nd(n, T, U, p, w):
    U0, Ux, Uy, Uz = U
    p0, px, py, pz = p
    pu = px * Ux + py * Uy + pz * Uz
    val = (p0**2 * (T**2 * (2 * U0**2 - Ux**2 - Uy**2 - 1) - 2 * T * U0 + 1)
           + 2 * p0 * (T * (T * (U0 * (pu - 4 * U0) + 1) - pu + 7 * U0) - 4)
           + T**2 * (px**2 * (-U0**2 + 2 * Ux**2 + Uy**2 + 1)
                     + 2 * px * Ux * (py * Uy + pz * Uz - 4 * U0)
                     + py**2 * (-U0**2 + Ux**2 + 2 * Uy**2 + 1)
                     + 2 * py * Uy * (pz * Uz - 4 * U0)
                     + 8 * U0 * (U0 - pz * Uz) - 2)
           + 2 * T * (5 * pu - 8 * U0) + 12)
    return n * w / (4 * T) * val
