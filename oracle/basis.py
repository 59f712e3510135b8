"""Table I: the polynomials J_0..J_29, orthonormal under the rest-frame
weight w(p0) = A exp(-p0) with measure d^3p/p0 (Sec. II B).

The table is restated here symbolically in the paper's notation
p^mu = (p0, px, py, pz).  One entry is garbled in the printed table: J_28
repeats J_27.  The reading used here is the polynomial that completes the
pattern of J_17/J_26 and makes all thirty orthonormal:
    J_28 = -py (p0^2 - 5 px^2) / (8 sqrt(30)).
"""
import sympy as sp
import numpy as np

p0, px, py, pz = sp.symbols("p0 px py pz")
s2, s3, s5, s6, s30 = sp.sqrt(2), sp.sqrt(3), sp.sqrt(5), sp.sqrt(6), sp.sqrt(30)

TABLE_I = [
    # 0th order
    sp.Integer(1),
    # 1st order
    (p0 - 2) / s2, px / s2, py / s2, pz / s2,
    # 2nd order
    ((p0 - 6) * p0 + 6) / (2 * s3),
    (p0 - 4) * px / (2 * s2), (p0 - 4) * py / (2 * s2), (p0 - 4) * pz / (2 * s2),
    (-p0**2 + px**2 + 2 * py**2) / (4 * s2),
    -(p0**2 - 3 * px**2) / (4 * s6),
    px * pz / (2 * s2), py * pz / (2 * s2), px * py / (2 * s2),
    # 3rd order
    sp.Rational(1, 12) * (p0 - 6)**2 * p0 - 2,
    ((p0 - 10) * p0 + 20) * px / (4 * s5),
    -sp.Rational(1, 24) * (p0 - 6) * (p0**2 - 3 * px**2),
    (5 * px**3 - 3 * p0**2 * px) / (24 * s5),
    ((p0 - 10) * p0 + 20) * py / (4 * s5),
    (p0 - 6) * px * py / (4 * s3),
    px * py * pz / (4 * s3),
    -(p0 - 6) * (p0**2 - px**2 - 2 * py**2) / (8 * s3),
    px * (-p0**2 + px**2 + 2 * py**2) / (8 * s3),
    py * (-3 * p0**2 + 3 * px**2 + 4 * py**2) / (24 * s2),
    ((p0 - 10) * p0 + 20) * pz / (4 * s5),
    (p0 - 6) * px * pz / (4 * s3),
    -pz * (p0**2 - 5 * px**2) / (8 * s30),
    (p0 - 6) * py * pz / (4 * s3),
    -py * (p0**2 - 5 * px**2) / (8 * s30),   # J_28, see module docstring
    pz * (-p0**2 + px**2 + 4 * py**2) / (24 * s2),
]
assert len(TABLE_I) == 30


def order(k):
    """Polynomial degree of J_k (0..3)."""
    return sp.Poly(TABLE_I[k], p0, px, py, pz).total_degree()


def terms(k):
    """J_k as a list of (exponents (a0, ax, ay, az), float coefficient)."""
    poly = sp.Poly(sp.expand(TABLE_I[k]), p0, px, py, pz)
    return [(tuple(int(e) for e in mon), float(c)) for mon, c in poly.terms()]


def evaluate(p, kmax=30):
    """J_k(p_i) for k < kmax at 4-momenta p[Q,4]; returns [kmax, Q]."""
    out = np.zeros((kmax, p.shape[0]))
    for k in range(kmax):
        for (a0, ax, ay, az), c in terms(k):
            out[k] += c * p[:, 0]**a0 * p[:, 1]**ax * p[:, 2]**ay * p[:, 3]**az
    return out
