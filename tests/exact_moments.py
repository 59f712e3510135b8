"""Exact integrals of monomials against the rest-frame weight, from the
definitions of Sec. II B: w(p0) = A exp(-p0) with measure d^3p/p0 on the
light cone p0 = |p|, normalised so that the integral of w is 1 (4 pi A = 1,
J_0 = 1 has unit norm).  In spherical coordinates

    int w p0^a px^b py^c pz^d d^3p/p0 = Gamma(D + 2) <nx^b ny^c nz^d>

with D = a + b + c + d and <.> the average over the unit sphere, which is
(b-1)!!(c-1)!!(d-1)!!/(b+c+d+1)!! for even b, c, d and zero otherwise.
"""
from fractions import Fraction
from math import factorial


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def sphere_average(b, c, d):
    if b % 2 or c % 2 or d % 2:
        return Fraction(0)
    return Fraction(_dfact(b - 1) * _dfact(c - 1) * _dfact(d - 1), _dfact(b + c + d + 1))


def weight_integral(a, b, c, d):
    return factorial(a + b + c + d + 1) * sphere_average(b, c, d)


def monomials(maxdeg):
    out = []
    for D in range(maxdeg + 1):
        for a in range(D + 1):
            for b in range(D - a + 1):
                for c in range(D - a - b + 1):
                    out.append((a, b, c, D - a - b - c))
    return out
