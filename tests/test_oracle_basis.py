"""Table I is orthonormal under the continuous weight (Sec. II B), with the
reading of the garbled J_28; as printed, it is not."""
import sympy as sp

from exact_moments import weight_integral
from oracle import basis


def _integral(expr):
    poly = sp.Poly(sp.expand(expr), basis.p0, basis.px, basis.py, basis.pz)
    tot = 0
    for (a, b, c, d), coef in poly.terms():
        fr = weight_integral(a, b, c, d)
        tot += coef * sp.Rational(fr.numerator, fr.denominator)
    return sp.nsimplify(sp.simplify(tot))


def test_table_I_orthonormal():
    J = basis.TABLE_I
    for k in range(30):
        for l in range(k, 30):
            val = _integral(J[k] * J[l])
            assert val == (1 if k == l else 0), (k, l, val)


def test_printed_J28_duplicates_J27():
    printed = (basis.p0 - 6) * basis.py * basis.pz / (4 * sp.sqrt(3))
    assert sp.simplify(printed - basis.TABLE_I[27]) == 0
    # the printed entry cannot be orthogonal to J_27
    assert _integral(printed * basis.TABLE_I[27]) == 1


def test_degrees():
    degs = [basis.order(k) for k in range(30)]
    assert degs == [0] + [1] * 4 + [2] * 9 + [3] * 16
