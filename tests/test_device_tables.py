"""The kernels' compile-time reference tables (paper_2402_00466_amd/csrc/mevp_ref.hpp)
against exact rational integrals, on the CPU.

The parallelogram and bilinear element updates apply the strain and
divergence as exact constant operators built from 1D integrals over one
reference interval (s = xi - 1/2 in [-1/2, 1/2]) of the Legendre factors
P0 = 1, P1 = s, P2 = s^2 - 1/12 and the quadratic Lagrange factors L0, L1, L2
on {-1/2, 0, 1/2}:
  I0[i][c] = int P_i L_c,  I1[i][c] = int P_i L_c',  I1s[i][c] = int P_i s L_c',
  norms int P_i^2.
The test parses the tables from the header and recomputes every entry with
exact rational polynomial arithmetic (fractions), independently of the
quadrature rules and of the oracle."""
import os
import re
from fractions import Fraction as Fr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2402_00466_amd", "csrc", "mevp_ref.hpp")


def _poly_mul(a, b):
    out = [Fr(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _deriv(a):
    return [i * a[i] for i in range(1, len(a))] or [Fr(0)]


def _integral(a):  # over [-1/2, 1/2]
    h = Fr(1, 2)
    return sum(c * (h ** (i + 1) - (-h) ** (i + 1)) / (i + 1) for i, c in enumerate(a))


P = [[Fr(1)], [Fr(0), Fr(1)], [Fr(-1, 12), Fr(0), Fr(1)]]
# Lagrange on nodes -1/2, 0, 1/2 (xi = 0, 1/2, 1)
L = [[Fr(0), Fr(-1), Fr(2)], [Fr(1), Fr(0), Fr(-4)], [Fr(0), Fr(1), Fr(2)]]
S = [Fr(0), Fr(1)]


def _table(name):
    text = open(HDR).read()
    m = re.search(name + r"\[3\]\[3\] = \{(.*?)\};", text, re.S)
    assert m, name
    vals = []
    for row in re.findall(r"\{([^{}]*)\}", m.group(1)):
        vals.append([_num(x) for x in row.split(",")])
    return vals


def _num(expr):
    expr = expr.strip()
    m = re.fullmatch(r"(-?\d+\.\d+)\s*/\s*(\d+\.\d+)", expr)
    if m:
        return Fr(m.group(1)) / Fr(m.group(2))
    return Fr(expr)


def test_lagrange_factors_interpolate():
    for c, node in enumerate((Fr(-1, 2), Fr(0), Fr(1, 2))):
        for d, poly in enumerate(L):
            val = sum(coef * node ** i for i, coef in enumerate(poly))
            assert val == (1 if c == d else 0)


def test_integral_tables_are_exact():
    I0, I1, I1s = _table("kI0"), _table("kI1"), _table("kI1s")
    for i in range(3):
        for c in range(3):
            assert I0[i][c] == _integral(_poly_mul(P[i], L[c])), ("I0", i, c)
            assert I1[i][c] == _integral(_poly_mul(P[i], _deriv(L[c]))), ("I1", i, c)
            assert I1s[i][c] == _integral(_poly_mul(_poly_mul(P[i], S), _deriv(L[c]))), ("I1s", i, c)


def test_norms_and_basis_index_tables():
    text = open(HDR).read()
    norms = [_num(x) for x in re.search(r"kNorm1D\[3\] = \{(.*?)\};", text).group(1).split(",")]
    assert norms == [_integral(_poly_mul(p, p)) for p in P]
    dgx = [int(x) for x in re.search(r"kDgX\[8\] = \{(.*?)\};", text).group(1).split(",")]
    dgy = [int(x) for x in re.search(r"kDgY\[8\] = \{(.*?)\};", text).group(1).split(",")]
    # 1, s, t, s^2-1/12, s t, t^2-1/12, (s^2-1/12) t, s (t^2-1/12)
    assert list(zip(dgx, dgy)) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (2, 1), (1, 2)]
