"""Pins of the oracle's stencil arithmetic against mathematics the paper fixes.

* Fourier symbol of the differenced flux reconstruction equals the printed
  leading error of Sec. 2.2 (i th + th^8/280 - i th^9/360 - th^10/560) and,
  for the fourth-order subset, i th + i th^5/720 + th^6/1440 (exact rationals).
* The oracle's interface routines (GRB states, F(f_L), F(f_R)) reproduce the
  exact rational results on polynomials: the differenced flux is exact for
  degree <= 7, the sixth-order gradient for degree <= 6.
"""
import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_coefficients.json")))


def symbol_series(name, nmax=10):
    """Coefficients c_n of th^n (complex as (re, im) Fractions) of
    sum_m a_m (e^{i m th} - e^{i (m-1) th})  (interface j+1/2 minus j-1/2)."""
    e = GOLD[name]
    a = [Fr(n, e["den"]) for n in e["num"]]
    out = {}
    for n in range(nmax + 1):
        s = sum(c * (Fr(m) ** n - Fr(m - 1) ** n) for c, m in zip(a, e["offsets"]))
        s = s / math.factorial(n)
        # multiply by i^n
        r = n % 4
        re, im = [(s, 0), (0, s), (-s, 0), (0, -s)][r]
        out[n] = (Fr(re), Fr(im))
    return out


def test_symbol_seventh_order():
    s = symbol_series("flux_left", 11)
    exp = {1: (0, 1), 8: (Fr(1, 280), 0), 9: (0, Fr(-1, 360)), 10: (Fr(-1, 560), 0)}
    for n in range(0, 11):
        assert s[n] == tuple(Fr(x) for x in exp.get(n, (0, 0))), n
    # the printed fixture in the golden file
    g = GOLD["symbol_7th"]["coeffs"]
    assert s[8][0] == Fr(g["8"][1], g["8"][2])
    assert s[9][1] == -Fr(g["9"][1], g["9"][2])
    assert s[10][0] == -Fr(g["10"][1], g["10"][2])


def test_symbol_fourth_order_subset():
    s = symbol_series("flux_left_4th", 7)
    exp = {1: (0, 1), 5: (0, Fr(1, 720)), 6: (Fr(1, 1440), 0)}
    for n in range(0, 7):
        assert s[n] == tuple(Fr(x) for x in exp.get(n, (0, 0))), n


def test_oracle_tables_symbol(orc):
    # the same symbol computed from the oracle's own table
    num, den = orc.table(5)
    offs = list(range(-4, 5))
    for n in range(2, 8):
        assert sum(Fr(c, den) * (Fr(m) ** n - Fr(m - 1) ** n) for c, m in zip(num, offs)) == 0
    assert sum(Fr(c, den) * (Fr(m) - Fr(m - 1)) for c, m in zip(num, offs)) == 1


def _interfaces(orc, f, h):
    """Apply the oracle's interface routine at j+1/2 and j-1/2 for j=0."""
    xs = np.arange(-5, 7) * h
    vals = f(xs)
    grads = np.array([orc.grad6(vals[k - 3:k + 4]) if 3 <= k <= len(vals) - 4 else np.nan
                      for k in range(len(vals))])
    # j=0 is index 5; j+1/2 needs values -4..5 -> idx 1..10, grads -2..3 -> idx 3..8
    right = orc.apply_interface(vals[1:11], grads[3:9])
    left = orc.apply_interface(vals[0:10], grads[2:8])
    return left, right


@pytest.mark.parametrize("m", range(0, 8))
def test_differenced_flux_exact_polynomials(orc, m):
    h = 0.5
    f = lambda x: (x + 0.3) ** m
    left, right = _interfaces(orc, f, h)
    deriv = m * (0.3) ** (m - 1) if m > 0 else 0.0
    for k in (2, 3):   # F(f_L), F(f_R)
        d = (right[k] - left[k]) / h
        assert abs(d - deriv) <= 1e-11 * (1 + abs(deriv)), (m, k, d, deriv)


def test_differenced_flux_not_exact_degree8(orc):
    h = 0.5
    f = lambda x: (x + 0.3) ** 8
    left, right = _interfaces(orc, f, h)
    d = (right[2] - left[2]) / h
    assert abs(d - 8 * 0.3 ** 7) > 1e-6


@pytest.mark.parametrize("m", range(0, 8))
def test_grb_states_are_flux_stencils(orc, m):
    """GRB states with the sixth-order gradient equal the flux stencils
    (the paper states eq. flux-full is eq. grb with the derivatives substituted)."""
    h = 0.37
    f = lambda x: np.cos(1.3 * x + 0.2) + (x + 0.1) ** m
    left, right = _interfaces(orc, f, h)
    for out in (left, right):
        assert abs(out[0] - out[2]) < 1e-13 and abs(out[1] - out[3]) < 1e-13


@pytest.mark.parametrize("m", range(0, 8))
def test_grad6_exact_degree6(orc, m):
    h = 0.25
    x = np.arange(-3, 4) * h + 0.7
    g = orc.grad6(x ** m) / h
    exact = m * 0.7 ** (m - 1) if m > 0 else 0.0
    if m <= 6:
        assert abs(g - exact) < 1e-12 * (1 + abs(exact))
    else:
        assert abs(g - exact) > 1e-8
