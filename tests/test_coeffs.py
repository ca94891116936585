"""Pins of the oracle's stencil tables.

Two independent checks per table:
  (1) the paper's derivation, carried out here in exact rational arithmetic
      from the two-parameter interface gradient (Sec. 2.2, eqs.
      (eqn:how-second), (good_6tth-order_scheme_flux), (alpha-beta) with
      alpha=38/7, beta=3/190) and the Legendre interface formula
      (eq. eqn:lingrb), reproduces the printed coefficients;
  (2) the oracle's tables equal the printed coefficients (golden fixture).
"""
import json
import os
from fractions import Fraction as Fr

import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_coefficients.json")))


# linear forms over symbols ('v', k) = Phi_{j+k} and ('g', k) = Phi'_{j+k}
def lin(**kw):
    return dict(kw)


def add(*forms, coef=None):
    out = {}
    coef = coef or [1] * len(forms)
    for f, c in zip(forms, coef):
        for k, v in f.items():
            out[k] = out.get(k, 0) + Fr(c) * v
    return {k: v for k, v in out.items() if v != 0}


def shift(f, s):
    return {(t, k + s): v for (t, k), v in f.items()}


def V(k):
    return {("v", k): Fr(1)}


def G(k):
    return {("g", k): Fr(1)}


def second_derivative(alpha, beta):
    """dx^2 Phi_xx,j from eqs. (eqn:how-second), (good_6tth-order_scheme_flux),
    (alpha-beta), with Phi' = dx Phi_x."""
    phiL = add(V(0), G(0), V(1), V(0), V(-1), coef=[1, Fr(1, 2), beta, -2 * beta, beta])
    phiR = add(V(1), G(1), V(2), V(1), V(0), coef=[1, Fr(-1, 2), beta, -2 * beta, beta])
    # dx * (Phi_x)_{j+1/2} = (Phi'_j + Phi'_{j+1})/2 + alpha/2 (Phi_R - Phi_L)
    gface = add(G(0), G(1), phiR, phiL, coef=[Fr(1, 2), Fr(1, 2), alpha / 2, -alpha / 2])
    return add(gface, shift(gface, -1), coef=[1, -1])


def grb_left(alpha, beta):
    # eq. (eqn:lingrb): Phi^L = Phi_j + dx/2 Phi_x + dx^2/12 Phi_xx
    return add(V(0), G(0), second_derivative(alpha, beta), coef=[1, Fr(1, 2), Fr(1, 12)])


def grb_right(alpha, beta):
    return add(V(1), G(1), shift(second_derivative(alpha, beta), 1),
               coef=[1, Fr(-1, 2), Fr(1, 12)])


def substitute_grad6(form):
    """Replace Phi'_{j+k} by the sixth-order formula of eq. (eqn:six)."""
    g = GOLD["grad6"]
    out = {}
    for (t, k), v in form.items():
        if t == "v":
            out[("v", k)] = out.get(("v", k), 0) + v
        else:
            for off, num in zip(g["offsets"], g["num"]):
                key = ("v", k + off)
                out[key] = out.get(key, 0) + v * Fr(num, g["den"])
    return {k: v for k, v in out.items() if v != 0}


def as_table(form, kind, offsets):
    return [form.get((kind, k), Fr(0)) for k in offsets]


def printed(name):
    e = GOLD[name]
    return [Fr(n, e["den"]) for n in e["num"]], e["offsets"]


A7 = Fr(*GOLD["alpha_beta_7th"]["alpha"])
B7 = Fr(*GOLD["alpha_beta_7th"]["beta"])


def test_second_derivative_matches_printed():
    f = second_derivative(A7, B7)
    vals, off = printed("second_values")
    assert as_table(f, "v", off) == vals
    grads, offg = printed("second_grads")
    assert as_table(f, "g", offg) == grads
    assert set(k for k in f if k[0] == "v") <= {("v", k) for k in off}


def test_grb_left_right_match_printed():
    L = grb_left(A7, B7)
    R = grb_right(A7, B7)
    for form, vn, gn in ((L, "grb_left_values", "grb_left_grads"),
                         (R, "grb_right_values", "grb_right_grads")):
        vals, off = printed(vn)
        grads, offg = printed(gn)
        assert as_table(form, "v", off) == vals
        assert as_table(form, "g", offg) == grads
        assert len(form) == len(off) + len(offg)


def test_flux_stencils_are_grb_with_grad6():
    FL = substitute_grad6(grb_left(A7, B7))
    FR = substitute_grad6(grb_right(A7, B7))
    vals, off = printed("flux_left")
    assert as_table(FL, "v", off) == vals and len(FL) == 9
    vals, off = printed("flux_right")
    assert as_table(FR, "v", off) == vals and len(FR) == 9


def test_fourth_order_subset():
    a4 = Fr(*GOLD["alpha_beta_4th"]["alpha"])
    b4 = Fr(*GOLD["alpha_beta_4th"]["beta"])
    FL = substitute_grad6(grb_left(a4, b4))
    vals, off = printed("flux_left_4th")
    assert as_table(FL, "v", off) == vals


def test_mp_curvature_is_fourth_order_second_derivative():
    # d_j of eq. (eqn:mp-procedure): 2(P_{j+1}-2P_j+P_{j-1}) - (P'_{j+1}-P'_{j-1})/2
    d = add(V(1), V(0), V(-1), G(1), G(-1), coef=[2, -4, 2, Fr(-1, 2), Fr(1, 2)])
    assert d == second_derivative(Fr(4), Fr(0))


TABLES = {0: "grad6", 1: "grb_left_values", 2: "grb_left_grads", 3: "grb_right_values",
          4: "grb_right_grads", 5: "flux_left", 6: "flux_right", 7: "second_values",
          8: "second_grads"}


@pytest.mark.parametrize("which", sorted(TABLES))
def test_oracle_tables_are_printed(orc, which):
    num, den = orc.table(which)
    e = GOLD[TABLES[which]]
    assert [Fr(n, den) for n in num] == [Fr(n, e["den"]) for n in e["num"]]


# The stage kernels hold the reconstruction as stencils on edge jumps
# E_a = Phi_{j+a-3} - Phi_{j+a-4} (a = 0..8, j the left cell of the interface):
# the GRB state with the sixth-order gradients substituted, minus Phi_j (left)
# or Phi_{j+1} (right), is linear in the jumps because its weights sum to one.
EDGE_STENCILS = {
    # order: (denominator, left weights E0..E8, right weights E0..E8)
    7: (840, [1, -1, -23, 123, 395, -89, 15, -1, 0], [0, 1, -15, 89, -395, -123, 23, 1, -1]),
    4: (1440, [1, 4, -60, 249, 639, -132, 20, -1, 0], [0, 1, -20, 132, -639, -249, 60, -4, -1]),
}


def edge_form(den, w):
    out = {}
    for a, c in enumerate(w):
        for k, s in ((a - 3, 1), (a - 4, -1)):
            out[("v", k)] = out.get(("v", k), 0) + Fr(c * s, den)
    return {k: v for k, v in out.items() if v != 0}


@pytest.mark.parametrize("order", [7, 4])
def test_edge_jump_stencils_are_grb_with_grad6(order):
    ab = GOLD["alpha_beta_7th" if order == 7 else "alpha_beta_4th"]
    a, b = Fr(*ab["alpha"]), Fr(*ab["beta"])
    den, wl, wr = EDGE_STENCILS[order]
    assert edge_form(den, wl) == add(substitute_grad6(grb_left(a, b)), V(0), coef=[1, -1])
    assert edge_form(den, wr) == add(substitute_grad6(grb_right(a, b)), V(1), coef=[1, -1])


def test_grad6_on_edge_pairs():
    # eq. (eqn:six) at cell 0 as (37, -8, 1)/60 on the edge pairs around it
    e = lambda k: add(V(k + 1), V(k), coef=[1, -1])
    g = add(e(-1), e(0), e(-2), e(1), e(-3), e(2),
            coef=[Fr(37, 60), Fr(37, 60), Fr(-8, 60), Fr(-8, 60), Fr(1, 60), Fr(1, 60)])
    assert g == substitute_grad6(G(0))
