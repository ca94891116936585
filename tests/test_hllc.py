"""Pins of the interface Riemann flux (HLLC, wave-sum form of eq. eqn:Riemann).

* Consistency: F(W, W, F(W), F(W)) = F(W).
* A stationary contact (u = 0, equal pressure) carries no mass flux.
* With F_L = F(Q_L), F_R = F(Q_R) the wave-sum form equals the piecewise
  textbook HLLC flux (Toro), written here in its other, case-by-case form.
"""
import numpy as np
import pytest

G = 1.4


def cons(W):
    r, u, v, p = W
    return np.array([r, r * u, r * v, p / (G - 1) + 0.5 * r * (u * u + v * v)])


def flux(W):
    r, u, v, p = W
    E = cons(W)[3]
    return np.array([r * u, r * u * u + p, r * u * v, u * (E + p)])


def textbook_hllc(WL, WR):
    rl, ul, vl, pl = WL
    rr, ur, vr, pr = WR
    QL, QR = cons(WL), cons(WR)
    cl, cr = np.sqrt(G * pl / rl), np.sqrt(G * pr / rr)
    hl, hr = (QL[3] + pl) / rl, (QR[3] + pr) / rr
    a, b = np.sqrt(rl), np.sqrt(rr)
    ut, vt, ht = (a * ul + b * ur) / (a + b), (a * vl + b * vr) / (a + b), (a * hl + b * hr) / (a + b)
    ct = np.sqrt((G - 1) * (ht - 0.5 * (ut * ut + vt * vt)))
    SL, SR = min(ul - cl, ut - ct), max(ur + cr, ut + ct)
    Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))

    def star(W, Q, S):
        r, u, v, p = W
        k = r * (S - u) / (S - Ss)
        return k * np.array([1, Ss, v, Q[3] / r + (Ss - u) * (Ss + p / (r * (S - u)))])

    if SL >= 0:
        return flux(WL)
    if Ss >= 0:
        return flux(WL) + SL * (star(WL, QL, SL) - QL)
    if SR >= 0:
        return flux(WR) + SR * (star(WR, QR, SR) - QR)
    return flux(WR)


@pytest.mark.parametrize("W", [(1.0, 0.3, -0.2, 0.7), (0.2, -2.0, 1.0, 0.05), (3.0, 5.0, 0.0, 1.0)])
def test_consistency(orc, W):
    W = np.array(W)
    F = orc.hllc(W, W, flux(W), flux(W))
    assert np.allclose(F, flux(W), rtol=1e-14, atol=1e-14)


def test_stationary_contact(orc):
    WL, WR = np.array([1.0, 0.0, 0.1, 1.0]), np.array([0.125, 0.0, -0.3, 1.0])
    F = orc.hllc(WL, WR, flux(WL), flux(WR))
    assert abs(F[0]) < 1e-15 and abs(F[1] - 1.0) < 1e-14


@pytest.mark.parametrize("seed", range(20))
def test_wave_sum_equals_textbook(orc, seed):
    rng = np.random.default_rng(seed)
    WL = np.array([rng.uniform(0.1, 2), rng.uniform(-3, 3), rng.uniform(-1, 1), rng.uniform(0.05, 2)])
    WR = np.array([rng.uniform(0.1, 2), rng.uniform(-3, 3), rng.uniform(-1, 1), rng.uniform(0.05, 2)])
    F = orc.hllc(WL, WR, flux(WL), flux(WR))
    T = textbook_hllc(WL, WR)
    assert np.allclose(F, T, rtol=1e-12, atol=1e-12 * np.abs(T).max())
