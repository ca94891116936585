"""Pins of the fourth-order GRB subset in the oracle (order = 4: alpha = 4,
beta = 0 in eqs. (good_6tth-order_scheme_flux), (alpha-beta); the flux
reconstruction of eq. (fourth)), and the comparison of the two schemes'
Fourier symbols (the dispersion and dissipation plots of the comparison of
fourth- and seventh-order GRB).

* the oracle's two-parameter path (eqs. alpha-beta, good_6tth-order_scheme_flux,
  eqn:how-second, eqn:lingrb written out in that order) at alpha = 38/7,
  beta = 3/190 reproduces the printed seventh-order states of eq. (eqn:grb);
* its states at alpha = 4, beta = 0 with the sixth-order gradient equal the
  printed eq. (fourth) and its mirror image;
* the differenced fourth-order flux is exact for polynomials of degree <= 4
  and not 5; the residual converges at order 4 on the vortex (7 for order 7);
* symbols from the oracle's own routines: at the grid cut-off the modified
  wavenumbers are exactly -2i/3 (fourth) and -32i/105 (seventh); the seventh-
  order scheme dissipates less at every resolved wavenumber, the fourth-order
  one disperses less above about 0.76 (and more below) -- as the paper states;
* free stream exact, conservation, x <-> y symmetry, and the same detector
  flags as order 7, in both variable sets.
"""
import math

import numpy as np
import pytest

from paper_2305_00762_amd import problems as PB


def sixth_order_gradient(v, k):
    """Delta x dPhi/dx at index k from the printed sixth-order formula."""
    return (45.0 * (v[k + 1] - v[k - 1]) - 9.0 * (v[k + 2] - v[k - 2]) + (v[k + 3] - v[k - 3])) / 60.0


def line_data(vals):
    """vals at offsets -7..8 (j = index 7) -> (v10 at -4..5, g6 at -2..3)."""
    g = np.array([sixth_order_gradient(vals, 7 + o) for o in range(-2, 4)])
    return vals[3:13], g


@pytest.mark.parametrize("seed", range(4))
def test_ab_family_reproduces_printed_seventh(orc, seed):
    rng = np.random.default_rng(seed)
    v10, g6 = rng.normal(size=10), rng.normal(size=6)
    ab = orc.apply_interface_ab(v10, g6, 38.0 / 7.0, 3.0 / 190.0)
    printed = orc.apply_interface(v10, g6, order=7)
    assert np.allclose(ab, printed[:2], rtol=0, atol=1e-13 * np.abs(v10).max())


@pytest.mark.parametrize("seed", range(4))
def test_fourth_order_states_are_printed_flux(orc, seed):
    rng = np.random.default_rng(100 + seed)
    v10, g6 = line_data(rng.normal(size=16))
    out = orc.apply_interface(v10, g6, order=4)
    # eq. (fourth) written out here, and its mirror image about j+1/2
    f = {o: v10[o + 4] for o in range(-4, 6)}
    c = [-1, -3, 64, -309, 1050, 771, -152, 21, -1]
    FL = sum(ci * f[o] for ci, o in zip(c, range(-4, 5))) / 1440.0
    FR = sum(ci * f[1 - o] for ci, o in zip(c, range(-4, 5))) / 1440.0
    assert abs(out[2] - FL) < 1e-13 and abs(out[3] - FR) < 1e-13
    assert abs(out[0] - out[2]) < 1e-13 and abs(out[1] - out[3]) < 1e-13
    # not the seventh-order values
    assert abs(orc.apply_interface(v10, g6, order=7)[2] - FL) > 1e-6


def _differenced(orc, f, h, order):
    xs = np.arange(-8, 10) * h           # j = 0 at index 8
    vals = f(xs)
    out = []
    for j in (-1, 0):                    # interfaces j+1/2 = -1/2 and +1/2
        v10, g6 = line_data(vals[8 + j - 7:8 + j + 9])
        out.append(orc.apply_interface(v10, g6, order=order))
    return (out[1] - out[0]) / h


@pytest.mark.parametrize("m", range(0, 6))
def test_fourth_order_differenced_flux_polynomials(orc, m):
    f = lambda x: (x + 0.3) ** m
    d = _differenced(orc, f, 0.5, 4)
    exact = m * 0.3 ** (m - 1) if m > 0 else 0.0
    for k in range(4):
        if m <= 4:
            assert abs(d[k] - exact) <= 1e-11 * (1 + abs(exact)), (m, k)
        else:
            assert abs(d[k] - exact) > 1e-6, (m, k)


def _symbol(orc, order, th):
    """Modified wavenumber K(th) of the differenced F(f_L) of the oracle: the
    routine applied to cos and sin of m th gives the real and imaginary parts
    of sum_m a_m e^{i m th}; K = -i (S(j+1/2) - S(j-1/2)), exact K = th."""
    m = np.arange(-8, 10)
    out = []
    for fn in (np.cos, np.sin):
        vals = fn(m * th)
        s = []
        for j in (-1, 0):
            v10 = vals[8 + j - 4:8 + j + 6]
            g6 = np.zeros(6)             # F(f_L) reads values only
            s.append(orc.apply_interface(v10, g6, order=order)[2])
        out.append(s[1] - s[0])
    d = out[0] + 1j * out[1]
    return -1j * d


def test_symbols_at_cutoff_are_exact(orc):
    assert abs(_symbol(orc, 4, math.pi) - (-2j / 3)) < 1e-14
    assert abs(_symbol(orc, 7, math.pi) - (-32j / 105)) < 1e-14


def test_symbol_leading_terms(orc):
    th = 0.05
    k4, k7 = _symbol(orc, 4, th), _symbol(orc, 7, th)
    # K = th - i th^6/1440 - th^5/720 ... (fourth); th - i th^8/280 - th^9/360 (seventh)
    assert abs(k4.imag / (-th ** 6 / 1440) - 1) < 2e-2
    assert abs((k4.real - th) / (th ** 5 / 720) - 1) < 2e-2
    assert abs(k7.imag / (-th ** 8 / 280) - 1) < 5e-2


def test_dissipation_and_dispersion_comparison(orc):
    ths = np.linspace(0.02, math.pi, 400)
    k4 = np.array([_symbol(orc, 4, t) for t in ths])
    k7 = np.array([_symbol(orc, 7, t) for t in ths])
    # seventh order: lower dissipation at every wavenumber
    assert (np.abs(k7.imag) < np.abs(k4.imag)).all()
    # fourth order: slightly better dispersion at the higher wavenumbers ...
    hi = (ths > 0.8) & (ths < 3.1)
    assert (np.abs(k4.real - ths)[hi] < np.abs(k7.real - ths)[hi]).all()
    # ... and worse at the well-resolved ones, where the seventh order wins
    lo = ths < 0.7
    assert (np.abs(k7.real - ths)[lo] <= np.abs(k4.real - ths)[lo]).all()
    # both are upwind-dissipative, never anti-dissipative
    assert (k4.imag <= 1e-15).all() and (k7.imag <= 1e-15).all()


def test_order4_truncation_order_four(orc):
    from test_convergence import exact_dqdt
    errs = []
    for n in (128, 256, 512):
        P = PB.vortex(n, L=20.0, x0=-10.0)
        cfg = orc.make_cfg(n, n, *P.geometry(), order=4)
        R = orc.residual(cfg, P.Q)
        errs.append(np.abs(R[0] - exact_dqdt(n, 20.0, -10.0)[0]).mean())
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    # observed 4.13, 4.01
    assert all(3.8 < o < 4.4 for o in orders), (errs, orders)


@pytest.mark.parametrize("recon", [0, 1])
def test_order4_invariants(orc, recon):
    for bc in (PB.BC_PERIODIC, PB.BC_TRANSMISSIVE):
        P = PB.free_stream(20, bc=bc, mu=1e-3, ny=16)
        cfg = orc.make_cfg(P.nx, P.ny, *P.geometry(), mu=1e-3, recon=recon, order=4)
        assert (orc.residual(cfg, P.Q) == 0.0).all()
    for P in (PB.vortex(40), PB.riemann(40, seed=3)):
        Q = P.Q
        n = Q.shape[-1]
        cfg = orc.make_cfg(n, n, 0, 1, 0, 1, 0, 0, mu=1e-3, recon=recon, order=4)
        R = orc.residual(cfg, Q)
        assert np.isfinite(R).all()
        scale = np.abs(R).max(axis=(1, 2)) + 1.0
        assert (np.abs(R.sum(axis=(1, 2))) <= 1e-12 * n * n * scale).all()
        QT = np.stack([Q[0].T, Q[2].T, Q[1].T, Q[3].T]).copy()
        RT = orc.residual(cfg, QT)
        assert (RT[0] == R[0].T).all() and (RT[1] == R[2].T).all()
        assert (RT[2] == R[1].T).all() and (RT[3] == R[3].T).all()


def test_order4_same_flags_different_residual(orc):
    P = PB.riemann(48, seed=4, ny=40)
    res = [orc.residual(orc.make_cfg(P.nx, P.ny, *P.geometry(), order=o), P.Q, want_flags=True)
           for o in (7, 4)]
    assert (res[0][1] == res[1][1]).all() and (res[0][2] == res[1][2]).all()
    assert res[0][1].min() == 0
    assert not np.array_equal(res[0][0], res[1][0])


def test_order_validated(orc):
    P = PB.free_stream(16)
    with pytest.raises(Exception):
        orc.residual(orc.make_cfg(16, 16, *P.geometry(), order=5), P.Q)
