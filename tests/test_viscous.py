"""Pins of the viscous flux (Sec. 2.1, eqs. visc-interface, alphad, sixth-ordergrad).

* Shear u = sin(2 pi y) on a still, uniform gas: the x-momentum residual is
  mu u_yy and converges at 4th order (alpha_v = 4 with the sixth-order
  gradient gives a fourth-order viscous operator, Sec. 2.1).
* Heat conduction: rho = 1 + 0.1 sin(2 pi x), p = 1, u = v = 0: the energy
  residual is mu/(Pr (gamma-1)) T_xx with T = gamma p / rho, at 4th order.
* Cross term: u = sin(2 pi y), v = sin(2 pi x): the y-momentum residual holds
  mu (v_xx) from tau_xy and the x-momentum one mu u_yy.
"""
import math

import numpy as np
import pytest

from paper_2305_00762_amd import problems as PB


def run(orc, rho, u, v, p, mu, Pr=0.72):
    ny, nx = rho.shape
    Q = PB.prim_to_state(rho, u, v, p)
    cfg = orc.make_cfg(nx, ny, 0.0, 1.0, 0.0, 1.0, 0, 0, gamma=1.4, mu=mu, Pr=Pr)
    return orc.residual(cfg, Q)


def orders(errs):
    return [math.log2(a / b) for a, b in zip(errs, errs[1:])]


def test_shear_fourth_order(orc):
    mu, errs = 0.01, []
    for n in (32, 64, 128):
        X, Y = PB.cell_centres(n, n, 0, 1, 0, 1)
        u = np.sin(2 * np.pi * Y)
        R = run(orc, np.ones_like(X), u, np.zeros_like(X), np.ones_like(X), mu)
        exact = -mu * (2 * np.pi) ** 2 * np.sin(2 * np.pi * Y)
        errs.append(np.abs(R[1] - exact).max())
        assert np.abs(R[0]).max() < 1e-12
    assert min(orders(errs)) > 3.7, errs


def test_heat_conduction_fourth_order(orc):
    mu, Pr, g, errs = 0.01, 0.72, 1.4, []
    for n in (64, 128, 256):
        X, Y = PB.cell_centres(n, n, 0, 1, 0, 1)
        rho = 1 + 0.1 * np.sin(2 * np.pi * X)
        zero, one = np.zeros_like(X), np.ones_like(X)
        # viscous part only: residual with mu minus residual without
        R = run(orc, rho, zero, zero, one, mu, Pr) - run(orc, rho, zero, zero, one, 0.0, Pr)
        k = 2 * np.pi
        s = np.sin(k * X)
        # T = g / rho; T_xx = g (2 rho_x^2 / rho^3 - rho_xx / rho^2)
        rx, rxx = 0.1 * k * np.cos(k * X), -0.1 * k * k * s
        Txx = g * (2 * rx ** 2 / rho ** 3 - rxx / rho ** 2)
        exact = mu / (Pr * (g - 1)) * Txx
        errs.append(np.abs(R[3] - exact).max())
    assert min(orders(errs)) > 3.7, errs


def test_cross_terms(orc):
    mu, n = 0.05, 64
    X, Y = PB.cell_centres(n, n, 0, 1, 0, 1)
    u, v = np.sin(2 * np.pi * Y), np.sin(2 * np.pi * X)
    R_visc = run(orc, np.ones_like(X), u, v, np.ones_like(X), mu)
    R_inv = run(orc, np.ones_like(X), u, v, np.ones_like(X), 0.0)
    k2 = (2 * np.pi) ** 2
    assert np.abs((R_visc - R_inv)[1] + mu * k2 * np.sin(2 * np.pi * Y)).max() < 2e-4
    assert np.abs((R_visc - R_inv)[2] + mu * k2 * np.sin(2 * np.pi * X)).max() < 2e-4
