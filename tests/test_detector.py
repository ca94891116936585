"""Pins of the density discontinuity detector (Sec. 2.4, eqs. detector, buffer).

* eps closed form: 0.9 psi_c/(1-0.9 psi_c) xi^2 = 9/11,000,000.
* a = 0, b = xi gives psi = 0.9 psi_c (the design value of eps).
* A density step of height H >= 1e-3 flags exactly the 9 interfaces s-4..s+4
  around it (four cells have psi < psi_c, the buffer spans j-2..j+3);
  H = 1e-4 flags none.
* The smooth vortex gives no flags; the free stream (a = b = 0) gives psi = 1.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2305_00762_amd import problems as PB


def test_eps_closed_form(orc):
    eps = orc.detector_eps()
    assert abs(eps - 9 / 11_000_000) <= 2e-22
    assert Fr(9, 20) / Fr(11, 20) * Fr(1, 10**6) == Fr(9, 11_000_000)


def test_psi_design_value(orc):
    xi = 1e-3
    # a = 0 (flat on the left), b = xi
    psi = orc.psi(1.0, 1.0, 1.0, 1.0, 1.0 + xi)
    assert abs(psi - 0.45) < 1e-9
    assert orc.psi(1.0, 1.0, 1.0, 1.0, 1.0) == 1.0


def _step(n, H, s, bc=PB.BC_TRANSMISSIVE):
    P = PB.free_stream(n, rho=1.0, u=0.0, v=0.0, p=1.0, bc=bc, ny=12)
    rho = np.ones((12, n))
    rho[:, s + 1:] += H
    P.Q = PB.prim_to_state(rho, np.zeros_like(rho), np.zeros_like(rho), np.ones_like(rho))
    return P


@pytest.mark.parametrize("H", [1.0, 1e-2, 1e-3])
def test_step_footprint_nine_interfaces(orc, H):
    n, s = 40, 19
    P = _step(n, H, s)
    cfg = orc.make_cfg(P.nx, P.ny, *P.geometry())
    _, sx, sy, _ = orc.residual(cfg, P.Q, want_flags=True)
    # interface j+1/2 is stored at column j+1
    flagged = sorted(set(np.nonzero(sx == 0)[1] - 1))
    assert flagged == list(range(s - 4, s + 5))
    assert (sx == 0).all(axis=1).sum() == 0 and (sx[:, s - 3] == 0).all()
    assert (sy == 1).all()


def test_step_tiny_no_flags(orc):
    P = _step(40, 1e-4, 19)
    cfg = orc.make_cfg(P.nx, P.ny, *P.geometry())
    _, sx, sy, _ = orc.residual(cfg, P.Q, want_flags=True)
    assert (sx == 1).all() and (sy == 1).all()


def test_vortex_no_flags(orc):
    P = PB.vortex(64)
    cfg = orc.make_cfg(P.nx, P.ny, *P.geometry())
    _, sx, sy, nl = orc.residual(cfg, P.Q, want_flags=True)
    assert (sx == 1).all() and (sy == 1).all() and nl == 0


def test_riemann_flags_lie_on_the_discontinuities(orc):
    P = PB.riemann(64, seed=0)
    cfg = orc.make_cfg(P.nx, P.ny, *P.geometry())
    _, sx, sy, _ = orc.residual(cfg, P.Q, want_flags=True)
    # quadrant boundary at x = 0.8 lies between cells 50 and 51 (centres 0.79, 0.805)
    cols = set(np.nonzero(sx == 0)[1] - 1)
    assert cols <= set(range(50 - 4, 50 + 5))
    rows = set(np.nonzero(sy == 0)[0] - 1)
    assert rows <= set(range(50 - 4, 50 + 5))
    assert len(cols) > 0 and len(rows) > 0
