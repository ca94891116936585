"""Temporal order of the SSP Runge-Kutta scheme (Sec. 2.5, eq. rk) in the
oracle: at a fixed grid the semi-discrete operator is fixed, so the
difference between runs with time steps dt and a much finer reference step
is the time-integration error alone.  Third order means that halving dt
divides it by 8.  The detector is forced to the smooth branch so that the
operator is the same (and smooth) in every run.

A dropped or mis-weighted stage coefficient makes the scheme first or
second order and fails the bounds below; so does a stage that evaluates its
residual on the wrong state.
"""
import math

import numpy as np

from paper_2305_00762_amd import problems as PB


def run(orc, cfg, Q0, dt, T):
    Q = Q0.copy()
    for _ in range(int(round(T / dt))):
        Q1 = orc.rk_stage(cfg, 1, dt, Q, Q)
        Q2 = orc.rk_stage(cfg, 2, dt, Q, Q1)
        Q = orc.rk_stage(cfg, 3, dt, Q, Q2)
    return Q


def test_ssp_rk3_temporal_order(orc):
    P = PB.vortex(32)
    cfg = orc.make_cfg(P.nx, P.ny, *P.geometry(), force_sigma=1)
    T = 0.48
    ref = run(orc, cfg, P.Q, T / 192, T)
    errs = [np.abs(run(orc, cfg, P.Q, T / m, T) - ref).mean() for m in (6, 12, 24)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(2.8 < o < 3.2 for o in orders), (errs, orders)
