"""Boundaries by side (walls, no-slip walls, inflow, moving segments) and the
shock-stable HLLC on the GPU vs the CPU oracle, through the C ABI.

Same bar as the periodic / transmissive paths: detector flags bit-exact;
residuals within 1e-12 of the flux-divergence scale; states after SSP-RK3
steps within 1e-12 relative.  Cases: each wall kind on each axis, all four
sides no-slip with viscosity (corners), inflow and transmissive sides, a side
split into two segments, a split moving with the device clock, both variable
sets, the fourth-order GRB, both tile shapes, ragged and smallest grids; the
double Mach reflection and the viscous shock tube as trajectories and at full
size; the option checks.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import gpu_residual, ocfg, relerr, report, require_gpu, res_err

pytestmark = pytest.mark.gpu
TOL = 1e-12
INF = float("inf")


def one(kind, state=None):
    return (kind, state, kind, state, INF, 0.0)


def with_sides(P, sides, riemann=0):
    P.sides = sides
    P.riemann = riemann
    return P


def gpu_residual_t(P, t, **kw):
    """GPU residual with the device clock at t."""
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    S = Solver(P, export_flags=True, **kw)
    gbr.gbr_set_time(S.ctx, t)
    R = S.residual()
    torch.cuda.synchronize()
    sx, sy = S.flags()
    st = S.check()
    out = R.cpu().numpy()
    S.close()
    return out, sx, sy, st


def check(name, P, t=0.0, tiling=None, **kw):
    if t == 0.0:
        R, sx, sy, st = gpu_residual(P, tiling=tiling, **kw)
    else:
        assert tiling is None
        R, sx, sy, st = gpu_residual_t(P, t, **kw)
    okw = {k: v for k, v in kw.items() if k in ("recon", "order")}
    Ro, sxo, syo, nlim = O.residual(ocfg(P, t=t, **okw), P.Q, want_flags=True)
    e = res_err(R, Ro, P)
    nflag = int((sxo == 0).sum() + (syo == 0).sum())
    report(name, relerr=e.max(), flagged=nflag,
           flag_mismatch=int((sx != sxo).sum() + (sy != syo).sum()))
    assert st == 0
    assert (sx == sxo).all() and (sy == syo).all()
    assert (e <= TOL).all(), e
    return nflag


R1 = (1.7, 0.6, -0.2, 2.1)
R2 = (0.4, -0.3, 0.5, 0.6)


@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("tiling", [0, 1])
@pytest.mark.parametrize("kind", [PB.BC_REFLECT, PB.BC_NOSLIP])
def test_wall_x(kind, tiling, recon):
    P = PB.riemann(45, seed=11, ny=29)
    with_sides(P, [one(kind), one(kind), one(PB.BC_PERIODIC), one(PB.BC_PERIODIC)])
    check(f"wall x k{kind} t{tiling} r{recon}", P, tiling=tiling, recon=recon)


@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("kind", [PB.BC_REFLECT, PB.BC_NOSLIP])
def test_wall_y_viscous(kind, recon):
    P = PB.riemann(40, seed=12, ny=33)
    P.mu = 2e-3
    with_sides(P, [one(PB.BC_PERIODIC), one(PB.BC_PERIODIC), one(kind), one(kind)])
    check(f"wall y k{kind} viscous r{recon}", P, recon=recon)


@pytest.mark.parametrize("tiling", [0, 1])
def test_noslip_box_viscous_corners(tiling):
    P = PB.viscous_shock_tube(64)
    P.sides = [one(PB.BC_NOSLIP)] * 4
    for recon in (0, 1):
        check(f"noslip box 64x32 t{tiling} r{recon}", P, tiling=tiling, recon=recon)


def test_inflow_transmissive_and_segments():
    P = PB.riemann(50, seed=13, ny=36)
    P.mu = 1e-3
    with_sides(P, [one(PB.BC_INFLOW, R1), one(PB.BC_TRANSMISSIVE),
                   (PB.BC_INFLOW, R2, PB.BC_REFLECT, None, 0.45, 0.0),
                   (PB.BC_NOSLIP, None, PB.BC_INFLOW, R1, 0.3, 0.0)])
    for recon in (0, 1):
        check(f"inflow+segments r{recon}", P, recon=recon)
    check("inflow+segments order4", P, order=4)


@pytest.mark.parametrize("t", [0.0, 0.013, 0.05])
def test_moving_split_device_clock(t):
    P = PB.riemann(48, seed=14, ny=24)
    with_sides(P, [one(PB.BC_TRANSMISSIVE), one(PB.BC_TRANSMISSIVE), one(PB.BC_REFLECT),
                   (PB.BC_INFLOW, R1, PB.BC_INFLOW, R2, 0.1, 9.0)])
    check(f"moving split t={t}", P, t=t)


@pytest.mark.parametrize("n", [12, 13])
def test_smallest_grids_walls(n):
    P = PB.riemann(n, seed=7, ny=12 if n != 13 else 17)
    P.mu = 1e-3
    with_sides(P, [one(PB.BC_NOSLIP), one(PB.BC_INFLOW, R1), one(PB.BC_REFLECT),
                   one(PB.BC_NOSLIP)])
    for recon in (0, 1):
        check(f"walls {n} r{recon}", P, recon=recon)


@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("tiling", [0, 1])
def test_shock_stable_hllc(tiling, recon):
    P = PB.double_mach(96)
    check(f"double mach 96x24 ss-hllc t{tiling} r{recon}", P, tiling=tiling, recon=recon)
    # the low-Mach branch is exercised: slow flow with a pressure jump
    Q = PB.riemann(40, seed=15, states=[(1.0, 0.01, 0.0, 1.0), (1.0, 0.02, 0.0, 1.1),
                                        (0.8, -0.01, 0.01, 0.9), (1.2, 0.0, 0.0, 1.0)])
    with_sides(Q, [one(PB.BC_TRANSMISSIVE)] * 4, riemann=1)
    check(f"low-mach ss-hllc t{tiling} r{recon}", Q, tiling=tiling, recon=recon)


def _trajectory(name, P, steps, recon=0):
    from paper_2305_00762_amd.solver import Solver
    require_gpu()
    cfg = ocfg(P, recon=recon)
    S = Solver(P, recon=recon)
    Q = P.Q.copy()
    for _ in range(steps):
        O.step(cfg, Q, P.cfl)
        S.step()
    e = relerr(S.state(), Q)
    tg = S.time()
    report(name, relerr=e.max(), t_gpu=tg, t_oracle=cfg.t)
    assert (e <= TOL).all(), e
    assert abs(tg - cfg.t) <= 1e-14 * cfg.t
    assert S.check() == gbr.GBR_OK
    S.close()


@pytest.mark.parametrize("recon", [0, 1])
def test_double_mach_trajectory(recon):
    _trajectory(f"double mach 128x32 30 steps r{recon}", PB.double_mach(128), 30, recon)


@pytest.mark.parametrize("recon", [0, 1])
def test_viscous_shock_tube_trajectory(recon):
    _trajectory(f"viscous shock tube 96x48 30 steps r{recon}", PB.viscous_shock_tube(96), 30,
                recon)


def test_double_mach_full_size():
    check("double mach 1024x256", PB.double_mach(1024))


def test_viscous_shock_tube_full_size():
    check("viscous shock tube 1280x640", PB.viscous_shock_tube(1280))


def test_options_and_clock():
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    P = PB.double_mach(64)
    S = Solver(P)
    with pytest.raises(gbr.GbrError):         # FP32 bulk with a side table
        gbr.gbr_set_scheme(S.ctx, 0, gbr.GBR_MP_FLAGGED, gbr.GBR_PREC_FP32_BULK, 0)
    with pytest.raises(gbr.GbrError):         # fourth order with the shock-stable HLLC
        gbr.gbr_set_order(S.ctx, 4)
    bad = [one(PB.BC_PERIODIC), one(PB.BC_TRANSMISSIVE), one(PB.BC_REFLECT), one(PB.BC_REFLECT)]
    with pytest.raises(gbr.GbrError):         # periodic on one side only
        gbr.gbr_set_sides(S.ctx, bad)
    with pytest.raises(gbr.GbrError):         # unknown kind
        gbr.gbr_set_sides(S.ctx, [one(7)] * 4)
    with pytest.raises(gbr.GbrError):         # non-physical inflow state
        gbr.gbr_set_sides(S.ctx, [one(PB.BC_INFLOW, (-1.0, 0, 0, 1.0))] * 4)
    gbr.gbr_set_time(S.ctx, 0.25)
    assert gbr.gbr_get_time(S.ctx) == 0.25
    dt = torch.tensor([0.125], dtype=torch.float64, device="cuda")
    gbr.gbr_advance_time(S.ctx, dt)
    torch.cuda.synchronize()
    assert gbr.gbr_get_time(S.ctx) == 0.375
    gbr.gbr_set_sides(S.ctx, None)            # back to per-direction types
    gbr.gbr_set_riemann(S.ctx, gbr.GBR_RIEMANN_HLLC)
    gbr.gbr_set_scheme(S.ctx, 0, gbr.GBR_MP_FLAGGED, gbr.GBR_PREC_FP32_BULK, 0)
    with pytest.raises(gbr.GbrError):         # side table in FP32 bulk
        gbr.gbr_set_sides(S.ctx, P.sides)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_set_riemann(S.ctx, gbr.GBR_RIEMANN_HLLC_SS)
    S.close()
