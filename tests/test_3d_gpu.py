"""The 3D extension (inviscid) vs the 3D CPU oracle, through the C ABI, in
each launch form: three line-sweep kernels, and the x and y sweeps fused over
15x15 tiles of each z plane (all lines at once, or 8 at a time) followed by
the z line sweep.

Bar as in 2D: interface flags bit-exact in all three directions; residuals
within 1e-12 of the flux-divergence scale; states after SSP-RK3 steps within
1e-12 relative; the time step bit-exact.  Cases: a smooth advected wave, the
eight-octant Riemann problem on ragged grids (several position tiles along
every direction, lines that do not fill the last workgroup) with both
boundary types, the smallest grid, the fourth-order subset, the paper's 64^3
Taylor-Green vortex at full size, trajectories, argument errors.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import relerr, report, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-12
FORMS = [gbr.GBR3_SWEEPS_LINES, gbr.GBR3_SWEEPS_XY_FUSED, gbr.GBR3_SWEEPS_XY_FUSED_HALF]


def ocfg3(P, order=7):
    return O.make_cfg3(P.nx, P.ny, P.nz, *P.geometry(), bc=P.bc, gamma=P.gamma, order=order)


def flux_scale3(P):
    Q = P.Q
    r = Q[0]
    u, v, w = Q[1] / r, Q[2] / r, Q[3] / r
    p = (P.gamma - 1) * (Q[4] - 0.5 * r * (u * u + v * v + w * w))
    m = np.zeros(5)
    for un, k in ((u, 1), (v, 2), (w, 3)):
        F = np.stack([r * un, r * un * u, r * un * v, r * un * w, un * (Q[4] + p)])
        F[k] += p
        m = np.maximum(m, np.abs(F).reshape(5, -1).max(1))
    d = min((P.hi[k] - P.lo[k]) / n for k, n in enumerate((P.nx, P.ny, P.nz)))
    return m / d


def check3(name, P, order=7, sweeps=gbr.GBR3_SWEEPS_LINES):
    from paper_2305_00762_amd.solver import Solver3
    torch = require_gpu()
    S = Solver3(P, export_flags=True, order=order, sweeps=sweeps)
    name = f"{name} form{sweeps}"
    R = S.residual()
    torch.cuda.synchronize()
    sx, sy, sz = S.flags()
    st = S.check()
    Rg = R.cpu().numpy()
    S.close()
    Ro, ox, oy, oz = O.residual3(ocfg3(P, order), P.Q, want_flags=True)
    scale = np.maximum(np.abs(Ro).reshape(5, -1).max(1), flux_scale3(P))
    e = np.abs(Rg - Ro).reshape(5, -1).max(1) / scale
    nflag = int((ox == 0).sum() + (oy == 0).sum() + (oz == 0).sum())
    report(name, relerr=e.max(), flagged=nflag,
           flag_mismatch=int((sx != ox).sum() + (sy != oy).sum() + (sz != oz).sum()))
    assert st == gbr.GBR_OK
    assert (sx == ox).all() and (sy == oy).all() and (sz == oz).all()
    assert (e <= TOL).all(), e
    return nflag


@pytest.mark.parametrize("sweeps", FORMS)
def test_advected_wave(sweeps):
    assert check3("3d advected wave 24^3", PB.advected_wave3d(24), sweeps=sweeps) == 0


@pytest.mark.parametrize("sweeps", FORMS)
@pytest.mark.parametrize("bc", [PB.BC_PERIODIC, PB.BC_TRANSMISSIVE])
@pytest.mark.parametrize("seed", [0, 1])
def test_riemann3d_ragged(seed, bc, sweeps):
    P = PB.riemann3d(40, seed=seed, ny=33, nz=20)
    P.bc = (bc,) * 3
    assert check3(f"3d riemann 40x33x20 s{seed} bc{bc}", P, sweeps=sweeps) > 0


@pytest.mark.parametrize("sweeps", FORMS)
def test_riemann3d_mixed_bc_and_order4(sweeps):
    P = PB.riemann3d(36, seed=3, ny=13, nz=45)
    P.bc = (PB.BC_TRANSMISSIVE, PB.BC_PERIODIC, PB.BC_TRANSMISSIVE)
    check3("3d riemann 36x13x45 mixed", P, sweeps=sweeps)
    check3("3d riemann 36x13x45 mixed order4", P, order=4, sweeps=sweeps)


@pytest.mark.parametrize("sweeps", FORMS)
def test_smallest_grid(sweeps):
    check3("3d riemann 12^3", PB.riemann3d(12, seed=4), sweeps=sweeps)


@pytest.mark.parametrize("sweeps", FORMS)
def test_taylor_green_64_full_size(sweeps):
    check3("3d taylor-green 64^3", PB.taylor_green3d(64), sweeps=sweeps)
    check3("3d taylor-green 64^3 order4", PB.taylor_green3d(64), order=4, sweeps=sweeps)


@pytest.mark.parametrize("sweeps", FORMS)
@pytest.mark.parametrize("order", [7, 4])
def test_trajectory_riemann3d(order, sweeps):
    from paper_2305_00762_amd.solver import Solver3
    torch = require_gpu()
    P = PB.riemann3d(32, seed=5, ny=24, nz=20)
    cfg = ocfg3(P, order)
    S = Solver3(P, order=order, sweeps=sweeps)
    Q = P.Q.copy()
    for k in range(10):
        do = O.step3(cfg, Q, P.cfl)
        S.step()
        if k == 0:
            torch.cuda.synchronize()
            assert float(S.dt.cpu()[0]) == do
    e = relerr(S.state().reshape(5, -1), Q.reshape(5, -1))
    report(f"3d riemann 32x24x20 10 steps order{order} form{sweeps}", relerr=e.max())
    assert (e <= TOL).all(), e
    assert S.check() == gbr.GBR_OK
    S.close()


def test_trajectory_taylor_green():
    from paper_2305_00762_amd.solver import Solver3
    require_gpu()
    P = PB.taylor_green3d(32)
    cfg = ocfg3(P)
    S = Solver3(P)
    Q = P.Q.copy()
    for _ in range(20):
        O.step3(cfg, Q, P.cfl)
        S.step()
    G = S.state()
    e = relerr(G.reshape(5, -1), Q.reshape(5, -1))
    ke = lambda q: 0.5 * ((q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]).mean()
    report("3d taylor-green 32^3 20 steps", relerr=e.max(), ke_gpu=ke(G), ke_oracle=ke(Q))
    assert (e <= TOL).all(), e
    S.close()


@pytest.mark.parametrize("sweeps", [gbr.GBR3_SWEEPS_LINES, gbr.GBR3_SWEEPS_XY_FUSED])
@pytest.mark.parametrize("case", ["riemann_ragged", "taylor_green"])
def test_stage_dt3_equals_two_pass(case, sweeps):
    """The 3D time step from the extrema the stage-3 z sweep reduces
    (gbr3_stage_dt) equals the two-pass reduction over the state it wrote and
    the oracle's time step, bit for bit; a second read without a stage-3 call
    in between is rejected."""
    from paper_2305_00762_amd.solver import Solver3
    torch = require_gpu()
    if case == "riemann_ragged":
        P = PB.riemann3d(40, seed=2, ny=33, nz=45)
        P.bc = (PB.BC_TRANSMISSIVE, PB.BC_PERIODIC, PB.BC_TRANSMISSIVE)
    else:
        P = PB.taylor_green3d(32)
    S = Solver3(P, sweeps=sweeps)
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_stage_dt(S.ctx, P.cfl, S.dt)             # no stage-3 output yet
    fused = torch.zeros(1, dtype=torch.float64, device="cuda")
    cfg = ocfg3(P)
    bits = lambda t: t.cpu().numpy().view(np.uint64)[0]
    for k in range(3):
        S.step()
        gbr.gbr3_stage_dt(S.ctx, P.cfl, fused)
        gbr.gbr3_compute_dt(S.ctx, S.Q, P.cfl, S.dt)
        torch.cuda.synchronize()
        o = np.float64(O.dt3(cfg, S.state(), P.cfl)).view(np.uint64)
        report(f"3d stage dt {case} form{sweeps} step {k}", fused=float(fused.item()),
               two_pass=float(S.dt.item()))
        assert bits(fused) == bits(S.dt) == o
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_stage_dt(S.ctx, P.cfl, fused)            # already read
    assert S.check() == gbr.GBR_OK
    S.close()


def test_trajectory_fused_dt3_bit_identical():
    """Steps taken with the fused time step equal, bit for bit, steps taken
    with the two-pass reduction."""
    from paper_2305_00762_amd.solver import Solver3
    require_gpu()
    P = PB.riemann3d(32, seed=5, ny=24, nz=20)
    A, B = Solver3(P), Solver3(P, fused_dt=True)
    for _ in range(5):
        A.step()
        B.step()
    qa, qb = A.state(), B.state()
    assert (qa.view(np.uint64) == qb.view(np.uint64)).all()
    A.close()
    B.close()


@pytest.mark.parametrize("order", [7, 4])
def test_forms_agree(order):
    """The fused forms against the line sweeps on the same state: interface
    flags identical, residuals equal to rounding (the cell pressure is formed
    with the squared velocities summed in another order)."""
    from paper_2305_00762_amd.solver import Solver3
    torch = require_gpu()
    P = PB.riemann3d(47, seed=6, ny=31, nz=17)
    out = []
    for f in FORMS:
        S = Solver3(P, export_flags=True, order=order, sweeps=f)
        R = S.residual()
        torch.cuda.synchronize()
        out.append((R.cpu().numpy(), S.flags()))
        S.close()
    R0, f0 = out[0]
    scale = np.maximum(np.abs(R0).reshape(5, -1).max(1), flux_scale3(P))
    for (R, fl), f in zip(out[1:], FORMS[1:]):
        e = np.abs(R - R0).reshape(5, -1).max(1) / scale
        report(f"3d forms {f} vs lines order{order}", relerr=e.max())
        assert all((a == b).all() for a, b in zip(fl, f0))
        assert (e <= 1e-13).all(), e


def test_argument_errors():
    torch = require_gpu()
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_init(11, 16, 16, 1.4)
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_init(16, 16, 16, 1.0)
    ctx = gbr.gbr3_init(16, 16, 16, 1.4)
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_set_order(ctx, 5)
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_set_sweeps(ctx, 3)
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_set_geometry(ctx, 0, 1, 0, 1, 1, 0, 0, 0, 0)
    Q = torch.zeros((5, 16, 16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_residual(ctx, Q, Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(gbr.GbrError):
        gbr.gbr3_rk_stage(ctx, 4, dt, Q, Q, torch.empty_like(Q))
    gbr.gbr3_destroy(ctx)
