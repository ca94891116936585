"""GPU FP64 path vs the CPU oracle, through the C ABI.

Bar: detector flags bit-exact; states within 1e-12 relative to max|Q| per
conserved variable; residuals within 1e-12 relative to the flux-divergence
scale max|F|/dx per variable (a residual is a difference of O(|F|) fluxes over
dx, so that is the scale of its rounding error); time step bit-exact.  Cases span several
31x15 tiles with ragged tails, both boundary types, the shock branch, the
viscous terms, the smallest grid, and the full workload sizes (1024^2
Riemann, 2048^2 shear layer) in the launch configuration the bench times.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import gpu_residual, ocfg, relerr, report, require_gpu, res_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


def check_residual(name, P, tiling=None):
    R, sx, sy, st = gpu_residual(P, tiling=tiling)
    Ro, sxo, syo, nlim = O.residual(ocfg(P), P.Q, want_flags=True)
    e = res_err(R, Ro, P)
    nflag = int((sxo == 0).sum() + (syo == 0).sum())
    report(name, relerr=e.max(), flagged=nflag, mp_limited=nlim,
           flag_mismatch=int((sx != sxo).sum() + (sy != syo).sum()))
    assert st == 0
    assert (sx == sxo).all() and (sy == syo).all()
    assert (e <= TOL).all(), e
    return nflag


def test_vortex_64():
    assert check_residual("vortex64", PB.vortex(64)) == 0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_riemann_ragged(seed):
    P = PB.riemann(100, seed=seed, ny=77)
    assert check_residual(f"riemann100x77 s{seed}", P) > 0


def test_riemann_paper_states_periodic():
    P = PB.riemann(64, states=PB.paper_riemann_states(), ny=70)
    P.bc_x = P.bc_y = PB.BC_PERIODIC
    check_residual("riemann-paper 64x70 periodic", P)


@pytest.mark.parametrize("n", [12, 13, 31, 32])
def test_smallest_grids(n):
    for bc in (PB.BC_PERIODIC, PB.BC_TRANSMISSIVE):
        P = PB.riemann(n, seed=7, ny=12 if n != 13 else 17)
        P.bc_x = P.bc_y = bc
        check_residual(f"riemann {n} bc{bc}", P)


def test_shear_viscous():
    P = PB.shear(96, seed=0, ny=80)
    P.mu = 2e-3        # strong viscosity so the viscous flux matters at this size
    check_residual("shear96x80 mu=2e-3", P)


def test_noise_all_flagged():
    rng = np.random.default_rng(11)
    n = 48
    rho = rng.uniform(0.5, 1.5, (n, n))
    u, v = rng.uniform(-0.5, 0.5, (2, n, n))
    p = rng.uniform(0.5, 1.5, (n, n))
    P = PB.free_stream(n)
    P.Q = PB.prim_to_state(rho, u, v, p)
    P.mu = 1e-3
    check_residual("noise48 viscous", P)


def _noise(rng, n, ny):
    rho = rng.uniform(0.5, 1.5, (ny, n))
    u, v = rng.uniform(-0.5, 0.5, (2, ny, n))
    p = rng.uniform(0.5, 1.5, (ny, n))
    P = PB.free_stream(n, ny=ny)
    P.Q = PB.prim_to_state(rho, u, v, p)
    return P


def check_residual_kw(name, P, tiling, **kw):
    R, sx, sy, st = gpu_residual(P, tiling=tiling, **kw)
    okw = {k: v for k, v in kw.items() if k in ("recon", "order")}
    Ro, sxo, syo, nlim = O.residual(ocfg(P, **okw), P.Q, want_flags=True)
    e = res_err(R, Ro, P)
    report(name, relerr=e.max(), flagged=int((sxo == 0).sum() + (syo == 0).sum()),
           flag_mismatch=int((sx != sxo).sum() + (sy != syo).sum()))
    assert st == 0
    assert (sx == sxo).all() and (sy == syo).all()
    assert (e <= TOL).all(), e


@pytest.mark.parametrize("order", [7, 4])
@pytest.mark.parametrize("tiling", [0, 1, 2, 3])
def test_noise_all_flagged_every_tiling(tiling, order):
    # every interface flagged, so the characteristic branch runs at the first
    # and last interface of every line of every tile: with the edge-jump form
    # its gradients there reach the outermost edges (the first of them formed
    # from the tile); inviscid and viscous (T as an edge field), periodic and
    # with walls and the shock-stable HLLC (the side table, ghost rules)
    rng = np.random.default_rng(21 + order)
    for n, ny, mu in ((48, 48, 0.0), (50, 37, 1e-3)):
        P = _noise(rng, n, ny)
        P.mu = mu
        check_residual_kw(f"noise{n}x{ny} mu={mu} t{tiling} o{order}", P, tiling, order=order)
    P = _noise(rng, 45, 34)
    P.sides = [(PB.BC_REFLECT, None, PB.BC_REFLECT, None, float("inf"), 0.0),
               (PB.BC_TRANSMISSIVE, None, PB.BC_TRANSMISSIVE, None, float("inf"), 0.0),
               (PB.BC_NOSLIP, None, PB.BC_NOSLIP, None, float("inf"), 0.0),
               (PB.BC_TRANSMISSIVE, None, PB.BC_TRANSMISSIVE, None, float("inf"), 0.0)]
    P.riemann = 1 if order == 7 else 0      # the shock-stable HLLC is built for order 7
    P.mu = 1e-3
    check_residual_kw(f"noise45x34 walls riemann{P.riemann} viscous t{tiling} o{order}", P,
                      tiling, order=order)


def test_free_stream_exact_zero():
    for bc in (PB.BC_PERIODIC, PB.BC_TRANSMISSIVE):
        P = PB.free_stream(40, bc=bc, ny=33, mu=1e-3)
        R, sx, sy, st = gpu_residual(P)
        assert (R == 0.0).all() and sx.all() and sy.all()


def test_riemann_1024_full_size():
    """Full-size residual of the 1024^2 Riemann workload."""
    check_residual("riemann1024", PB.riemann(1024, seed=0))


def test_shear_2048_full_size():
    """Full-size residual of the 2048^2 viscous shear layer."""
    check_residual("shear2048", PB.shear(2048, seed=0))


def _dt_gpu(P, cfl):
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    S = Solver(P)
    d = S.compute_dt(cfl)
    torch.cuda.synchronize()
    v = float(d.cpu()[0])
    S.close()
    return v


@pytest.mark.parametrize("fam", ["vortex", "riemann", "shear"])
def test_dt_bit_exact(fam):
    P = PB.make(fam, 200, seed=3) if fam != "vortex" else PB.vortex(200)
    d = _dt_gpu(P, P.cfl)
    do = O.dt(ocfg(P), P.Q, P.cfl)
    report(f"dt {fam}", gpu=d, oracle=do)
    assert d == do


def test_rk_stages_and_trajectory_vortex():
    """Config-1 workload: 64^2 vortex, CFL 0.5, 10 SSP-RK3 steps."""
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    P = PB.vortex(64, cfl=0.5)
    cfg = ocfg(P)
    S = Solver(P)
    Q = P.Q.copy()
    for step in range(10):
        dto = O.dt(cfg, Q, 0.5)
        Q1 = O.rk_stage(cfg, 1, dto, Q, Q)
        Q2 = O.rk_stage(cfg, 2, dto, Q, Q1)
        Q = O.rk_stage(cfg, 3, dto, Q, Q2)
        S.step(0.5)
        if step == 0:
            torch.cuda.synchronize()
            assert float(S.dt.cpu()[0]) == dto
    G = S.state()
    e = relerr(G, Q)
    report("vortex64 10 steps", relerr=e.max())
    assert (e <= TOL).all(), e
    assert S.check() == 0
    S.close()


def test_trajectory_riemann_shock_branch():
    """30 steps of a 128^2 seeded Riemann problem: the shock branch is active."""
    from paper_2305_00762_amd.solver import Solver
    require_gpu()
    P = PB.riemann(128, seed=0)
    cfg = ocfg(P)
    S = Solver(P, export_flags=True)
    Q = P.Q.copy()
    for _ in range(30):
        O.step(cfg, Q, P.cfl)
        S.step()
    G = S.state()
    e = relerr(G, Q)
    report("riemann128 30 steps", relerr=e.max())
    assert (e <= TOL).all(), e
    S.close()


@pytest.mark.parametrize("stage", [1, 2, 3])
def test_single_stage_viscous(stage):
    from paper_2305_00762_amd.solver import Solver
    from paper_2305_00762_amd import gbr
    torch = require_gpu()
    P = PB.shear(64, seed=1, ny=50)
    P.mu = 1e-3
    cfg = ocfg(P)
    rng = np.random.default_rng(stage)
    Qn = P.Q
    Qk = P.Q * (1 + 1e-3 * rng.standard_normal(P.Q.shape))
    dt = 1.7e-3
    if stage == 1:
        Qk = Qn
    ref = O.rk_stage(cfg, stage, dt, Qn, Qk)
    S = Solver(P)
    tQn = torch.from_numpy(Qn).cuda()
    tQk = torch.from_numpy(np.ascontiguousarray(Qk)).cuda() if stage > 1 else tQn
    out = torch.empty_like(tQn)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    gbr.gbr_rk_stage(S.ctx, stage, dtd, tQn, tQk, out)
    torch.cuda.synchronize()
    e = relerr(out.cpu().numpy(), ref)
    report(f"stage{stage} viscous", relerr=e.max())
    assert (e <= TOL).all(), e
    S.close()


def test_conservation_gpu():
    P = PB.vortex(96)
    R, *_ = gpu_residual(P)
    s = np.abs(R.sum(axis=(1, 2)))
    assert (s <= 1e-12 * R.size * (np.abs(R).max(axis=(1, 2)) + 1)).all()


def test_bad_state_reported():
    from paper_2305_00762_amd.solver import Solver
    from paper_2305_00762_amd import gbr
    torch = require_gpu()
    P = PB.vortex(32)
    S = Solver(P)
    assert S.check() == gbr.GBR_OK
    Q = P.Q.copy()
    Q[0, 5, 7] = -1.0
    S.set_state(Q)
    S.residual()
    assert S.check() == gbr.GBR_ESTATE
    assert S.check() == gbr.GBR_OK      # cleared
    Q = P.Q.copy()
    Q[3, 20, 3] = np.nan
    S.set_state(Q)
    S.compute_dt(0.5)
    assert S.check() == gbr.GBR_ESTATE
    S.close()


def test_argument_errors():
    from paper_2305_00762_amd import gbr
    require_gpu()
    with pytest.raises(gbr.GbrError):
        gbr.gbr_init(11, 40, 1.4, 0.0, 0.72)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_init(40, 40, 1.0, 0.0, 0.72)
    ctx = gbr.gbr_init(40, 40, 1.4, 0.0, 0.72)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_set_geometry(ctx, 1, 0, 0, 1, 0, 0)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_set_geometry(ctx, 0, 1, 0, 1, 5, 0)
    import torch
    Q = torch.zeros(4, 40, 40, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(gbr.GbrError):
        gbr.gbr_rk_stage(ctx, 4, dt, Q, Q, torch.empty_like(Q))
    with pytest.raises(gbr.GbrError):
        gbr.gbr_rk_stage(ctx, 2, dt, Q, Q, Q)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_residual(ctx, Q, Q)
    gbr.gbr_destroy(ctx)


@pytest.mark.parametrize("tiling", [0, 1, 2])
def test_tile_variants(tiling):
    """Every compiled tile shape gives the same flags and residual."""
    for P in (PB.riemann(100, seed=1, ny=77), PB.vortex(40)):
        check_residual(f"tiling{tiling} {P.family}", P, tiling=tiling)
    P = PB.shear(70, seed=2, ny=45)
    P.mu = 2e-3
    check_residual(f"tiling{tiling} viscous", P, tiling=tiling)
    P = PB.riemann(12, seed=4, ny=12)
    P.bc_x = P.bc_y = PB.BC_PERIODIC
    check_residual(f"tiling{tiling} 12x12 periodic", P, tiling=tiling)


def test_autotune_picks_a_variant():
    from paper_2305_00762_amd import gbr
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    P = PB.riemann(256, seed=0)
    S = Solver(P)
    v, tx, ty = gbr.gbr_autotune(S.ctx, S.Q, 2)
    assert 0 <= v < gbr.gbr_tiling_count() and tx > 0 and ty > 0
    report("autotune riemann256", variant=v, tile=f"{tx}x{ty}")
    R = S.residual()
    torch.cuda.synchronize()
    Ro = O.residual(ocfg(P), P.Q)
    assert (res_err(R.cpu().numpy(), Ro, P) <= TOL).all()
    S.close()


def test_positivity_fallback_trajectory():
    """Seeded Riemann problem whose interacting discontinuities make the
    characteristic MP states unphysical at step 21: the first-order fallback
    (both sides) keeps it running, and GPU and oracle agree through it."""
    from paper_2305_00762_amd.solver import Solver
    require_gpu()
    P = PB.riemann(128, seed=1008)
    cfg = ocfg(P)
    S = Solver(P)
    Q = P.Q.copy()
    for _ in range(25):
        O.step(cfg, Q, P.cfl)
        S.step()
    G = S.state()
    assert np.isfinite(Q).all() and S.check() == 0
    e = relerr(G, Q)
    report("riemann128 seed1008 25 steps", relerr=e.max())
    assert (e <= TOL).all(), e
    S.close()


def test_timing_hook_counts_launches():
    """gbr_timing records one flag-map/stage event triple per stage call."""
    torch = require_gpu()
    from paper_2305_00762_amd.solver import Solver
    P = PB.riemann(64, seed=2, ny=48)
    S = Solver(P)
    gbr.gbr_timing(S.ctx, True)
    S.step()
    S.step()
    torch.cuda.synchronize()
    det_ms, stage_ms, n = gbr.gbr_timing_read(S.ctx)
    assert n == 6 and stage_ms > 0.0 and det_ms >= 0.0
    assert gbr.gbr_timing_read(S.ctx)[2] == 0
    gbr.gbr_timing(S.ctx, False)
    S.step()
    assert gbr.gbr_timing_read(S.ctx)[2] == 0
    S.close()
