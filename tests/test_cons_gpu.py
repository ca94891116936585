"""MEG7-cons (conservative-variable reconstruction, Secs. 2.2-2.3, Table 2) on
the GPU vs the CPU oracle with recon = 1, through the C ABI.

Same bar as MEG7-prim: detector flags bit-exact; residuals within 1e-12 of
the flux-divergence scale max|F|/dx per variable; states after SSP-RK3 steps
within 1e-12 relative to max|Q|.  Cases: the smooth vortex, ragged Riemann
grids with the shock branch active, both boundary types, the smallest grids,
the viscous shear layer (chain-rule velocity gradients), an all-flagged
noise field, both tile shapes that carry the scheme, the full 1024^2 Riemann
workload, and the scheme options the library rejects.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import gpu_residual, ocfg, relerr, report, require_gpu, res_err

pytestmark = pytest.mark.gpu
TOL = 1e-12
CONS = gbr.GBR_RECON_CONS


def check(name, P, tiling=None):
    R, sx, sy, st = gpu_residual(P, tiling=tiling, recon=CONS)
    Ro, sxo, syo, nlim = O.residual(ocfg(P, recon=1), P.Q, want_flags=True)
    e = res_err(R, Ro, P)
    nflag = int((sxo == 0).sum() + (syo == 0).sum())
    report(name, relerr=e.max(), flagged=nflag, mp_limited=nlim,
           flag_mismatch=int((sx != sxo).sum() + (sy != syo).sum()))
    assert st == 0
    assert (sx == sxo).all() and (sy == syo).all()
    assert (e <= TOL).all(), e
    return nflag


@pytest.mark.parametrize("tiling", [0, 1])
def test_cons_vortex(tiling):
    assert check(f"cons vortex64 t{tiling}", PB.vortex(64), tiling) == 0


@pytest.mark.parametrize("tiling", [0, 1])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cons_riemann_ragged(seed, tiling):
    P = PB.riemann(100, seed=seed, ny=77)
    assert check(f"cons riemann100x77 s{seed} t{tiling}", P, tiling) > 0


@pytest.mark.parametrize("n", [12, 13, 32])
def test_cons_smallest_grids(n):
    for bc in (PB.BC_PERIODIC, PB.BC_TRANSMISSIVE):
        P = PB.riemann(n, seed=7, ny=12 if n != 13 else 17)
        P.bc_x = P.bc_y = bc
        check(f"cons riemann {n} bc{bc}", P)


@pytest.mark.parametrize("tiling", [0, 1])
def test_cons_shear_viscous(tiling):
    P = PB.shear(96, seed=0, ny=80)
    P.mu = 2e-3
    check(f"cons shear96x80 mu=2e-3 t{tiling}", P, tiling)


def test_cons_noise_all_flagged():
    rng = np.random.default_rng(11)
    n = 48
    rho = rng.uniform(0.5, 1.5, (n, n))
    u, v = rng.uniform(-0.5, 0.5, (2, n, n))
    p = rng.uniform(0.5, 1.5, (n, n))
    P = PB.free_stream(n)
    P.Q = PB.prim_to_state(rho, u, v, p)
    P.mu = 1e-3
    check("cons noise48 viscous", P)


def test_cons_free_stream_exact_zero():
    for bc in (PB.BC_PERIODIC, PB.BC_TRANSMISSIVE):
        P = PB.free_stream(40, bc=bc, ny=33, mu=1e-3)
        R, sx, sy, st = gpu_residual(P, recon=CONS)
        assert (R == 0.0).all() and sx.all() and sy.all()


def test_cons_riemann_1024_full_size():
    """Full-size residual of the 1024^2 Riemann workload under MEG7-cons."""
    check("cons riemann1024", PB.riemann(1024, seed=0))


def test_cons_trajectory_riemann():
    """20 SSP-RK3 steps of a 128^2 Riemann problem (shock branch active)."""
    from paper_2305_00762_amd.solver import Solver
    require_gpu()
    P = PB.riemann(128, seed=0)
    cfg = ocfg(P, recon=1)
    S = Solver(P, recon=CONS)
    Q = P.Q.copy()
    for _ in range(20):
        O.step(cfg, Q, P.cfl)
        S.step()
    e = relerr(S.state(), Q)
    report("cons riemann128 20 steps", relerr=e.max())
    assert (e <= TOL).all(), e
    assert S.check() == gbr.GBR_OK
    S.close()


def test_cons_trajectory_shear_viscous():
    from paper_2305_00762_amd.solver import Solver
    require_gpu()
    P = PB.shear(64, seed=1)
    P.mu = 1e-3
    cfg = ocfg(P, recon=1)
    S = Solver(P, recon=CONS)
    Q = P.Q.copy()
    for _ in range(5):
        O.step(cfg, Q, P.cfl)
        S.step()
    e = relerr(S.state(), Q)
    report("cons shear64 5 steps", relerr=e.max())
    assert (e <= TOL).all(), e
    S.close()


def test_cons_differs_from_prim_and_options():
    """The two schemes give different residuals on a Riemann problem; MEG7-cons
    is rejected in FP32 bulk and with the learned detector, leaving the scheme
    unchanged; tile shapes without a MEG7-cons build fall back to 31x15."""
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    P = PB.riemann(64, seed=5)
    Rp = gpu_residual(P)[0]
    Rc = gpu_residual(P, recon=CONS)[0]
    assert not np.array_equal(Rp, Rc)
    S = Solver(P, recon=CONS)
    for prec, det in ((gbr.GBR_PREC_FP32_BULK, gbr.GBR_DET_PLAIN),
                      (gbr.GBR_PREC_FP64, gbr.GBR_DET_MLP)):
        with pytest.raises(gbr.GbrError):
            gbr.gbr_set_scheme(S.ctx, CONS, gbr.GBR_MP_FLAGGED, prec, det)
    for t in range(gbr.gbr_tiling_count()):
        gbr.gbr_set_tiling(S.ctx, t)
        v, tx, ty = gbr.gbr_get_tiling(S.ctx)
        assert (tx, ty) in ((31, 15), (15, 15))
        R = S.residual()
        torch.cuda.synchronize()
        assert res_err(R.cpu().numpy(), Rc, P).max() <= TOL
    S.close()
