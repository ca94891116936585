"""FP32-bulk path (FP32 reconstruction/fluxes on local jumps, FP64 state,
stage update and flux differencing) vs the FP64 CPU oracle.

Bars (derived from the arithmetic): detector flags are the FP64 flags, bit
for bit; a residual differs from the oracle by at most 1e-6 of the
flux-divergence scale max|F|/dx (FP32 unit roundoff 6e-8 times the local
variation that the FP32 part carries, times a modest stencil gain);
conservation and free-stream preservation hold as in FP64; over a run the L1
density error against the oracle stays at or below 1e-6.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import gpu_residual, ocfg, relerr, report, require_gpu, res_err

pytestmark = pytest.mark.gpu
FP32 = gbr.GBR_PREC_FP32_BULK
RES_TOL = 1e-6


def check(name, P, tiling=None):
    R, sx, sy, st = gpu_residual(P, precision=FP32, tiling=tiling)
    Ro, sxo, syo, _ = O.residual(ocfg(P), P.Q, want_flags=True)
    e = res_err(R, Ro, P)
    report(name, res_err=e.max(), flag_mismatch=int((sx != sxo).sum() + (sy != syo).sum()))
    assert st == 0
    assert (sx == sxo).all() and (sy == syo).all()
    assert (e <= RES_TOL).all(), e
    return e


@pytest.mark.parametrize("tiling", [0, 1, 2, 3])
def test_residual_variants(tiling):
    check(f"f32 vortex64 t{tiling}", PB.vortex(64), tiling)
    check(f"f32 riemann100x77 t{tiling}", PB.riemann(100, seed=2, ny=77), tiling)
    P = PB.shear(96, seed=0, ny=80)
    P.mu = 2e-3
    check(f"f32 shear96 viscous t{tiling}", P, tiling)


@pytest.mark.parametrize("tiling", [0, 1, 2, 3])
def test_noise_all_flagged(tiling):
    # every interface flagged: the characteristic branch runs at every line
    # end of every tile, where its gradients reach one edge past the first
    # pass's range (the edge the flagged interface stores itself)
    rng = np.random.default_rng(12)
    for n, ny, mu in ((48, 48, 0.0), (50, 37, 1e-3)):
        rho = rng.uniform(0.5, 1.5, (ny, n))
        u, v = rng.uniform(-0.5, 0.5, (2, ny, n))
        p = rng.uniform(0.5, 1.5, (ny, n))
        P = PB.free_stream(n, ny=ny)
        P.Q = PB.prim_to_state(rho, u, v, p)
        P.mu = mu
        check(f"f32 noise{n}x{ny} mu={mu} t{tiling}", P, tiling)


def test_residual_full_sizes():
    check("f32 riemann1024", PB.riemann(1024, seed=0))
    check("f32 shear2048", PB.shear(2048, seed=0))


def test_free_stream_and_conservation():
    for bc in (PB.BC_PERIODIC, PB.BC_TRANSMISSIVE):
        P = PB.free_stream(40, bc=bc, ny=33, mu=1e-3)
        R, *_ = gpu_residual(P, precision=FP32)
        assert (R == 0.0).all()
    P = PB.vortex(96)
    R, *_ = gpu_residual(P, precision=FP32)
    s = np.abs(R.sum(axis=(1, 2)))
    assert (s <= 1e-12 * R.size * (np.abs(R).max(axis=(1, 2)) + 1)).all()


def run_pair(P, steps):
    from paper_2305_00762_amd.solver import Solver
    require_gpu()
    cfg = ocfg(P)
    Q = P.Q.copy()
    S = Solver(P, precision=FP32)
    for _ in range(steps):
        O.step(cfg, Q, P.cfl)
        S.step()
    G = S.state()
    assert S.check() == 0
    S.close()
    d = np.abs(G - Q).reshape(4, -1)
    return d.mean(axis=1), d.max(axis=1)


@pytest.mark.parametrize("fam,n,steps", [("shear", 256, 50), ("vortex", 64, 10),
                                         ("riemann", 256, 50)])
def test_trajectory_l1(fam, n, steps):
    P = PB.make(fam, n, seed=0) if fam != "vortex" else PB.vortex(n, cfl=0.5)
    l1, linf = run_pair(P, steps)
    report(f"f32 {fam}{n} {steps} steps", L1=[f"{v:.2e}" for v in l1],
           Linf=[f"{v:.2e}" for v in linf])
    # every conserved variable, relative to its magnitude
    scale = np.abs(P.Q).reshape(4, -1).max(axis=1)
    assert (l1 <= 1e-6 * scale).all(), (l1, scale)
    assert (linf <= 1e-3 * scale).all(), (linf, scale)
