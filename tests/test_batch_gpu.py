"""Batched grids through the C ABI (gbr_batch_*).

* every grid of a batch -- mixed families, ragged sizes, viscous and
  inviscid, both boundary types -- reproduces the single-grid path with the
  same tile shape and precision (state and per-grid time step) to 1e-12
  norm-wise relative per variable, for every launch form (persistent or one
  workgroup per tile, 31x15 or 15x15 tiles) and both precisions.  The two
  paths run the same tile function inlined into different kernels, where the
  compiler may contract multiply-adds differently: a few cells of smooth
  fields differ by an ulp or so after a step (and those differences feed back
  through later residuals); constant regions agree bit for bit;
* graph replay: each replay is checked against eager launches of the same
  steps, with eager torch work and synchronisation between the replays;
* two small grids of an FP64 batch against the CPU oracle after two steps
  (norm-wise relative 1e-12 per variable);
* autotune picks a valid form; bad arguments are rejected before any launch.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import ocfg, relerr, report, require_gpu

pytestmark = pytest.mark.gpu


def mixed_problems():
    ps = [PB.riemann(70, seed=21, ny=50), PB.shear(64, seed=22, ny=48), PB.vortex(48),
          PB.riemann(33, seed=23, ny=17), PB.shear(40, seed=24), PB.free_stream(12, ny=13),
          PB.riemann(96, seed=25)]
    ps[4].bc_x = PB.BC_TRANSMISSIVE          # mixed boundary types on a viscous grid
    return ps


def single_run(P, precision, tiling, steps):
    from paper_2305_00762_amd.solver import Solver
    S = Solver(P, precision=precision)
    gbr.gbr_set_tiling(S.ctx, tiling)
    dts = []
    for _ in range(steps):
        S.step()
        dts.append(float(S.dt.cpu()[0]))
    out = S.Q.clone()
    assert S.check() == gbr.GBR_OK
    S.close()
    return out, dts


@pytest.mark.parametrize("precision", [gbr.GBR_PREC_FP64, gbr.GBR_PREC_FP32_BULK])
@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_batch_matches_single_grids(precision, form):
    torch = require_gpu()
    from paper_2305_00762_amd.solver import BatchSolver
    ps = mixed_problems()
    B = BatchSolver(ps, precision=precision)
    gbr.gbr_batch_set_tiling(B.b, form)
    form_, tx, ty, total, wg = gbr.gbr_batch_info(B.b)
    assert form_ == form and wg % 8 == 0 and total > 0
    steps = 3
    dts = []
    for _ in range(steps):
        B.step()
        dts.append(B.dt())
    torch.cuda.synchronize()
    assert B.check() == gbr.GBR_OK
    tiling = 0 if tx == 31 else 1
    worst, worst_dt = 0.0, 0.0
    for k, P in enumerate(ps):
        ref, ref_dt = single_run(P, precision, tiling, steps)
        got = B.states()[k]
        worst = max(worst, float(relerr(got.cpu().numpy(), ref.cpu().numpy()).max()))
        bdt = np.array([d[k] for d in dts])
        worst_dt = max(worst_dt, float(np.abs(bdt - ref_dt).max() / max(ref_dt)))
    report(f"batch form {form} prec {precision}", tiles=total, workgroups=wg, relerr=worst,
           dt_relerr=worst_dt)
    assert worst <= 1e-12 and worst_dt <= 1e-12
    B.close()


def test_batch_graph_replays_match_eager():
    torch = require_gpu()
    from paper_2305_00762_amd.solver import BatchSolver
    s = torch.cuda.Stream()
    ps = mixed_problems()
    with torch.cuda.stream(s):
        G = BatchSolver(ps, stream=s)
        E = BatchSolver(ps, stream=s)
        gbr.gbr_batch_use_graph(E.b, False)
    s.synchronize()
    scratch = torch.zeros(1 << 20, device="cuda")
    for k in range(7):                     # more than the three captured roles
        with torch.cuda.stream(s):
            G.step()
            E.step()
        s.synchronize()
        scratch.add_(1.0)                  # eager work between replays
        torch.cuda.synchronize()
        assert gbr.gbr_batch_current(G.b) == gbr.gbr_batch_current(E.b)
        for a, b in zip(G.states(), E.states()):
            assert torch.equal(a, b), k
        assert (G.dt() == E.dt()).all()
    assert G.check() == gbr.GBR_OK and E.check() == gbr.GBR_OK
    G.close()
    E.close()


def test_batch_fp64_matches_oracle():
    torch = require_gpu()
    from paper_2305_00762_amd.solver import BatchSolver
    ps = [PB.riemann(40, seed=31, ny=28), PB.shear(32, seed=32, ny=24)]
    B = BatchSolver(ps, precision=gbr.GBR_PREC_FP64)
    B.step()
    B.step()
    torch.cuda.synchronize()
    for k, P in enumerate(ps):
        cfg = ocfg(P)
        Q = np.ascontiguousarray(P.Q.copy())
        O.step(cfg, Q, P.cfl)
        O.step(cfg, Q, P.cfl)
        got = B.states()[k].cpu().numpy()
        err = relerr(got, Q)
        report(f"batch vs oracle grid {k}", relerr=float(err.max()))
        assert (err <= 1e-12).all()
    B.close()


def test_batch_autotune_and_argument_errors():
    torch = require_gpu()
    from paper_2305_00762_amd.solver import BatchSolver
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B = BatchSolver(mixed_problems(), stream=s)
    s.synchronize()
    form, tx, ty, total, wg = gbr.gbr_batch_autotune(B.b, 2, s)
    assert 0 <= form < gbr.gbr_batch_tiling_count()
    B.step()
    assert B.check() == gbr.GBR_OK
    with pytest.raises(gbr.GbrError):
        gbr.gbr_batch_set_tiling(B.b, 99)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_batch_set_arrays(B.b, B.bufs[0], B.bufs[0], B.bufs[2])   # aliasing sets
    B.close()
    with pytest.raises(gbr.GbrError):
        gbr.gbr_batch_init([8], [64], [[0, 1, 0, 1]], [[0, 0]], [1.4], [0.0], [0.72], [0.2],
                           gbr.GBR_PREC_FP64)                              # nx < 12
    with pytest.raises(gbr.GbrError):
        gbr.gbr_batch_init([64], [64], [[0, 1, 0, 1]], [[0, 0]], [1.4], [0.0], [0.72], [0.2], 7)


def test_batch512_full_size():
    """The batched workload at full size -- 512 grids of sides U{64..768}
    (about 1.1e8 cells), FP32 bulk, autotuned launch form, steps replayed as a
    graph, as the bench runs it: no bad state, and the four smallest grids,
    the largest Riemann grid and the largest (viscous) shear-layer grid agree
    with the CPU oracle after two steps to the FP32-bulk trajectory bar (L1 <=
    1e-6 per conserved variable)."""
    torch = require_gpu()
    from paper_2305_00762_amd.solver import BatchSolver
    ps = [PB.vortex(n, cfl=0.5) if fam == "vortex" else PB.make(fam, n, seed=sd)
          for fam, n, sd in PB.batch_spec(512, seed=0)]
    by_size = sorted(range(len(ps)), key=lambda k: ps[k].nx * ps[k].ny)
    small = by_size[:4]
    large = [max((k for k in by_size if ps[k].family == fam), key=lambda k: ps[k].nx * ps[k].ny)
             for fam in ("riemann", "shear")]
    assert ps[large[1]].mu > 0.0
    init = {k: np.ascontiguousarray(ps[k].Q.copy()) for k in small + large}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B = BatchSolver(ps, precision=gbr.GBR_PREC_FP32_BULK, stream=s)
    s.synchronize()
    for P in ps:
        P.Q = None                      # the oracle starts from the saved copies
    # autotuning times first stages into a scratch set; the state stays
    form, tx, ty, total, wg = gbr.gbr_batch_autotune(B.b, 2, s)
    with torch.cuda.stream(s):
        B.step()
        B.step()
    s.synchronize()
    assert B.check() == gbr.GBR_OK
    st = B.states()
    for k in small + large:
        P = ps[k]
        Q = init[k].copy()
        cfg = ocfg(P)
        O.step(cfg, Q, P.cfl)
        O.step(cfg, Q, P.cfl)
        l1 = np.abs(st[k].cpu().numpy() - Q).reshape(4, -1).mean(axis=1)
        report(f"batch512 grid {k} ({P.family} {P.nx})", form=form, L1=l1.max())
        assert (l1 <= 1e-6).all(), (k, l1)
    B.close()
