"""The time step reduced inside the stage-3 kernel (Sec. 2.5; gbr_stage_dt)
against the two-pass reduction over the state (gbr_compute_dt) and the
oracle's time step: its division replica equals IEEE division on random
operands; bit for bit on the state the stage-3 call wrote, for
inviscid and viscous grids, periodic and transmissive, FP64 and FP32 bulk,
both default tilings; a trajectory stepped with it equals, bit for bit, one
stepped with the separate reduction; without a stage-3 call since the last
read the call is rejected."""
import numpy as np
import pytest

import oracle as O
from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import ocfg, report, require_gpu

pytestmark = pytest.mark.gpu

CASES = {
    "riemann": lambda: PB.riemann(90, seed=3, ny=70),
    "shear": lambda: PB.shear(64, seed=2, ny=48),
    "shear_square": lambda: PB.shear(64, seed=2),
    "vortex": lambda: PB.vortex(48),
}


def test_division_replica_is_ieee():
    """The shared-reciprocal quotient of the stage-3 extrema equals IEEE
    division on 2^27 random operand pairs of its range (and zero numerators)."""
    require_gpu()
    assert gbr.gbr_selftest_division(seed=1, count=1 << 27) == 0
    assert gbr.gbr_selftest_division(seed=2 ** 40 + 7, count=1 << 27) == 0


def dt_bits(t):
    return t.cpu().numpy().view(np.uint64)[0]


@pytest.mark.parametrize("fam", sorted(CASES))
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("tiling", [0, 1])
def test_stage_dt_equals_two_pass_reduction(fam, precision, tiling):
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    P = CASES[fam]()
    S = Solver(P, precision=precision)
    gbr.gbr_set_tiling(S.ctx, tiling)
    with pytest.raises(gbr.GbrError):
        gbr.gbr_stage_dt(S.ctx, P.cfl, S.dt)           # no stage-3 output yet
    d_fused = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(3):
        S.step()                                        # compute_dt + 3 stages
        gbr.gbr_stage_dt(S.ctx, P.cfl, d_fused)
        S.compute_dt()
        torch.cuda.synchronize()
        a, b = dt_bits(d_fused), dt_bits(S.dt)
        Qg = S.state()
        o = np.float64(O.dt(ocfg(P), Qg, P.cfl)).view(np.uint64)
        report(f"stage dt {fam} p{precision} t{tiling} step {k}", fused=float(d_fused.item()),
               two_pass=float(S.dt.item()))
        assert a == b == o
    with pytest.raises(gbr.GbrError):
        gbr.gbr_stage_dt(S.ctx, P.cfl, d_fused)         # already read
    assert S.check() == gbr.GBR_OK
    S.close()


@pytest.mark.parametrize("fam", ["riemann", "shear"])
def test_trajectory_with_stage_dt_bit_identical(fam):
    from paper_2305_00762_amd.solver import Solver
    torch = require_gpu()
    P = CASES[fam]()
    A = Solver(P)
    B = Solver(P, fused_dt=True)
    for _ in range(5):
        A.step()
        B.step()
    qa, qb = A.state(), B.state()
    assert (qa.view(np.uint64) == qb.view(np.uint64)).all()
    assert float(A.dt.item()) == float(B.dt.item())
    A.close()
    B.close()
