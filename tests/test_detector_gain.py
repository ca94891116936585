"""What the trained detector network gains over the same network untrained,
and what it costs against the plain detector (through the C ABI).

On a fresh-seed four-quadrant Riemann field (seed 7000, not among the
training seeds) advanced with the plain FP64 method:

* raw agreement with the plain detector's directional labels (margin 0,
  the network decides everything): the trained network's balanced error
  (mean of its false-negative and false-positive rates) is at most 15 %,
  the untrained network's (its initial weights) at least 25 %;
* as the method uses it (default margin, plain fallback below it): the
  trained network decides at least 90 % of the evaluations itself and its
  decisions disagree with the plain labels on at most 0.1 % of all
  evaluations, while the untrained one falls back on more than half (there
  the method is the plain detector plus the network's cost);
* the solution: 20 FP32-bulk steps with the learned detector stay within L1
  density 1e-6 of the same steps with the plain detector, and the learned
  path's fallback count matches the evaluations it reports.
"""
import numpy as np
import pytest

from paper_2305_00762_amd import gbr
from paper_2305_00762_amd import problems as PB
from gpu_util import report, require_gpu

pytestmark = pytest.mark.gpu


def _rates(m, S, n, margin):
    from paper_2305_00762_amd import detector as D
    return D.flag_rates(m, S.ctx, S.Q, n * n, margin)


def test_trained_network_gain():
    torch = require_gpu()
    from paper_2305_00762_amd import detector as D
    from paper_2305_00762_amd.solver import Solver
    n = 512
    P = PB.riemann(n, seed=7000)
    S = Solver(P)
    for _ in range(30):
        S.step()
    trained = D.load()
    untrained = gbr.gbr_mlp_create()
    gbr.gbr_mlp_set_params(untrained, *PB.mlp_init_params(0))
    t0 = _rates(trained, S, n, 0.0)
    u0 = _rates(untrained, S, n, 0.0)
    tm = _rates(trained, S, n, D.DEFAULT_MARGIN)
    um = _rates(untrained, S, n, D.DEFAULT_MARGIN)
    bal = lambda r: 0.5 * (r["false_neg_rate"] + r["false_pos_rate"])
    report("detector gain", trained_balanced_error=bal(t0), untrained_balanced_error=bal(u0),
           trained_mismatch=t0["mismatch_rate"], untrained_mismatch=u0["mismatch_rate"],
           trained_mismatch_at_margin=tm["mismatch_rate"],
           trained_fallback=tm["fallback_rate"], untrained_fallback=um["fallback_rate"],
           flagged=t0["flagged_fraction"])
    assert t0["flagged_fraction"] > 1e-3               # the field has discontinuities
    assert bal(t0) <= 0.15 and bal(u0) >= 0.25
    assert tm["fallback_rate"] <= 0.10 and tm["mismatch_rate"] <= 1e-3
    assert um["fallback_rate"] >= 0.5
    S.close()
    gbr.gbr_mlp_destroy(untrained)

    # solution: learned vs plain detector on the FP32-bulk path, same steps
    runs = {}
    for name, det in (("plain", None), ("learned", trained)):
        R = Solver(P, precision=gbr.GBR_PREC_FP32_BULK)
        if det is not None:
            gbr.gbr_set_mlp_detector(R.ctx, det, D.DEFAULT_MARGIN)
            gbr.gbr_set_scheme(R.ctx, gbr.GBR_RECON_PRIM, gbr.GBR_MP_FLAGGED,
                               gbr.GBR_PREC_FP32_BULK, gbr.GBR_DET_MLP)
        for _ in range(20):
            R.step()
        assert R.check() == gbr.GBR_OK
        if det is not None:
            ev, fb = gbr.gbr_mlp_stats(R.ctx, reset=True)
            assert ev == 2 * n * n * 3 * 20 and fb <= 0.10 * ev
        runs[name] = R.Q.clone()
        R.close()
    l1 = (runs["learned"] - runs["plain"]).abs().reshape(4, -1).mean(dim=1).cpu().numpy()
    report("learned vs plain detector, 20 steps", L1=l1.tolist())
    assert l1[0] <= 1e-6
    gbr.gbr_mlp_destroy(trained)
