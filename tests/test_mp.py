"""Pins of the MP limiter (Sec. 2.3, eqs. mp5Condition, alpha, mp-procedure).

* Linear data is never limited: the activation product is -h^2/4 <= 1e-40
  and the GRB value is the exact interface value.
* Where the limiter acts on a step, the result lies between the two cell
  values beside the interface (no new extremum).
* The right value is the mirror image of the left one (index reflection with
  the gradient sign flipped).
"""
import numpy as np
import pytest


def grad(p):
    # sixth-order gradient of eq. (eqn:six) on an extended array; test-local
    # (only used to build inputs)
    q = np.pad(p, 3, mode="edge")
    return (45 * (q[4:-2] - q[2:-4]) - 9 * (q[5:-1] - q[1:-5]) + (q[6:] - q[:-6])) / 60


@pytest.mark.parametrize("h", [1.0, -0.3, 1e-6])
def test_linear_unlimited(orc, h):
    p = np.arange(-2, 4) * h + 0.4
    g = np.full(6, h)
    v, lim = orc.meg7_left(p, g)
    assert lim == 0 and abs(v - (0.4 + 0.5 * h)) < 1e-14
    v, lim = orc.meg7_right(p, g)
    assert lim == 0 and abs(v - (0.4 + 0.5 * h)) < 1e-14


@pytest.mark.parametrize("pos", range(-2, 4))
@pytest.mark.parametrize("H", [1.0, -2.5])
def test_step_no_new_extrema(orc, pos, H):
    full = np.zeros(12)
    full[pos + 5 + 1:] = H
    g = grad(full)
    p6, g6 = full[3:9], g[3:9]
    lo, hi = min(p6[2], p6[3]), max(p6[2], p6[3])
    for fn in (orc.meg7_left, orc.meg7_right):
        v, _ = fn(p6, g6)
        assert lo - 1e-14 <= v <= hi + 1e-14, (pos, v, lo, hi)


def test_limiter_acts_on_step(orc):
    full = np.zeros(12)
    full[6:] = 1.0          # step between cells j=0 (idx 5) and j+1
    g = grad(full)
    p6, g6 = full[3:9], g[3:9]
    vl, liml = orc.meg7_left(p6, g6)
    vr, limr = orc.meg7_right(p6, g6)
    assert liml == 1 or limr == 1


@pytest.mark.parametrize("seed", range(8))
def test_mirror_symmetry(orc, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=6)
    g = rng.normal(size=6)
    # mirror about the interface: offset m -> 1-m, gradients change sign
    pm = p[::-1].copy()
    gm = -g[::-1].copy()
    vl, _ = orc.meg7_left(p, g)
    vr, _ = orc.meg7_right(pm, gm)
    assert vl == pytest.approx(vr, abs=1e-13)


def test_mp_everywhere_equals_flagged_where_all_flagged(orc):
    """With every interface flagged (sigma forced to 0) the two MP modes
    compute the same thing, MEG7 states and F(Q) at every interface, bit for
    bit; with sigma free they differ exactly where the detector passes an
    interface (the smooth ones take MEG7 states under mp_mode 1)."""
    from paper_2305_00762_amd import problems as PB
    P = PB.riemann(40, seed=9, ny=36)
    for recon in (0, 1):
        R0 = orc.residual(orc.make_cfg(40, 36, force_sigma=0, recon=recon), P.Q)
        R1 = orc.residual(orc.make_cfg(40, 36, force_sigma=0, recon=recon, mp_mode=1), P.Q)
        assert np.array_equal(R0, R1)
        F0, sx, sy, _ = orc.residual(orc.make_cfg(40, 36, recon=recon), P.Q, want_flags=True)
        F1 = orc.residual(orc.make_cfg(40, 36, recon=recon, mp_mode=1), P.Q)
        assert sx.min() == 0 and sx.max() == 1
        assert not np.array_equal(F0, F1)
