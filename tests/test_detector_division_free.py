"""The stage kernels take the detector's decision psi < psi_c (Sec. 2.4,
eq. buffer; psi_c = 1/2) without its division: fl(num/den) < 1/2 exactly
when fl(2 num - den) < -den 2^-54.  This pins that equivalence in IEEE
double arithmetic (numpy rounds as the device does, one rounding per
operation), on random detector inputs over many scales and on inputs built
to put num/den within a few ulps of 1/2 on either side, against the oracle's
psi (the division the paper's formula calls for)."""
import numpy as np

import oracle as O


def ab_of(r):
    # the detector's smoothness measures of a 5-point density stencil,
    # rounded as the device rounds them
    rm2, rm1, r0, rp1, rp2 = r
    a = np.abs(r0 - rm1) + np.abs((r0 - 2.0 * rm1) + rm2)
    b = np.abs(r0 - rp1) + np.abs((r0 - 2.0 * rp1) + rp2)
    return a, b


def both(a, b):
    eps = O.detector_eps()
    num = (2.0 * a) * b + eps
    den = (a * a + b * b) + eps
    return (num / den) < 0.5, (2.0 * num - den) < -(den * 2.0 ** -54)


def test_random_stencils_match_oracle_psi():
    rng = np.random.default_rng(3)
    n = 400000
    r = rng.uniform(0.1, 2.0, (5, n)) * 10.0 ** rng.integers(-6, 3, (1, n))
    r[:, : n // 4] = 1.0 + 1e-4 * rng.standard_normal((5, n // 4))   # near-smooth
    a, b = ab_of(r)
    div, free = both(a, b)
    assert (div == free).all()
    # against the oracle's own psi on a sample
    for k in range(0, n, 997):
        assert (O.psi(*r[:, k]) < 0.5) == free[k]


def test_inputs_at_the_threshold():
    # psi = 1/2 where a^2 - 4ab + b^2 - eps = 0, i.e. a = 2b - sqrt(3b^2 + eps):
    # walk a across that point in steps of one ulp, at many scales of b
    rng = np.random.default_rng(4)
    eps = O.detector_eps()
    flips = 0
    for b in 10.0 ** rng.uniform(-3, 2, 400):
        a0 = 2.0 * b - np.sqrt(3.0 * b * b + eps)
        a = a0 + np.arange(-200, 201) * np.spacing(a0)
        div, free = both(a, np.full_like(a, b))
        assert (div == free).all()
        flips += int(div.any() and (~div).any())
    assert flips > 300          # the walk does cross the threshold
