"""The seeded inputs: the batched workload's Riemann draws, run with the CPU
oracle at 48^2 for 40 steps, stay finite, and the draws the recipe replaces
(BATCH_VACUUM_SEEDS) are exactly the ones that do not -- their corner
expansion reaches vacuum, which the method (no positivity limiter) cannot
pass."""
import numpy as np

import oracle as O
from paper_2305_00762_amd import problems as PB


def _fails(seed, n=48, steps=40):
    P = PB.riemann(n, seed=seed)
    cfg = O.make_cfg(P.nx, P.ny, *P.geometry(), gamma=P.gamma)
    Q = P.Q.copy()
    for _ in range(steps):
        O.step(cfg, Q, P.cfl)
        if not np.isfinite(Q).all():
            return True
    return False


def test_batch_riemann_draws_run_and_the_replaced_ones_fail():
    spec = PB.batch_spec(512, seed=0)
    seeds = [sd for fam, n, sd in spec if fam == "riemann"]
    assert len(seeds) > 150
    replaced = {sd - 100000 for sd in seeds if sd >= 100000}
    assert replaced == set(PB.BATCH_VACUUM_SEEDS)
    assert all(_fails(sd) for sd in PB.BATCH_VACUUM_SEEDS)
    bad = [sd for sd in seeds if _fails(sd)]
    assert bad == []


def test_batch_spec_is_seeded_and_sized():
    a = PB.batch_spec(512, seed=0)
    assert a == PB.batch_spec(512, seed=0)
    sides = np.array([n for _, n, _ in a])
    assert sides.min() >= 64 and sides.max() <= 768
    fams = {f for f, _, _ in a}
    assert fams == {"vortex", "riemann", "shear"}
