"""Training and evaluation of the learned discontinuity detector.

Everything numeric runs in the library's kernels (features, labels, forward,
backward, Adam, the stage kernels); this module only orchestrates:

  training set   seeded four-quadrant Riemann runs advanced with the plain
                 FP64 method; features and directional plain labels of every
                 cell of a snapshot, one sample per cell and direction
                 (default: 48 runs, seeds 1000-1047, 512^2, run k snapshotted
                 after the k-th entry, cyclically, of 1..200 steps: 1.26e7
                 cells, 2.5e7 samples);
  training       minibatches of 8192: half flagged samples, 30 % smooth
                 samples within 3 cells of a flagged one (hard negatives),
                 the rest other smooth samples, drawn from
                 numpy.random.default_rng(seed); Adam, cosine learning-rate
                 decay, 40000 steps;
  evaluation     fresh-seed fields (Riemann seed 5000, shear layer seed 5001,
                 4096^2, 50 steps): the FP32-bulk path with the plain and with
                 the learned detector against the plain FP64 path -- flag
                 mismatch (false negatives/positives of the network against
                 the plain labels on the same state, both directions),
                 fallback rate, L1/Linf per conserved variable, throughputs.

  python -m paper_2305_00762_amd.detector train [--out FILE] [--runs 40] ...
  python -m paper_2305_00762_amd.detector eval  [--weights FILE] [--n 4096] ...
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import gbr
from . import problems as PB

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "meg7_detector.npz")
DEFAULT_MARGIN = 48.0


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the learned detector runs on the GPU")
    return torch


def training_set(n=512, seeds=range(1000, 1040), steps=(100,), log=None, spread=False):
    """Features [S*2*n*n][32] (bf16 bits as int16) and directional plain
    labels [S*2*n*n] on the device, from seeded Riemann runs snapshotted after
    each count in `steps` (S = runs x snapshots; per snapshot: the n*n
    evaluations along x, then those along y).  spread: run k takes one
    snapshot only, after steps[k % len(steps)] steps (S = runs)."""
    from .solver import Solver
    torch = _torch()
    seeds = list(seeds)
    steps = sorted(steps)
    cells = 2 * n * n
    total = len(seeds) * (1 if spread else len(steps)) * cells
    feat = torch.empty((total, 32), dtype=torch.int16, device="cuda")
    lab = torch.empty(total, dtype=torch.uint8, device="cuda")
    k = 0
    for r, seed in enumerate(seeds):
        S = Solver(PB.riemann(n, seed=seed))
        done = 0
        for st in ([steps[r % len(steps)]] if spread else steps):
            for _ in range(st - done):
                S.step()
            done = st
            gbr.gbr_mlp_features(S.ctx, S.Q, feat[k * cells:], lab[k * cells:])
            k += 1
        if S.check() != gbr.GBR_OK:
            raise RuntimeError(f"bad state in training run seed {seed}")
        S.close()
        if log:
            log(f"training run seed {seed}: snapshot(s) after {done} steps")
    torch.cuda.synchronize()
    return feat, lab


def near_mask(labels, n, width=3):
    """Cells within `width` cells, along their own direction, of a labelled
    cell (per 2*n*n block: x-evaluations then y-evaluations)."""
    lab = labels.reshape(-1, 2, n, n).astype(bool)
    near = np.zeros_like(lab)
    for k in range(-width, width + 1):
        near[:, 0] |= np.roll(lab[:, 0], k, axis=2)
        near[:, 1] |= np.roll(lab[:, 1], k, axis=1)
    return near.reshape(-1)


def train(feat, lab, steps=3000, batch=4096, lr=3e-3, seed=0, init_seed=0, log=None,
          near=None, frac_near=0.25):
    """Train a new network; returns (handle, per-step mean losses).  With a
    `near` mask, a quarter of every batch are hard negatives (smooth cells
    next to a flagged one)."""
    torch = _torch()
    m = gbr.gbr_mlp_create()
    w, b = PB.mlp_init_params(init_seed)
    gbr.gbr_mlp_set_params(m, w, b)
    labels = lab.cpu().numpy()
    if near is None:
        idx = PB.balanced_batches(labels, batch, steps, seed)
    else:
        idx = PB.hard_batches(labels, near, batch, steps, seed, frac_near)
    idx = torch.from_numpy(idx).cuda()
    loss = torch.zeros(steps, dtype=torch.float32, device="cuda")
    for k in range(steps):
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps))
        gbr.gbr_mlp_train_step(m, feat, lab, idx[k], batch, rate, loss[k:k + 1])
        if log and (k + 1) % max(1, steps // 10) == 0:
            torch.cuda.synchronize()
            log(f"step {k + 1}: loss {float(loss[k]) / batch:.5f}")
    torch.cuda.synchronize()
    return m, (loss.cpu().numpy() / batch)


def save(m, path=DEFAULT_WEIGHTS, meta=None):
    w, b = gbr.gbr_mlp_get_params(m)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, w=w, b=b, meta=json.dumps(meta or {}))


def load(path=DEFAULT_WEIGHTS):
    d = np.load(path, allow_pickle=False)
    m = gbr.gbr_mlp_create()
    gbr.gbr_mlp_set_params(m, d["w"], d["b"])
    return m


def flag_rates(m, ctx, Q, n_cells, margin):
    """Network decision (with plain fallback below the margin) against the
    plain label on the same state, over both directions of every cell:
    (false-negative rate, false-positive rate, overall mismatch, fallback
    rate, flagged fraction)."""
    torch = _torch()
    n_cells = 2 * n_cells
    feat = torch.empty((n_cells, 32), dtype=torch.int16, device="cuda")
    chi = torch.empty(n_cells, dtype=torch.uint8, device="cuda")
    z = torch.empty(n_cells, dtype=torch.float32, device="cuda")
    gbr.gbr_mlp_features(ctx, Q, feat, chi)
    gbr.gbr_mlp_forward(m, feat, n_cells, z)
    torch.cuda.synchronize()
    plain = chi.bool()
    low = z.abs() < margin
    net = torch.where(low, plain, z > 0)
    pos = int(plain.sum())
    neg = n_cells - pos
    fn = int((plain & ~net).sum())
    fp = int((~plain & net).sum())
    del feat
    return {"false_neg_rate": fn / max(pos, 1), "false_pos_rate": fp / max(neg, 1),
            "mismatch_rate": (fn + fp) / n_cells, "fallback_rate": float(low.float().mean()),
            "flagged_fraction": pos / n_cells}


def run(P, steps, precision, detector=None, margin=DEFAULT_MARGIN, autotune=True):
    """Advance P for `steps` SSP-RK3 steps; returns (solver, seconds)."""
    from .solver import Solver
    torch = _torch()
    S = Solver(P, precision=precision)
    if detector is not None:
        gbr.gbr_set_mlp_detector(S.ctx, detector, margin)
        gbr.gbr_set_scheme(S.ctx, gbr.GBR_RECON_PRIM, gbr.GBR_MP_FLAGGED, precision,
                           gbr.GBR_DET_MLP)
    if autotune:
        gbr.gbr_autotune(S.ctx, S.Q, 3)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        S.step()
    stop.record()
    torch.cuda.synchronize()
    return S, start.elapsed_time(stop) * 1e-3


def evaluate(m, n=4096, steps=50, margin=DEFAULT_MARGIN,
             cases=(("riemann", 5000), ("shear", 5001)), log=None):
    """Per case: the plain FP64 path (the reference), the FP32-bulk path with
    the plain detector and with the learned one; L1/Linf of each against the
    FP64 path per conserved variable, throughputs, and the network's flag
    rates on the FP64 path's final state."""
    out = {}
    for fam, seed in cases:
        P = PB.make(fam, n, seed=seed)
        cells = n * n * 3 * steps
        base, t_base = run(P, steps, gbr.GBR_PREC_FP64)
        res = {"n": n, "steps": steps, "seed": seed,
               "fp64_plain_cell_stage_per_s": cells / t_base}
        ok = base.check() == gbr.GBR_OK
        for name, det in (("fp32_plain", None), ("fp32_mlp", m)):
            S, t = run(P, steps, gbr.GBR_PREC_FP32_BULK, detector=det, margin=margin)
            d = (S.Q - base.Q).abs().reshape(4, -1)
            res[f"{name}_cell_stage_per_s"] = cells / t
            res[f"{name}_speedup"] = t_base / t
            res[f"{name}_L1"] = [float(v) for v in d.mean(dim=1).cpu()]
            res[f"{name}_Linf"] = [float(v) for v in d.max(dim=1).values.cpu()]
            if det is not None:
                ev, fb = gbr.gbr_mlp_stats(S.ctx, reset=True)
                res["fallback_rate_in_run"] = fb / max(ev, 1)
            ok = ok and S.check() == gbr.GBR_OK
            S.close()
        res.update(flag_rates(m, base.ctx, base.Q, n * n, margin))
        res["status_ok"] = ok
        base.close()
        out[f"{fam}{n}"] = res
        if log:
            log(f"{fam}{n}: " + json.dumps(res))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--runs", type=int, default=48)
    t.add_argument("--n", type=int, default=512)
    t.add_argument("--run-steps", default="1,2,3,4,6,8,12,16,24,32,48,64,96,128,160,200",
                   help="comma-separated snapshot step counts")
    t.add_argument("--steps", type=int, default=40000)
    t.add_argument("--all-snapshots", action="store_true",
                   help="every run takes every snapshot (default: one per run, cycling)")
    t.add_argument("--hard", type=float, default=0.3,
                   help="fraction of each batch drawn from hard negatives (0: balanced only)")
    t.add_argument("--batch", type=int, default=8192)
    t.add_argument("--lr", type=float, default=3e-3)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--n", type=int, default=4096)
    e.add_argument("--steps", type=int, default=50)
    e.add_argument("--margin", type=float, default=DEFAULT_MARGIN)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    if a.cmd == "train":
        t0 = time.time()
        snaps = [int(v) for v in str(a.run_steps).split(",")]
        feat, lab = training_set(a.n, range(1000, 1000 + a.runs), snaps, log,
                                 spread=not a.all_snapshots)
        log(f"training set: {feat.shape[0]} samples, flagged fraction {float(lab.float().mean()):.4f}")
        near = near_mask(lab.cpu().numpy(), a.n) if a.hard > 0 else None
        m, losses = train(feat, lab, a.steps, a.batch, a.lr, log=log, near=near, frac_near=a.hard)
        save(m, a.out, {"runs": a.runs, "n": a.n, "run_steps": snaps, "spread": not a.all_snapshots,
                        "steps": a.steps,
                        "batch": a.batch, "lr": a.lr, "hard": a.hard,
                        "final_loss": float(losses[-20:].mean())})
        log(f"saved {a.out} ({time.time() - t0:.1f} s)")
    else:
        m = load(a.weights)
        print(json.dumps(evaluate(m, a.n, a.steps, a.margin, log=log)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
