"""Pins of the learned-detector oracle (oracle/mlp.py), independent of it:

* bf16 rounding equals torch's float32 -> bfloat16 conversion (round to
  nearest even), including ties;
* the FP64 gradient equals central finite differences of the FP64 loss;
* the gradient with the matrix-unit rounding points stays within the bf16
  error of the exact one;
* one Adam step equals torch.optim.Adam's;
* features: the free stream gives zeros; a density step gives the closed
  form (k - 3 + ...)/(H + 1e-3) pattern; padding is zero;
* inference: without the h2 rounding it is the training forward pass; the
  h2 rounding moves a logit by no more than its bf16 bound.
"""
import numpy as np
import pytest
import torch

import oracle.mlp as M
from paper_2305_00762_amd import problems as PB


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000).astype(np.float32) * 10,
                        np.float32([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8,
                                    1.00390625, 65504.0, 1e-30])])
    t = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert (M.bf16_round(x) == t).all()
    assert (M.bits_to_f32(M.bf16_bits(x)) == t).all()


def _data(seed, B=64):
    rng = np.random.default_rng(seed)
    feat = M.bf16_bits(rng.uniform(-0.6, 0.6, (B, 32)).astype(np.float32))
    feat[:, 28:] = 0
    labels = rng.integers(0, 2, B).astype(np.uint8)
    w, b = PB.mlp_init_params(seed)
    b = b + np.float32(0.05) * rng.standard_normal(65).astype(np.float32)
    return feat, labels, w, b


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_gradient_is_finite_difference(seed):
    feat, y, w, b = _data(seed)
    w = w.astype(np.float64)
    b = b.astype(np.float64)
    _, dw, db = M.loss_and_grad(feat, y, w, b, round_ops=False)
    rng = np.random.default_rng(seed + 7)
    h = 1e-6
    for k in rng.choice(M.NW, 40, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (M.loss_and_grad(feat, y, wp, b, False)[0] - M.loss_and_grad(feat, y, wm, b, False)[0]) / (2 * h)
        assert abs(fd - dw[k]) <= 1e-6 * max(1.0, abs(dw[k])) + 1e-8, (k, fd, dw[k])
    for k in range(M.NB):
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        fd = (M.loss_and_grad(feat, y, w, bp, False)[0] - M.loss_and_grad(feat, y, w, bm, False)[0]) / (2 * h)
        assert abs(fd - db[k]) <= 1e-6 * max(1.0, abs(db[k])) + 1e-8, (k, fd, db[k])


def test_rounded_gradient_close_to_exact():
    feat, y, w, b = _data(3, 512)
    _, dw0, db0 = M.loss_and_grad(feat, y, M.bf16_round(w), b, round_ops=False)
    _, dw1, db1 = M.loss_and_grad(feat, y, w, b, round_ops=True)
    assert np.linalg.norm(dw1 - dw0) <= 2e-2 * np.linalg.norm(dw0)
    assert np.linalg.norm(db1 - db0) <= 2e-2 * np.linalg.norm(db0)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(50)
    g1, g2 = rng.standard_normal(50), rng.standard_normal(50)
    p = torch.nn.Parameter(torch.from_numpy(w.copy()))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    ww = w.copy()
    for t, g in enumerate((g1, g2), start=1):
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        ww, m, v = M.adam(ww, g, m, v, t, 1e-2)
    assert np.allclose(ww, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_free_stream_zero():
    P = PB.free_stream(16, ny=12)
    f = M.features(P.Q, P.bc_x, P.bc_y)
    assert f.shape == (16 * 12, 32) and (f == 0).all()


def test_features_step_closed_form():
    n, s, H = 20, 9, 0.5
    rho = np.ones((12, n))
    rho[:, s + 1:] += H
    P = PB.free_stream(n, ny=12, u=0.0, v=0.0, p=1.0, bc=PB.BC_TRANSMISSIVE)
    P.Q = PB.prim_to_state(rho, np.zeros_like(rho), np.zeros_like(rho), np.ones_like(rho))
    f = M.bits_to_f32(M.features(P.Q, P.bc_x, P.bc_y)).reshape(12, n, 32)
    # cell s: stencil rho_{s-3..s+3} = [1,1,1,1,1+H,1+H,1+H]
    sten = np.float32([1, 1, 1, 1, 1 + H, 1 + H, 1 + H])
    mean = np.float32(sten.sum(dtype=np.float32)) * np.float32(1 / 7)
    expect = M.bf16_round((sten - mean) / np.float32(H + 1e-3))
    assert np.allclose(f[5, s, :7], expect, atol=0, rtol=2 ** -7)
    # constant stencils: only the rounding of the fixed-order mean remains
    # (7 s fl(1/7) need not round back to s), scaled by 1/1e-3
    assert np.abs(f[:, :, 14:21]).max() <= 2e-4        # rho along y is constant
    assert np.abs(f[:, :, 7:14]).max() <= 2e-4 and np.abs(f[:, :, 21:28]).max() <= 2e-4
    assert (f[:, :, 28:] == 0).all()


def test_features_y_direction_is_the_transposed_x_direction():
    """Evaluating along y equals evaluating the transposed field (x <-> y,
    u <-> v) along x, transposed back."""
    P = PB.riemann(18, seed=3, ny=14)
    Qt = np.stack([P.Q[0].T, P.Q[2].T, P.Q[1].T, P.Q[3].T])
    fy = M.features(P.Q, P.bc_x, P.bc_y, direction=1).reshape(14, 18, 32)
    fx_t = M.features(Qt, P.bc_y, P.bc_x, direction=0).reshape(18, 14, 32)
    assert (fy == fx_t.transpose(1, 0, 2)).all()
    fx = M.features(P.Q, P.bc_x, P.bc_y, direction=0).reshape(14, 18, 32)
    assert (fx[:, :, :14] == fy[:, :, 14:28]).all() and (fx[:, :, 14:28] == fy[:, :, :14]).all()


@pytest.mark.parametrize("fam,bc", [("riemann", None), ("shear", None), ("riemann", 0)])
def test_directional_labels_reproduce_the_method_flags(fam, bc):
    """The 6-cell buffer over the directional per-cell labels gives exactly
    the interface flags of the oracle's residual (eq. buffer): with correct
    labels the learned detector leaves the method unchanged."""
    import oracle as O
    P = PB.make(fam, 40, seed=11, ny=30)
    if bc is not None:
        P.bc_x = P.bc_y = bc
    cfg = O.make_cfg(P.nx, P.ny, *P.geometry(), gamma=P.gamma, mu=P.mu, Pr=P.Pr)
    _, sx, sy, _ = O.residual(cfg, P.Q, want_flags=True)
    _, px, py = O.cell_flags(cfg, P.Q)
    cx, cy = M.labels(px, py)
    ex, ey = O.sigma_from_cells(cx, cy, P.bc_x, P.bc_y)
    assert (ex == sx).all() and (ey == sy).all()
    if fam == "riemann":
        assert sx.min() == 0 and sy.min() == 0     # the case does flag


@pytest.mark.parametrize("seed", [0, 3])
def test_inference_forward_rounding_points(seed):
    """Inference takes h1 and h2 to bf16 as matrix-unit operands: without the
    h2 rounding its logits are the training forward pass's (same loss), and
    with it they move by no more than the bf16 bound sum_n |w3_n| h2_n 2^-9 --
    and do move."""
    feat, labels, w, b = _data(seed, B=256)
    wq = M.bf16_round(w)
    z0 = M.forward(feat, wq, b, round_h2=False)
    loss, _, _ = M.loss_and_grad(feat, labels, w, b, round_ops=True)
    y = labels.astype(np.float64)
    assert np.isclose(np.mean(np.logaddexp(0.0, z0) - y * z0), loss, rtol=1e-13, atol=0)
    z1 = M.forward(feat, wq, b)
    # h2 of the same pass, computed here from its definition
    x = M.bits_to_f32(feat)[:, :M.NF].astype(np.float64)
    W1, W2, w3, b1, b2, _ = M.unpack(wq, b)
    h1 = M.bf16_round(np.maximum(x @ W1.T + b1, 0.0).astype(np.float32)).astype(np.float64)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    # bf16 unit roundoff 2^-9, plus the float32 step before it and FP64 sums
    bound = (np.abs(w3) * h2).sum(axis=1) * 2.0 ** -9 * (1 + 2.0 ** -14)
    assert (np.abs(z1 - z0) <= bound).all()
    assert (z1 != z0).any()
