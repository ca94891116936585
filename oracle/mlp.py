"""Oracle of the learned discontinuity detector (test infrastructure only).

A small MLP stands in for the density detector of Sec. 2.4.  That detector
works dimension by dimension (psi^x from x-lines flags x-interfaces, psi^y
from y-lines flags y-interfaces), so the network is applied once per
direction d of a cell: its label is the plain per-cell outcome
chi^d = [psi^d < psi_c] (computed by the C oracle), its input 28 features:

  four 7-point stencils, normal direction first: rho along d, p along d, rho
  along the other direction, p along it (offsets -3..3, ghost cells as in the
  scheme; for d = x this is rho_x, p_x, rho_y, p_y), each taken to
  float32 and normalised as (s_k - mean) * r with
      sum  = ((((((s0+s1)+s2)+s3)+s4)+s5)+s6),  mean = sum * float32(1/7),
      r    = 1 / ((max - min) + 1e-3)           (IEEE float32 division),
  then rounded to bfloat16 (round to nearest even); features 28..31 are 0.

Network 28 -> 32 -> 32 -> 1: h1 = relu(W1 x + b1), h1 rounded to bf16,
h2 = relu(W2 h1 + b2), z = w3 . h2 + b3; weights are bf16, biases float32.
Inference rounds h2 to bf16 as well (the output layer is a matrix-core
product); training keeps h2 in float32.
Loss: binary cross-entropy with logits, mean over the batch.

Functions take numpy arrays; the forward/backward pass is evaluated in FP64
on the bf16-rounded operands (the GPU accumulates in FP32), and a pure FP64
variant (no intermediate rounding) serves the finite-difference pin.
"""
import numpy as np

NF = 28
NIN = 32       # padded input width
NH = 32
NW = NH * NF + NH * NH + NH      # 1952 weights
NB = NH + NH + 1                 # 65 biases


def bf16_round(x):
    """float32 -> bfloat16 (as float32 values), round to nearest even."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).reshape(a.shape)


def bf16_bits(x):
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16).reshape(a.shape)


def bits_to_f32(b):
    return (np.asarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32)


def _ghost(a, axis, off, bc):
    n = a.shape[axis]
    idx = np.arange(n) + off
    idx = idx % n if bc == 0 else np.clip(idx, 0, n - 1)
    return np.take(a, idx, axis=axis)


def primitives(Q, gamma=1.4):
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho
    p = (gamma - 1.0) * (Q[3] - rho * (u * u + v * v) / 2.0)
    return rho, p


def features(Q, bc_x, bc_y, gamma=1.4, direction=0):
    """Per-cell features [ny*nx][32] as bf16 bit patterns (uint16) for the
    evaluation along x (direction 0) or y (direction 1)."""
    rho, p = primitives(Q, gamma)
    ny, nx = rho.shape
    out = np.zeros((ny, nx, NIN), np.float32)
    one7 = np.float32(1.0 / 7.0)
    col = 0
    groups = [(rho, 1, bc_x), (p, 1, bc_x), (rho, 0, bc_y), (p, 0, bc_y)]
    if direction == 1:
        groups = groups[2:] + groups[:2]
    for field, axis, bc in groups:
        s = [_ghost(field, axis, k - 3, bc).astype(np.float32) for k in range(7)]
        tot = s[0]
        for k in range(1, 7):
            tot = (tot + s[k]).astype(np.float32)
        mean = (tot * one7).astype(np.float32)
        mx = np.maximum.reduce(s)
        mn = np.minimum.reduce(s)
        den = ((mx - mn).astype(np.float32) + np.float32(1e-3)).astype(np.float32)
        r = (np.float32(1.0) / den).astype(np.float32)
        for k in range(7):
            out[:, :, col] = ((s[k] - mean).astype(np.float32) * r).astype(np.float32)
            col += 1
    return bf16_bits(out.reshape(ny * nx, NIN))


def labels(psi_x, psi_y, psi_c=0.5):
    """Directional plain labels (chi^x, chi^y) from the detector values."""
    return (psi_x < psi_c).astype(np.uint8), (psi_y < psi_c).astype(np.uint8)


def unpack(w, b):
    w = np.asarray(w, np.float64)
    W1 = w[:NH * NF].reshape(NH, NF)
    W2 = w[NH * NF:NH * NF + NH * NH].reshape(NH, NH)
    w3 = w[NH * NF + NH * NH:]
    b = np.asarray(b, np.float64)
    return W1, W2, w3, b[:NH], b[NH:2 * NH], b[2 * NH]


def forward(feat_bits, w_bf16, b, round_h1=True, round_h2=True):
    """Logits (FP64) for bf16 features and bf16-valued weights (float arrays).

    Inference takes both hidden layers to bf16 as the next layer's operand
    (round_h1, round_h2); training keeps h2 in float32 (loss_and_grad)."""
    x = bits_to_f32(feat_bits)[:, :NF].astype(np.float64)
    W1, W2, w3, b1, b2, b3 = unpack(w_bf16, b)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h1r = bf16_round(h1.astype(np.float32)).astype(np.float64) if round_h1 else h1
    h2 = np.maximum(h1r @ W2.T + b2, 0.0)
    h2r = bf16_round(h2.astype(np.float32)).astype(np.float64) if round_h2 else h2
    return h2r @ w3 + b3


def loss_and_grad(feat_bits, labels, w, b, round_ops=True):
    """Mean BCE-with-logits loss and its gradient (dw [1952], db [65]).

    round_ops: evaluate with bf16 weights, bf16 h1, and bf16-rounded dh2 and
    dh1 as matrix-unit operands, as the GPU does; False gives the exact FP64
    gradient of the FP64 network (finite-difference pin)."""
    x = bits_to_f32(feat_bits)[:, :NF].astype(np.float64)
    y = np.asarray(labels, np.float64)
    B = x.shape[0]
    wq = bf16_round(np.asarray(w, np.float32)).astype(np.float64) if round_ops else np.asarray(w, np.float64)
    W1, W2, w3, b1, b2, b3 = unpack(wq, b)
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    h1o = bf16_round(h1.astype(np.float32)).astype(np.float64) if round_ops else h1
    a2 = h1o @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    # BCE with logits: log(1+exp(z)) - y z
    loss = np.mean(np.logaddexp(0.0, z) - y * z)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B
    dw3 = h2.T @ dz
    db3 = dz.sum()
    dh2 = np.outer(dz, w3) * (a2 > 0)
    dh2o = bf16_round(dh2.astype(np.float32)).astype(np.float64) if round_ops else dh2
    dW2 = dh2o.T @ h1o
    db2 = dh2.sum(axis=0)
    dh1 = (dh2o @ W2) * (a1 > 0)
    dh1o = bf16_round(dh1.astype(np.float32)).astype(np.float64) if round_ops else dh1
    dW1 = dh1o.T @ x
    db1 = dh1.sum(axis=0)
    dw = np.concatenate([dW1.ravel(), dW2.ravel(), dw3])
    db = np.concatenate([db1, db2, [db3]])
    return loss, dw, db


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), bias-corrected, returns (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
