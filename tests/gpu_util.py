"""Helpers shared by the GPU parity tests (compare the HIP path, called
through the C ABI, with the CPU oracle on identical seeded inputs)."""
import numpy as np
import pytest

import oracle as O


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def ocfg(P, **kw):
    if P.sides is not None:
        kw.setdefault("sides", [O.side(*s) for s in P.sides])
        kw.setdefault("riemann", P.riemann)
    return O.make_cfg(P.nx, P.ny, *P.geometry(), gamma=P.gamma, mu=P.mu, Pr=P.Pr, **kw)


def relerr(a, b):
    """Norm-wise relative error per conserved variable: max|a-b| / max|b|."""
    a = np.asarray(a).reshape(4, -1)
    b = np.asarray(b).reshape(4, -1)
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def flux_scale(P):
    """Per-variable scale of a residual: max |F_m| / min(dx, dy) over the
    convective fluxes of Q in x and y.  The residual is a difference of O(|F|)
    interface fluxes divided by the spacing, so its rounding error in any
    precision is ~eps |F| / dx, whatever the size of the difference."""
    Q = P.Q
    g = P.gamma
    r = Q[0]
    u, v = Q[1] / r, Q[2] / r
    p = (g - 1) * (Q[3] - 0.5 * r * (u * u + v * v))
    F = np.stack([r * u, r * u * u + p, r * u * v, u * (Q[3] + p)])
    G = np.stack([r * v, r * u * v, r * v * v + p, v * (Q[3] + p)])
    m = np.maximum(np.abs(F).reshape(4, -1).max(1), np.abs(G).reshape(4, -1).max(1))
    return m / min(P.dx, P.dy)


def res_err(R, Ro, P):
    """Residual error per variable relative to max(max|Res|, flux scale)."""
    R = np.asarray(R).reshape(4, -1)
    Ro = np.asarray(Ro).reshape(4, -1)
    scale = np.maximum(np.abs(Ro).max(1), flux_scale(P))
    return np.abs(R - Ro).max(1) / scale


def gpu_residual(P, precision=0, tiling=None, detector=0, recon=0, order=7, mp_mode=0):
    from paper_2305_00762_amd.solver import Solver
    from paper_2305_00762_amd import gbr
    torch = require_gpu()
    S = Solver(P, export_flags=True, precision=precision, detector=detector, recon=recon,
               order=order, mp_mode=mp_mode)
    if tiling is not None:
        gbr.gbr_set_tiling(S.ctx, tiling)
    R = S.residual()
    torch.cuda.synchronize()
    sx, sy = S.flags()
    st = S.check()
    out = R.cpu().numpy()
    S.close()
    return out, sx, sy, st


def report(name, **vals):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)
