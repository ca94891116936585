"""Pins of the primitive characteristic projection of the shock branch
(Sec. 2.3: MEG7 states in characteristic variables; reading R-CHAR, the
eigenvectors of the primitive normal Jacobian at the mean density and
pressure of the two cells beside the interface), independent of its
arithmetic:

* L R = I;
* R diagonalises the primitive-variable Jacobian A = (dQ/dW)^-1 dF/dW of the
  2D Euler flux of Sec. 1 (central differences of the flux and of the
  primitive-to-conservative map, both written here from their definitions)
  with eigenvalues u-c, u, u, u+c in that column order;
* on linear data the flagged branch (sigma = 0) returns the unlimited GRB
  states of the smooth branch, which are the exact interface values;
* a contact discontinuity (a density jump at constant velocity and pressure)
  lives in one characteristic field only: the limited states keep velocity
  and pressure exactly and bound the density by its two cell values.
A sign or index slip in a row of L or a column of R fails one of these.
"""
import math

import numpy as np
import pytest

G = 1.4


def cons(W, g=G):
    r, u, v, p = W
    return np.array([r, r * u, r * v, p / (g - 1) + 0.5 * r * (u * u + v * v)])


def flux(W, g=G):
    r, u, v, p = W
    E = p / (g - 1) + 0.5 * r * (u * u + v * v)
    return np.array([r * u, r * u * u + p, r * u * v, u * (E + p)])


def jac(fn, W, h=1e-6):
    J = np.zeros((4, 4))
    for k in range(4):
        e = np.zeros(4)
        e[k] = h * max(1.0, abs(W[k]))
        J[:, k] = (fn(W + e) - fn(W - e)) / (2 * e[k])
    return J


def rand_state(rng):
    return np.array([rng.uniform(0.2, 2.0), rng.uniform(-1, 1), rng.uniform(-1, 1),
                     rng.uniform(0.1, 2.0)])


@pytest.mark.parametrize("seed", range(5))
def test_char_prim_eigensystem(orc, seed):
    rng = np.random.default_rng(seed)
    Wa, Wb = rand_state(rng), rand_state(rng)
    Lm, Rm = orc.char_prim(Wa, Wb, G)
    assert np.allclose(Lm @ Rm, np.eye(4), atol=1e-13)
    assert np.allclose(Rm @ Lm, np.eye(4), atol=1e-13)
    # the Jacobian at the mean density and pressure (any velocity: the
    # eigenvectors do not depend on it)
    W = np.array([0.5 * (Wa[0] + Wb[0]), 0.5 * (Wa[1] + Wb[1]), 0.5 * (Wa[2] + Wb[2]),
                  0.5 * (Wa[3] + Wb[3])])
    A = np.linalg.solve(jac(cons, W), jac(flux, W))
    c = math.sqrt(G * W[3] / W[0])
    lam = np.diag([W[1] - c, W[1], W[1], W[1] + c])
    assert np.allclose(A @ Rm, Rm @ lam, atol=1e-7 * np.abs(A).max())


def linear_line(rng):
    a = rand_state(rng)
    b = rng.uniform(-0.05, 0.05, 4)
    off = np.arange(-4, 6)
    W = a[:, None] + b[:, None] * off[None, :]
    G6 = np.repeat(b[:, None], 6, axis=1)   # spacing-scaled gradient of linear data
    return W, G6, a + 0.5 * b


@pytest.mark.parametrize("seed", range(8))
def test_flagged_states_equal_grb_on_linear_data(orc, seed):
    W, G6, exact = linear_line(np.random.default_rng(100 + seed))
    L0, R0 = orc.interface_states(W, G6, sigma=0)
    L1, R1 = orc.interface_states(W, G6, sigma=1)
    scale = np.abs(W).max(axis=1)
    for a, b in ((L0, L1), (R0, R1), (L1, exact), (R1, exact)):
        assert (np.abs(a - b) <= 1e-14 * scale).all(), (a, b)


@pytest.mark.parametrize("pos", range(-2, 4))
@pytest.mark.parametrize("ratio", [0.125, 4.0])
def test_contact_limits_density_only(orc, pos, ratio):
    # density jump between offsets pos and pos + 1; u, v, p constant
    off = np.arange(-4, 6)
    rho = np.where(off > pos, ratio, 1.0)
    W = np.stack([rho, np.full(10, 0.3), np.full(10, -0.2), np.full(10, 0.9)])
    q = np.pad(rho, 3, mode="edge")
    grad = (45 * (q[4:-2] - q[2:-4]) - 9 * (q[5:-1] - q[1:-5]) + (q[6:] - q[:-6])) / 60
    G6 = np.zeros((4, 6))
    G6[0] = grad[2:8]
    WL, WR = orc.interface_states(W, G6, sigma=0)
    for S in (WL, WR):
        assert abs(S[1] - 0.3) <= 1e-15 and abs(S[2] + 0.2) <= 1e-15
        assert abs(S[3] - 0.9) <= 1e-15
        assert min(W[0, 4], W[0, 5]) - 1e-15 <= S[0] <= max(W[0, 4], W[0, 5]) + 1e-15
