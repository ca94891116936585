"""ctypes front end of the C oracle (test infrastructure only).

Arrays are numpy float64, structure of arrays [4][ny][nx] with x fastest:
Q = (rho, rho u, rho v, E).
"""
import ctypes as C
import math
import os

import numpy as np

from .build import ensure_built

BC_PERIODIC = 0
BC_TRANSMISSIVE = 1


class OrcSide(C.Structure):
    """One side of the domain: segment 0 where the tangential cell-centre
    coordinate is below split0 + split_speed * t, segment 1 elsewhere."""
    _fields_ = [("kind", C.c_int * 2), ("state", (C.c_double * 4) * 2),
                ("split0", C.c_double), ("split_speed", C.c_double)]


class OrcCfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("bc_x", C.c_int), ("bc_y", C.c_int),
        ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
        ("mp_mode", C.c_int), ("force_sigma", C.c_int), ("recon", C.c_int), ("order", C.c_int),
        ("riemann", C.c_int), ("use_sides", C.c_int), ("t", C.c_double),
        ("side", OrcSide * 4),
    ]


BC_REFLECT, BC_NOSLIP, BC_INFLOW = 2, 3, 4


def side(kind, state=None, kind1=None, state1=None, split0=math.inf, split_speed=0.0):
    """A side with one kind, or two segments split at split0 + split_speed t."""
    S = OrcSide()
    k1 = kind if kind1 is None else kind1
    S.kind[0], S.kind[1] = kind, k1
    for g, st in enumerate((state, state1 if kind1 is not None else state)):
        if st is not None:
            for m in range(4):
                S.state[g][m] = st[m]
    S.split0, S.split_speed = split0, split_speed
    return S


class Orc3Cfg(C.Structure):
    """3D Euler configuration (inviscid)."""
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("z0", C.c_double), ("z1", C.c_double),
        ("bc", C.c_int * 3), ("gamma", C.c_double), ("order", C.c_int),
    ]


class OrcCState(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("ub", "vb", "hb", "cb", "b1", "b2")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = ensure_built()
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.orc_residual.restype = C.c_long
        L.orc_residual.argtypes = [C.POINTER(OrcCfg), dp, dp, C.c_void_p, C.c_void_p]
        L.orc_residual_sigma.restype = C.c_long
        L.orc_residual_sigma.argtypes = [C.POINTER(OrcCfg), dp, dp, up, up]
        L.orc_rk_stage.restype = C.c_long
        L.orc_rk_stage.argtypes = [C.POINTER(OrcCfg), C.c_int, C.c_double, dp, dp, dp,
                                   C.c_void_p, C.c_void_p]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [C.POINTER(OrcCfg), dp, C.c_double]
        L.orc_step.restype = C.c_double
        L.orc_step.argtypes = [C.POINTER(OrcCfg), dp, C.c_double]
        L.orc3_residual.restype = C.c_long
        L.orc3_residual.argtypes = [C.POINTER(Orc3Cfg), dp, dp, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        L.orc3_rk_stage.restype = C.c_long
        L.orc3_rk_stage.argtypes = [C.POINTER(Orc3Cfg), C.c_int, C.c_double, dp, dp, dp,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc3_dt.restype = C.c_double
        L.orc3_dt.argtypes = [C.POINTER(Orc3Cfg), dp, C.c_double]
        L.orc3_step.restype = C.c_double
        L.orc3_step.argtypes = [C.POINTER(Orc3Cfg), dp, C.c_double]
        L.orc_detector_eps.restype = C.c_double
        L.orc_detector_eps.argtypes = []
        L.orc_psi.restype = C.c_double
        L.orc_psi.argtypes = [C.c_double] * 5
        L.orc_grad6.restype = C.c_double
        L.orc_grad6.argtypes = [dp]
        L.orc_table.restype = C.c_int
        L.orc_table.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_apply_interface.restype = None
        L.orc_apply_interface.argtypes = [dp, dp, dp]
        L.orc_apply_interface4.restype = None
        L.orc_apply_interface4.argtypes = [dp, dp, dp]
        L.orc_apply_interface_ab.restype = None
        L.orc_apply_interface_ab.argtypes = [dp, dp, C.c_double, C.c_double, dp]
        L.orc_meg7_left.restype = C.c_double
        L.orc_meg7_left.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]
        L.orc_meg7_right.restype = C.c_double
        L.orc_meg7_right.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]
        L.orc_hllc.restype = None
        L.orc_hllc.argtypes = [dp, dp, dp, dp, C.c_double, dp]
        L.orc_hllc_ss.restype = None
        L.orc_hllc_ss.argtypes = [dp, dp, dp, dp, C.c_double, dp]
        L.orc_line_flux.restype = None
        L.orc_line_flux.argtypes = [dp, dp, dp, dp, dp, dp, dp, C.c_double,
                                    C.POINTER(OrcCfg), dp, C.POINTER(C.c_int)]
        L.orc_cell_flags.restype = C.c_int
        L.orc_cell_flags.argtypes = [C.POINTER(OrcCfg), dp, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        L.orc_char_cons_state.restype = None
        L.orc_char_cons_state.argtypes = [dp, dp, C.c_double, C.POINTER(OrcCState)]
        L.orc_char_cons_fwd.restype = None
        L.orc_char_cons_fwd.argtypes = [C.POINTER(OrcCState), dp, dp]
        L.orc_char_cons_bwd.restype = None
        L.orc_char_cons_bwd.argtypes = [C.POINTER(OrcCState), dp, dp]
        L.orc_interface_states.restype = None
        L.orc_interface_states.argtypes = [dp, dp, C.POINTER(OrcCfg), C.c_int, dp, dp]
        L.orc_char_prim.restype = None
        L.orc_char_prim.argtypes = [dp, dp, C.c_double, dp, dp]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_get_threads.argtypes = []
        _lib = L
    return _lib


def make_cfg(nx, ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC,
             gamma=1.4, mu=0.0, Pr=0.72, mp_mode=0, force_sigma=-1, recon=0, order=7,
             riemann=0, sides=None, t=0.0):
    """recon 0: MEG7-prim (primitive variables), 1: MEG7-cons (conservative);
    order 7: the seventh-order GRB, 4: its fourth-order subset (alpha=4, beta=0);
    riemann 0: HLLC, 1: shock-stable HLLC; sides: four OrcSide (left, right,
    bottom, top) replacing bc_x / bc_y; t: time of the state (moving sides)."""
    cfg = OrcCfg(nx, ny, x0, x1, y0, y1, bc_x, bc_y, gamma, mu, Pr, mp_mode, force_sigma, recon,
                 order, riemann, 0, t)
    if sides is not None:
        cfg.use_sides = 1
        for k in range(4):
            cfg.side[k] = sides[k]
    return cfg


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def residual(cfg, Q, want_flags=False):
    """Res = Res(Q) (eq. eqn-differencing_residual).  Returns Res or
    (Res, sig_x [ny][nx+1], sig_y [ny+1][nx], n_mp_limited)."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    R = np.empty_like(Q)
    sx = np.zeros((cfg.ny, cfg.nx + 1), np.uint8) if want_flags else None
    sy = np.zeros((cfg.ny + 1, cfg.nx), np.uint8) if want_flags else None
    nl = lib().orc_residual(C.byref(cfg), Q, R, _ptr(sx), _ptr(sy))
    if nl < 0:
        raise ValueError("oracle residual: bad configuration")
    if want_flags:
        return R, sx, sy, nl
    return R


def residual_sigma(cfg, Q, sig_x, sig_y):
    """Residual with given interface flags (sig_x [ny][nx+1], sig_y [ny+1][nx])."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    R = np.empty_like(Q)
    sx = np.ascontiguousarray(sig_x, np.uint8)
    sy = np.ascontiguousarray(sig_y, np.uint8)
    if lib().orc_residual_sigma(C.byref(cfg), Q, R, sx, sy) < 0:
        raise ValueError("oracle residual: bad arguments")
    return R


def sigma_from_cells(chi_x, chi_y, bc_x, bc_y):
    """Interface flags from per-cell directional flags chi_x, chi_y [ny][nx]:
    sigma^x = 0 where any cell of the 6-cell buffer j-2..j+3 along x has
    chi_x set, sigma^y likewise from chi_y along y (the buffer of
    eq. buffer applied to per-cell flags; ghost cells take the flag of the
    cell they copy)."""
    ny, nx = chi_x.shape
    sx = np.ones((ny, nx + 1), np.uint8)
    sy = np.ones((ny + 1, nx), np.uint8)
    for j in range(-1, nx):
        cols = [k % nx if bc_x == 0 else min(max(k, 0), nx - 1) for k in range(j - 2, j + 4)]
        sx[:, j + 1] = (chi_x[:, cols].max(axis=1) == 0)
    for i in range(-1, ny):
        rows = [k % ny if bc_y == 0 else min(max(k, 0), ny - 1) for k in range(i - 2, i + 4)]
        sy[i + 1, :] = (chi_y[rows, :].max(axis=0) == 0)
    return sx, sy


def rk_stage(cfg, stage, dt, Qn, Qk, want_flags=False):
    Qn = np.ascontiguousarray(Qn, dtype=np.float64)
    Qk = np.ascontiguousarray(Qk, dtype=np.float64)
    out = np.empty_like(Qn)
    sx = np.zeros((cfg.ny, cfg.nx + 1), np.uint8) if want_flags else None
    sy = np.zeros((cfg.ny + 1, cfg.nx), np.uint8) if want_flags else None
    nl = lib().orc_rk_stage(C.byref(cfg), stage, dt, Qn, Qk, out, _ptr(sx), _ptr(sy))
    if nl < 0:
        raise ValueError("oracle rk stage: bad arguments")
    if want_flags:
        return out, sx, sy
    return out


def dt(cfg, Q, cfl):
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    return lib().orc_dt(C.byref(cfg), Q, cfl)


def step(cfg, Q, cfl):
    """One SSP-RK3 step in place; returns dt."""
    assert Q.flags.c_contiguous and Q.dtype == np.float64
    return lib().orc_step(C.byref(cfg), Q, cfl)


def detector_eps():
    return lib().orc_detector_eps()


def psi(rm2, rm1, r0, rp1, rp2):
    return lib().orc_psi(rm2, rm1, r0, rp1, rp2)


def grad6(p7):
    return lib().orc_grad6(np.ascontiguousarray(p7, dtype=np.float64))


def table(which):
    num = (C.c_int * 16)()
    den = C.c_int()
    n = lib().orc_table(which, num, C.byref(den))
    return [num[k] for k in range(n)], den.value


def apply_interface(v10, g6, order=7):
    """{GRB left, GRB right, F(f_L), F(f_R)} at j+1/2 from values at offsets
    -4..5 and gradients at -2..3, for the seventh-order GRB or its
    fourth-order subset."""
    out = np.empty(4)
    fn = lib().orc_apply_interface4 if order == 4 else lib().orc_apply_interface
    fn(np.ascontiguousarray(v10, np.float64), np.ascontiguousarray(g6, np.float64), out)
    return out


def apply_interface_ab(v10, g6, alpha, beta):
    """GRB left and right states at j+1/2 of the two-parameter family."""
    out = np.empty(2)
    lib().orc_apply_interface_ab(np.ascontiguousarray(v10, np.float64),
                                 np.ascontiguousarray(g6, np.float64), alpha, beta, out)
    return out


def meg7_left(p6, g6):
    """MEG7 left value at j+1/2; p6, g6 hold offsets -2..3 (cell j at index 2)."""
    p = np.ascontiguousarray(p6, np.float64)
    g = np.ascontiguousarray(g6, np.float64)
    lim = C.c_int()
    v = lib().orc_meg7_left(p.ctypes.data + 16, g.ctypes.data + 16, C.byref(lim))
    return v, lim.value


def meg7_right(p6, g6):
    p = np.ascontiguousarray(p6, np.float64)
    g = np.ascontiguousarray(g6, np.float64)
    lim = C.c_int()
    v = lib().orc_meg7_right(p.ctypes.data + 16, g.ctypes.data + 16, C.byref(lim))
    return v, lim.value


def hllc(WL, WR, FL, FR, gamma=1.4, riemann=0):
    """HLLC flux (riemann 0) or its shock-stable form (riemann 1)."""
    out = np.empty(4)
    fn = lib().orc_hllc_ss if riemann == 1 else lib().orc_hllc
    fn(*[np.ascontiguousarray(a, np.float64) for a in (WL, WR, FL, FR)], gamma, out)
    return out


def cell_flags(cfg, Q):
    """Per-cell plain detector label chi and psi_x, psi_y."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    chi = np.zeros((cfg.ny, cfg.nx), np.uint8)
    px = np.zeros((cfg.ny, cfg.nx))
    py = np.zeros((cfg.ny, cfg.nx))
    if lib().orc_cell_flags(C.byref(cfg), Q, _ptr(chi), _ptr(px), _ptr(py)) != 0:
        raise ValueError("oracle cell flags: bad configuration")
    return chi, px, py


def threads():
    """OpenMP threads the oracle's parallel loops use now."""
    return int(lib().orc_get_threads())


def set_threads(n):
    """Threads for the oracle's parallel loops (n < 1: all processors)."""
    lib().orc_set_threads(int(n))


def char_cons(Qa, Qb, gamma=1.4):
    """(L, R): the MEG7-cons characteristic projection at the mean of the
    conservative states Qa, Qb, as 4x4 matrices (columns: images of unit
    vectors)."""
    st = OrcCState()
    lib().orc_char_cons_state(np.ascontiguousarray(Qa, np.float64),
                              np.ascontiguousarray(Qb, np.float64), gamma, C.byref(st))
    Lm = np.zeros((4, 4))
    Rm = np.zeros((4, 4))
    for k in range(4):
        e = np.zeros(4)
        e[k] = 1.0
        out = np.zeros(4)
        lib().orc_char_cons_fwd(C.byref(st), e, out)
        Lm[:, k] = out
        lib().orc_char_cons_bwd(C.byref(st), e, out)
        Rm[:, k] = out
    return Lm, Rm


def interface_states(W40, G24, sigma, gamma=1.4, order=7, mp_mode=0):
    """(WL, WR): the rotated primitive states at interface j+1/2 that the
    Riemann solver receives, sigma = 1 the GRB states (Sec. 2.2), sigma = 0
    the MEG7 characteristic states (Sec. 2.3), from W [4][10] (offsets -4..5)
    and spacing-scaled gradients G [4][6] (offsets -2..3)."""
    cfg = make_cfg(16, 16, gamma=gamma, order=order, mp_mode=mp_mode)
    WL, WR = np.zeros(4), np.zeros(4)
    lib().orc_interface_states(np.ascontiguousarray(W40, np.float64).reshape(40),
                               np.ascontiguousarray(G24, np.float64).reshape(24),
                               C.byref(cfg), int(sigma), WL, WR)
    return WL, WR


def char_prim(Wa, Wb, gamma=1.4):
    """(L, R): the primitive characteristic projection (reading R-CHAR) at the
    interface between rotated primitive states Wa, Wb, as 4x4 matrices."""
    Lm, Rm = np.zeros(16), np.zeros(16)
    lib().orc_char_prim(np.ascontiguousarray(Wa, np.float64), np.ascontiguousarray(Wb, np.float64),
                        gamma, Lm, Rm)
    return Lm.reshape(4, 4), Rm.reshape(4, 4)


# ---------------------------------------------------------------- 3D ---
def make_cfg3(nx, ny, nz, x0=0.0, x1=1.0, y0=0.0, y1=1.0, z0=0.0, z1=1.0,
              bc=(BC_PERIODIC, BC_PERIODIC, BC_PERIODIC), gamma=1.4, order=7):
    cfg = Orc3Cfg(nx, ny, nz, x0, x1, y0, y1, z0, z1)
    for d in range(3):
        cfg.bc[d] = bc[d]
    cfg.gamma, cfg.order = gamma, order
    return cfg


def residual3(cfg, Q, want_flags=False):
    """3D Euler residual; Q [5][nz][ny][nx] = (rho, rho u, rho v, rho w, E).
    With want_flags: also the interface flags along x [nz][ny][nx+1], along y
    [nz][ny+1][nx] and along z [nz+1][ny][nx]."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    R = np.empty_like(Q)
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    sig = [np.zeros((nz, ny, nx + 1), np.uint8), np.zeros((nz, ny + 1, nx), np.uint8),
           np.zeros((nz + 1, ny, nx), np.uint8)] if want_flags else [None] * 3
    if lib().orc3_residual(C.byref(cfg), Q, R, *[_ptr(x) for x in sig]) < 0:
        raise ValueError("oracle 3D residual: bad arguments")
    return (R, *sig) if want_flags else R


def rk_stage3(cfg, stage, dt, Qn, Qk):
    Qn = np.ascontiguousarray(Qn, dtype=np.float64)
    Qk = np.ascontiguousarray(Qk, dtype=np.float64)
    out = np.empty_like(Qn)
    if lib().orc3_rk_stage(C.byref(cfg), stage, dt, Qn, Qk, out, None, None, None) < 0:
        raise ValueError("oracle 3D rk stage: bad arguments")
    return out


def dt3(cfg, Q, cfl):
    return lib().orc3_dt(C.byref(cfg), np.ascontiguousarray(Q, dtype=np.float64), cfl)


def step3(cfg, Q, cfl):
    """One SSP-RK3 step in place; returns dt."""
    assert Q.flags.c_contiguous and Q.dtype == np.float64
    return lib().orc3_step(C.byref(cfg), Q, cfl)
