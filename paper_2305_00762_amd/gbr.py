"""ctypes binding of libgbr.so (argument marshalling only).

Every function forwards to the C entry point of the same name declared in
include/gbr.h.  Device arrays are passed as torch tensors (float64, CUDA/HIP
device, contiguous, [4][ny][nx]) or as raw integer device addresses; streams
as torch.cuda.Stream, a raw hipStream_t integer, or None (current stream).
The library must be built (``python -m paper_2305_00762_amd.build`` or
``__graft_entry__.build()``); there is no fallback: a missing library is an
error.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgbr.so")

GBR_OK = 0
GBR_EINVAL = -1
GBR_ENOMEM = -2
GBR_EDEVICE = -3
GBR_ESTATE = -4
GBR_EUNSUPPORTED = -5
GBR_BC_PERIODIC = 0
GBR_BC_TRANSMISSIVE = 1
GBR_BC_REFLECT = 2
GBR_BC_NOSLIP = 3
GBR_BC_INFLOW = 4
GBR_RIEMANN_HLLC = 0
GBR_RIEMANN_HLLC_SS = 1
GBR_RECON_PRIM = 0
GBR_RECON_CONS = 1
GBR_MP_FLAGGED = 0
GBR_MP_EVERYWHERE = 1
GBR_PREC_FP64 = 0
GBR_PREC_FP32_BULK = 1
GBR_DET_PLAIN = 0
GBR_DET_MLP = 1

# every symbol include/gbr.h declares, with (restype, argtypes)
_vp, _i, _d = C.c_void_p, C.c_int, C.c_double
SIGNATURES = {
    "gbr_strerror": (C.c_char_p, [_i]),
    "gbr_version": (C.c_char_p, []),
    "gbr_init": (_i, [_i, _i, _d, _d, _d, C.POINTER(_vp)]),
    "gbr_destroy": (_i, [_vp]),
    "gbr_set_geometry": (_i, [_vp, _d, _d, _d, _d, _i, _i]),
    "gbr_set_scheme": (_i, [_vp, _i, _i, _i, _i]),
    "gbr_set_order": (_i, [_vp, _i]),
    "gbr_set_sides": (_i, [_vp, _vp]),
    "gbr_set_riemann": (_i, [_vp, _i]),
    "gbr_set_time": (_i, [_vp, _d]),
    "gbr_get_time": (_i, [_vp, C.POINTER(C.c_double)]),
    "gbr_advance_time": (_i, [_vp, _vp, _vp]),
    "gbr_residual": (_i, [_vp, _vp, _vp, _vp]),
    "gbr_rk_stage": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
    "gbr_compute_dt": (_i, [_vp, _vp, _d, _vp, _vp]),
    "gbr_export_flags": (_i, [_vp, _i]),
    "gbr_get_flags": (_i, [_vp, _vp, _vp, _vp]),
    "gbr_check": (_i, [_vp, _vp]),
    "gbr_tiling_count": (_i, []),
    "gbr_set_tiling": (_i, [_vp, _i]),
    "gbr_get_tiling": (_i, [_vp, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i)]),
    "gbr_autotune": (_i, [_vp, _vp, _i, _vp]),
    "gbr_mlp_create": (_i, [C.POINTER(_vp)]),
    "gbr_mlp_destroy": (_i, [_vp]),
    "gbr_mlp_set_params": (_i, [_vp, _vp, _vp]),
    "gbr_mlp_get_params": (_i, [_vp, _vp, _vp]),
    "gbr_mlp_features": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "gbr_mlp_forward": (_i, [_vp, _vp, _i, _vp, _vp]),
    "gbr_mlp_grad": (_i, [_vp, _vp, _vp, _vp, _i, _vp, _vp]),
    "gbr_mlp_train_step": (_i, [_vp, _vp, _vp, _vp, _i, C.c_float, _vp, _vp]),
    "gbr_set_mlp_detector": (_i, [_vp, _vp, C.c_float, _vp]),
    "gbr_batch_init": (_i, [_i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, C.POINTER(_vp)]),
    "gbr_batch_destroy": (_i, [_vp]),
    "gbr_batch_set_arrays": (_i, [_vp, _vp, _vp, _vp]),
    "gbr_batch_current": (_i, [_vp, C.POINTER(_i)]),
    "gbr_batch_step": (_i, [_vp, _vp]),
    "gbr_batch_use_graph": (_i, [_vp, _i]),
    "gbr_batch_tiling_count": (_i, []),
    "gbr_batch_set_tiling": (_i, [_vp, _i]),
    "gbr_batch_autotune": (_i, [_vp, _i, _vp]),
    "gbr_batch_info": (_i, [_vp] + [C.POINTER(_i)] * 5),
    "gbr_batch_get_dt": (_i, [_vp, _vp, _vp]),
    "gbr_batch_check": (_i, [_vp, _vp]),
    "gbr_batch_timing": (_i, [_vp, _i]),
    "gbr_batch_timing_read": (_i, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "gbr_timing": (_i, [_vp, _i]),
    "gbr_timing_read": (_i, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                             C.POINTER(C.c_uint64)]),
    "gbr_mlp_stats": (_i, [_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), _i]),
    "gbr_selftest_reciprocal": (_i, [C.c_uint32, C.c_uint32, C.POINTER(C.c_uint64)]),
    "gbr3_init": (_i, [_i, _i, _i, _d, C.POINTER(_vp)]),
    "gbr3_destroy": (_i, [_vp]),
    "gbr3_set_geometry": (_i, [_vp, _d, _d, _d, _d, _d, _d, _i, _i, _i]),
    "gbr3_set_order": (_i, [_vp, _i]),
    "gbr3_residual": (_i, [_vp, _vp, _vp, _vp]),
    "gbr3_rk_stage": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
    "gbr3_compute_dt": (_i, [_vp, _vp, _d, _vp, _vp]),
    "gbr3_export_flags": (_i, [_vp, _i]),
    "gbr3_get_flags": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "gbr3_check": (_i, [_vp, _vp]),
    "gbr3_timing": (_i, [_vp, _i]),
    "gbr3_timing_read": (_i, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
}

_lib = None


class GbrError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def load(path=LIB_PATH):
    """Load libgbr.so; raises if it is not built.

    torch is imported first: torch ships its own HIP runtime under the same
    soname (libamdhip64.so.7) as the system one libgbr.so is linked against,
    and the first one loaded serves the whole process.  Loading torch's first
    keeps one runtime, the one that owns torch's device memory and streams."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run __graft_entry__.build() "
                               "(the HIP library is required; there is no CPU fallback)")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code):
    return load().gbr_strerror(code).decode()


def version():
    return load().gbr_version().decode()


def _addr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(code, where):
    if code != GBR_OK:
        raise GbrError(code, where)
    return code


def gbr_init(nx, ny, gamma, mu, Pr):
    h = C.c_void_p()
    _check(load().gbr_init(nx, ny, gamma, mu, Pr, C.byref(h)), "gbr_init")
    return h.value


def gbr_destroy(ctx):
    return _check(load().gbr_destroy(ctx), "gbr_destroy")


def gbr_set_geometry(ctx, x0, x1, y0, y1, bc_x, bc_y):
    return _check(load().gbr_set_geometry(ctx, x0, x1, y0, y1, bc_x, bc_y), "gbr_set_geometry")


def gbr_set_scheme(ctx, recon=GBR_RECON_PRIM, mp_mode=GBR_MP_FLAGGED,
                   precision=GBR_PREC_FP64, detector=GBR_DET_PLAIN):
    return _check(load().gbr_set_scheme(ctx, recon, mp_mode, precision, detector),
                  "gbr_set_scheme")


def gbr_set_order(ctx, order):
    return _check(load().gbr_set_order(ctx, order), "gbr_set_order")


class GbrSide(C.Structure):
    """gbr_side of include/gbr.h."""
    _fields_ = [("kind", C.c_int * 2), ("state", (C.c_double * 4) * 2),
                ("split0", C.c_double), ("split_speed", C.c_double)]


def gbr_set_sides(ctx, sides):
    """sides: four (kind, state, kind1, state1, split0, split_speed) tuples
    (left, right, bottom, top), or None."""
    if sides is None:
        return _check(load().gbr_set_sides(ctx, None), "gbr_set_sides")
    arr = (GbrSide * 4)()
    for k, (k0, s0, k1, s1, split0, speed) in enumerate(sides):
        arr[k].kind[0], arr[k].kind[1] = k0, k1
        for g, st in enumerate((s0, s1)):
            if st is not None:
                for m in range(4):
                    arr[k].state[g][m] = st[m]
        arr[k].split0, arr[k].split_speed = split0, speed
    return _check(load().gbr_set_sides(ctx, C.cast(arr, C.c_void_p)), "gbr_set_sides")


def gbr_set_riemann(ctx, kind):
    return _check(load().gbr_set_riemann(ctx, kind), "gbr_set_riemann")


def gbr_set_time(ctx, t):
    return _check(load().gbr_set_time(ctx, t), "gbr_set_time")


def gbr_get_time(ctx):
    t = C.c_double()
    _check(load().gbr_get_time(ctx, C.byref(t)), "gbr_get_time")
    return t.value


def gbr_advance_time(ctx, dt, stream=None):
    return _check(load().gbr_advance_time(ctx, _addr(dt), _stream(stream)), "gbr_advance_time")


def gbr_residual(ctx, Q, Res, stream=None):
    return _check(load().gbr_residual(ctx, _addr(Q), _addr(Res), _stream(stream)),
                  "gbr_residual")


def gbr_rk_stage(ctx, stage, dt_dev, Qn, Qk, Qout, stream=None):
    return _check(load().gbr_rk_stage(ctx, stage, _addr(dt_dev), _addr(Qn), _addr(Qk),
                                      _addr(Qout), _stream(stream)), "gbr_rk_stage")


def gbr_compute_dt(ctx, Q, cfl, dt_dev, stream=None):
    return _check(load().gbr_compute_dt(ctx, _addr(Q), cfl, _addr(dt_dev), _stream(stream)),
                  "gbr_compute_dt")


def gbr_export_flags(ctx, enable=True):
    return _check(load().gbr_export_flags(ctx, 1 if enable else 0), "gbr_export_flags")


def gbr_get_flags(ctx, sig_x, sig_y, stream=None):
    return _check(load().gbr_get_flags(ctx, _addr(sig_x), _addr(sig_y), _stream(stream)),
                  "gbr_get_flags")


def gbr_check(ctx, stream=None):
    """Returns the status code (GBR_OK or GBR_ESTATE) without raising on ESTATE."""
    code = load().gbr_check(ctx, _stream(stream))
    if code not in (GBR_OK, GBR_ESTATE):
        raise GbrError(code, "gbr_check")
    return code


def gbr_tiling_count():
    return load().gbr_tiling_count()


def gbr_set_tiling(ctx, variant):
    return _check(load().gbr_set_tiling(ctx, variant), "gbr_set_tiling")


def gbr_get_tiling(ctx):
    """Returns (variant, tile_x, tile_y)."""
    v, tx, ty = C.c_int(), C.c_int(), C.c_int()
    _check(load().gbr_get_tiling(ctx, C.byref(v), C.byref(tx), C.byref(ty)), "gbr_get_tiling")
    return v.value, tx.value, ty.value


def gbr_autotune(ctx, Q, reps=3, stream=None):
    _check(load().gbr_autotune(ctx, _addr(Q), reps, _stream(stream)), "gbr_autotune")
    return gbr_get_tiling(ctx)


MLP_NW = 1952
MLP_NB = 65


def gbr_mlp_create():
    h = C.c_void_p()
    _check(load().gbr_mlp_create(C.byref(h)), "gbr_mlp_create")
    return h.value


def gbr_mlp_destroy(m):
    return _check(load().gbr_mlp_destroy(m), "gbr_mlp_destroy")


def gbr_mlp_set_params(m, w, b):
    import numpy as np
    w = np.ascontiguousarray(w, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    assert w.size == MLP_NW and b.size == MLP_NB
    return _check(load().gbr_mlp_set_params(m, w.ctypes.data, b.ctypes.data), "gbr_mlp_set_params")


def gbr_mlp_get_params(m):
    import numpy as np
    w = np.empty(MLP_NW, np.float32)
    b = np.empty(MLP_NB, np.float32)
    _check(load().gbr_mlp_get_params(m, w.ctypes.data, b.ctypes.data), "gbr_mlp_get_params")
    return w, b


def gbr_mlp_features(ctx, Q, feat, chi=None, stream=None):
    return _check(load().gbr_mlp_features(ctx, _addr(Q), _addr(feat), _addr(chi), _stream(stream)),
                  "gbr_mlp_features")


def gbr_mlp_forward(m, feat, n, logits, stream=None):
    return _check(load().gbr_mlp_forward(m, _addr(feat), n, _addr(logits), _stream(stream)),
                  "gbr_mlp_forward")


def gbr_mlp_grad(m, feat, labels, idx, batch, grad, stream=None):
    return _check(load().gbr_mlp_grad(m, _addr(feat), _addr(labels), _addr(idx), batch,
                                      _addr(grad), _stream(stream)), "gbr_mlp_grad")


def gbr_mlp_train_step(m, feat, labels, idx, batch, lr, loss=None, stream=None):
    return _check(load().gbr_mlp_train_step(m, _addr(feat), _addr(labels), _addr(idx), batch, lr,
                                            _addr(loss), _stream(stream)), "gbr_mlp_train_step")


def gbr_set_mlp_detector(ctx, m, margin, stream=None):
    return _check(load().gbr_set_mlp_detector(ctx, m, margin, _stream(stream)),
                  "gbr_set_mlp_detector")


def gbr_selftest_reciprocal(lo=0x00800000, hi=0x7E800000):
    """Floats with bit patterns in [lo, hi) whose detector reciprocal differs
    from IEEE division (0 over the default range)."""
    n = C.c_uint64()
    _check(load().gbr_selftest_reciprocal(lo, hi, C.byref(n)), "gbr_selftest_reciprocal")
    return n.value


def gbr_mlp_stats(ctx, reset=False):
    ev, fb = C.c_uint64(), C.c_uint64()
    _check(load().gbr_mlp_stats(ctx, C.byref(ev), C.byref(fb), 1 if reset else 0), "gbr_mlp_stats")
    return ev.value, fb.value


def gbr_timing(ctx, enable=True):
    return _check(load().gbr_timing(ctx, 1 if enable else 0), "gbr_timing")


def gbr_timing_read(ctx):
    """(flag-map ms, stage ms, calls) summed since timing was enabled or read."""
    d, st, n = C.c_double(), C.c_double(), C.c_uint64()
    _check(load().gbr_timing_read(ctx, C.byref(d), C.byref(st), C.byref(n)), "gbr_timing_read")
    return d.value, st.value, n.value


# ---------------------------------------------------------------- batches ---
def gbr_batch_init(nx, ny, geom, bc, gamma, mu, Pr, cfl, precision):
    """nx, ny, gamma, mu, Pr, cfl: sequences of length nprob; geom: [nprob][4]
    (x0, x1, y0, y1); bc: [nprob][2] (x, y)."""
    import numpy as np
    n = len(nx)
    a_i = lambda v: np.ascontiguousarray(v, dtype=np.int32).reshape(-1)
    a_d = lambda v: np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    arrs = [a_i(nx), a_i(ny), a_d(geom), a_i(bc), a_d(gamma), a_d(mu), a_d(Pr), a_d(cfl)]
    if any(len(x) != m * n for x, m in zip(arrs, (1, 1, 4, 2, 1, 1, 1, 1))):
        raise ValueError("gbr_batch_init: array lengths do not match nprob")
    h = C.c_void_p()
    _check(load().gbr_batch_init(n, *[x.ctypes.data for x in arrs], precision, C.byref(h)),
           "gbr_batch_init")
    return h.value


def gbr_batch_destroy(b):
    return _check(load().gbr_batch_destroy(b), "gbr_batch_destroy")


def gbr_batch_set_arrays(b, X, Y, Z):
    """X, Y, Z: sequences of device arrays (tensors or addresses), one per grid."""
    tabs = [(C.c_void_p * len(v))(*[_addr(t) for t in v]) for v in (X, Y, Z)]
    return _check(load().gbr_batch_set_arrays(b, *[C.cast(t, C.c_void_p) for t in tabs]),
                  "gbr_batch_set_arrays")


def gbr_batch_current(b):
    w = C.c_int()
    _check(load().gbr_batch_current(b, C.byref(w)), "gbr_batch_current")
    return w.value


def gbr_batch_step(b, stream=None):
    return _check(load().gbr_batch_step(b, _stream(stream)), "gbr_batch_step")


def gbr_batch_use_graph(b, enable=True):
    return _check(load().gbr_batch_use_graph(b, 1 if enable else 0), "gbr_batch_use_graph")


def gbr_batch_tiling_count():
    return load().gbr_batch_tiling_count()


def gbr_batch_set_tiling(b, variant):
    return _check(load().gbr_batch_set_tiling(b, variant), "gbr_batch_set_tiling")


def gbr_batch_autotune(b, reps=3, stream=None):
    _check(load().gbr_batch_autotune(b, reps, _stream(stream)), "gbr_batch_autotune")
    return gbr_batch_info(b)


def gbr_batch_info(b):
    """(form, tile_x, tile_y, total_tiles, workgroups)."""
    v = [C.c_int() for _ in range(5)]
    _check(load().gbr_batch_info(b, *[C.byref(x) for x in v]), "gbr_batch_info")
    return tuple(x.value for x in v)


def gbr_batch_get_dt(b, nprob, stream=None):
    import numpy as np
    out = np.zeros(nprob, np.float64)
    _check(load().gbr_batch_get_dt(b, out.ctypes.data, _stream(stream)), "gbr_batch_get_dt")
    return out


def gbr_batch_check(b, stream=None):
    return load().gbr_batch_check(b, _stream(stream))


def gbr_batch_timing(b, enable=True):
    return _check(load().gbr_batch_timing(b, 1 if enable else 0), "gbr_batch_timing")


def gbr_batch_timing_read(b):
    """(summed stage-launch ms, stage launches) since timing was enabled or read."""
    t, n = C.c_double(), C.c_uint64()
    _check(load().gbr_batch_timing_read(b, C.byref(t), C.byref(n)), "gbr_batch_timing_read")
    return t.value, n.value


# --------------------------------------------------------------------- 3D ---
def gbr3_init(nx, ny, nz, gamma):
    h = C.c_void_p()
    _check(load().gbr3_init(nx, ny, nz, gamma, C.byref(h)), "gbr3_init")
    return h.value


def gbr3_destroy(ctx):
    return _check(load().gbr3_destroy(ctx), "gbr3_destroy")


def gbr3_set_geometry(ctx, x0, x1, y0, y1, z0, z1, bc_x, bc_y, bc_z):
    return _check(load().gbr3_set_geometry(ctx, x0, x1, y0, y1, z0, z1, bc_x, bc_y, bc_z),
                  "gbr3_set_geometry")


def gbr3_set_order(ctx, order):
    return _check(load().gbr3_set_order(ctx, order), "gbr3_set_order")


def gbr3_residual(ctx, Q, Res, stream=None):
    return _check(load().gbr3_residual(ctx, _addr(Q), _addr(Res), _stream(stream)),
                  "gbr3_residual")


def gbr3_rk_stage(ctx, stage, dt, Qn, Qk, Qout, stream=None):
    return _check(load().gbr3_rk_stage(ctx, stage, _addr(dt), _addr(Qn), _addr(Qk), _addr(Qout),
                                       _stream(stream)), "gbr3_rk_stage")


def gbr3_compute_dt(ctx, Q, cfl, dt, stream=None):
    return _check(load().gbr3_compute_dt(ctx, _addr(Q), cfl, _addr(dt), _stream(stream)),
                  "gbr3_compute_dt")


def gbr3_export_flags(ctx, enable):
    return _check(load().gbr3_export_flags(ctx, 1 if enable else 0), "gbr3_export_flags")


def gbr3_get_flags(ctx, sig_x, sig_y, sig_z, stream=None):
    return _check(load().gbr3_get_flags(ctx, _addr(sig_x), _addr(sig_y), _addr(sig_z),
                                        _stream(stream)), "gbr3_get_flags")


def gbr3_check(ctx, stream=None):
    code = load().gbr3_check(ctx, _stream(stream))
    if code not in (GBR_OK, GBR_ESTATE):
        raise GbrError(code, "gbr3_check")
    return code


def gbr3_timing(ctx, enable):
    return _check(load().gbr3_timing(ctx, 1 if enable else 0), "gbr3_timing")


def gbr3_timing_read(ctx):
    """(summed ms of the sweep kernels, calls) since timing was enabled or read."""
    t, n = C.c_double(), C.c_uint64()
    _check(load().gbr3_timing_read(ctx, C.byref(t), C.byref(n)), "gbr3_timing_read")
    return t.value, n.value
