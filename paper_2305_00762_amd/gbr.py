"""ctypes binding of libgbr.so (argument marshalling only).

Every function forwards to the C entry point of the same name declared in
include/gbr.h.  Device arrays are passed as torch tensors on the HIP device,
or as raw integer device addresses (taken as given); streams as
torch.cuda.Stream, a raw hipStream_t integer, or None (current stream).
Before any call is made, a tensor argument is checked against what the
entry point reads or writes: on the device, contiguous, of the element type
and at least the size the call accesses (state arrays: exactly the
context's [4][ny][nx] or [5][nz][ny][nx]).  A host array (numpy or a CPU
tensor) is accepted only where the header allows host memory (flag export,
MLP parameters, the batch tables).  A violation raises GbrError(GBR_EINVAL)
and nothing is enqueued.
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
GBR3_SWEEPS_LINES = 0
GBR3_SWEEPS_XY_FUSED = 1
GBR3_SWEEPS_XY_FUSED_HALF = 2

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
    "gbr_stage_dt": (_i, [_vp, _d, _vp, _vp]),
    "gbr_compute_dt_noalloc": (_i, [_i, _i, _d, _d, _d, _d, _vp, _d, _vp, _vp]),
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
    "gbr_set_mlp_reuse": (_i, [_vp, _i]),
    "gbr_mlp_get_flagmap": (_i, [_vp, _vp, _vp]),
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
    "gbr_selftest_division": (_i, [C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64)]),
    "gbr3_init": (_i, [_i, _i, _i, _d, C.POINTER(_vp)]),
    "gbr3_destroy": (_i, [_vp]),
    "gbr3_set_geometry": (_i, [_vp, _d, _d, _d, _d, _d, _d, _i, _i, _i]),
    "gbr3_set_order": (_i, [_vp, _i]),
    "gbr3_set_sweeps": (_i, [_vp, _i]),
    "gbr3_stage_dt": (_i, [_vp, _d, _vp, _vp]),
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


# grid sizes of live contexts, for the size checks: handle -> (nx, ny[, nz])
_dims = {}


def _bad(where, what):
    raise GbrError(GBR_EINVAL, f"{where}: {what}")


def _dev(x, where, name, dtypes, numel, exact=False, optional=False, host_ok=False):
    """Address of argument x after checking it against the call: a torch
    tensor on the HIP device (or, with host_ok, a host array), contiguous, of
    one of the element types `dtypes` (names, e.g. "float64"), with numel
    elements (at least numel unless exact).  Raw integers pass unchecked."""
    if x is None:
        if optional:
            return None
        _bad(where, f"{name} is required")
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda and not host_ok:
            _bad(where, f"{name} must be a device tensor (got a host tensor)")
        if not x.is_contiguous():
            _bad(where, f"{name} must be contiguous")
        dt = str(x.dtype).replace("torch.", "")
        n = x.numel()
    elif hasattr(x, "ctypes") and hasattr(x, "dtype"):
        if not host_ok:
            _bad(where, f"{name} must be device memory (got a host array)")
        if not x.flags.c_contiguous:
            _bad(where, f"{name} must be contiguous")
        dt = str(x.dtype)
        n = x.size
    else:
        raise TypeError(f"{where}: cannot take the address of {type(x)} ({name})")
    if dt not in dtypes:
        _bad(where, f"{name} must have element type {' or '.join(dtypes)} (got {dt})")
    if (n != numel) if exact else (n < numel):
        _bad(where, f"{name} has {n} elements, the call {'needs exactly' if exact else 'accesses'}"
                    f" {numel}")
    return _addr(x)


def _cells(ctx, where):
    d = _dims.get(ctx)
    if d is None:
        _bad(where, "unknown or destroyed context")
    n = 1
    for v in d:
        n *= v
    return n


def _state(ctx, x, where, name, nvar=4, optional=False):
    return _dev(x, where, name, ("float64",), nvar * _cells(ctx, where), exact=True,
                optional=optional)


def _scalar(x, where, name, dtype="float64", optional=False, host_ok=False):
    return _dev(x, where, name, (dtype,), 1, optional=optional, host_ok=host_ok)


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
    _dims[h.value] = (nx, ny)
    return h.value


def gbr_destroy(ctx):
    _dims.pop(ctx, None)
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
    w = "gbr_advance_time"
    return _check(load().gbr_advance_time(ctx, _scalar(dt, w, "dt"), _stream(stream)), w)


def gbr_residual(ctx, Q, Res, stream=None):
    w = "gbr_residual"
    return _check(load().gbr_residual(ctx, _state(ctx, Q, w, "Q"), _state(ctx, Res, w, "Res"),
                                      _stream(stream)), w)


def gbr_rk_stage(ctx, stage, dt_dev, Qn, Qk, Qout, stream=None):
    w = "gbr_rk_stage"
    return _check(load().gbr_rk_stage(ctx, stage, _scalar(dt_dev, w, "dt_dev"),
                                      _state(ctx, Qn, w, "Qn"), _state(ctx, Qk, w, "Qk"),
                                      _state(ctx, Qout, w, "Qout"), _stream(stream)), w)


def gbr_compute_dt(ctx, Q, cfl, dt_dev, stream=None):
    w = "gbr_compute_dt"
    return _check(load().gbr_compute_dt(ctx, _state(ctx, Q, w, "Q"), cfl,
                                        _scalar(dt_dev, w, "dt_dev"), _stream(stream)), w)


def gbr_stage_dt(ctx, cfl, dt_dev, stream=None):
    w = "gbr_stage_dt"
    return _check(load().gbr_stage_dt(ctx, cfl, _scalar(dt_dev, w, "dt_dev"), _stream(stream)), w)


def gbr_compute_dt_noalloc(nx, ny, dx, dy, gamma, mu, Q, cfl, dt_dev, stream=None):
    w = "gbr_compute_dt_noalloc"
    q = _dev(Q, w, "Q", ("float64",), 4 * nx * ny, exact=True)
    return _check(load().gbr_compute_dt_noalloc(nx, ny, dx, dy, gamma, mu, q, cfl,
                                                _scalar(dt_dev, w, "dt_dev"), _stream(stream)), w)


def gbr_export_flags(ctx, enable=True):
    return _check(load().gbr_export_flags(ctx, 1 if enable else 0), "gbr_export_flags")


def gbr_get_flags(ctx, sig_x, sig_y, stream=None):
    w = "gbr_get_flags"
    nx, ny = _dims.get(ctx) or _bad(w, "unknown or destroyed context")
    return _check(load().gbr_get_flags(
        ctx, _dev(sig_x, w, "sig_x", ("uint8",), ny * (nx + 1), optional=True, host_ok=True),
        _dev(sig_y, w, "sig_y", ("uint8",), (ny + 1) * nx, optional=True, host_ok=True),
        _stream(stream)), w)


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
    w = "gbr_autotune"
    _check(load().gbr_autotune(ctx, _state(ctx, Q, w, "Q"), reps, _stream(stream)), w)
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


_BF16 = ("int16", "uint16")


def gbr_mlp_features(ctx, Q, feat, chi=None, stream=None):
    w = "gbr_mlp_features"
    n = _cells(ctx, w)
    return _check(load().gbr_mlp_features(
        ctx, _state(ctx, Q, w, "Q"), _dev(feat, w, "feat", _BF16, 2 * n * 32),
        _dev(chi, w, "chi", ("uint8",), 2 * n, optional=True), _stream(stream)), w)


def gbr_mlp_forward(m, feat, n, logits, stream=None):
    w = "gbr_mlp_forward"
    return _check(load().gbr_mlp_forward(m, _dev(feat, w, "feat", _BF16, 32 * n), n,
                                         _dev(logits, w, "logits", ("float32",), n),
                                         _stream(stream)), w)


def _train_args(w, feat, labels, idx, batch):
    # the indices address rows of feat and labels; their values are the
    # caller's (checking them would read device memory)
    return (_dev(feat, w, "feat", _BF16, 32), _dev(labels, w, "labels", ("uint8",), 1),
            _dev(idx, w, "idx", ("int32",), batch))


def gbr_mlp_grad(m, feat, labels, idx, batch, grad, stream=None):
    w = "gbr_mlp_grad"
    return _check(load().gbr_mlp_grad(m, *_train_args(w, feat, labels, idx, batch), batch,
                                      _dev(grad, w, "grad", ("float32",), MLP_NW + MLP_NB + 1),
                                      _stream(stream)), w)


def gbr_mlp_train_step(m, feat, labels, idx, batch, lr, loss=None, stream=None):
    w = "gbr_mlp_train_step"
    return _check(load().gbr_mlp_train_step(
        m, *_train_args(w, feat, labels, idx, batch), batch, lr,
        _scalar(loss, w, "loss", "float32", optional=True, host_ok=True), _stream(stream)), w)


def gbr_set_mlp_detector(ctx, m, margin, stream=None):
    return _check(load().gbr_set_mlp_detector(ctx, m, margin, _stream(stream)),
                  "gbr_set_mlp_detector")


def gbr_set_mlp_reuse(ctx, per_step=True):
    return _check(load().gbr_set_mlp_reuse(ctx, 1 if per_step else 0), "gbr_set_mlp_reuse")


def gbr_mlp_get_flagmap(ctx, chi=None, stream=None):
    """The per-cell flag map of the last learned-detector evaluation as a host
    uint8 array [ny][nx] (bit 0 chi^x, bit 1 chi^y), or into chi."""
    import numpy as np
    w = "gbr_mlp_get_flagmap"
    nx, ny = _dims.get(ctx) or _bad(w, "unknown or destroyed context")
    out = np.zeros((ny, nx), np.uint8) if chi is None else chi
    _check(load().gbr_mlp_get_flagmap(ctx, _dev(out, w, "chi", ("uint8",), nx * ny, host_ok=True),
                                      _stream(stream)), w)
    return out


def gbr_selftest_reciprocal(lo=0x00800000, hi=0x7E800000):
    """Floats with bit patterns in [lo, hi) whose detector reciprocal differs
    from IEEE division (0 over the default range)."""
    n = C.c_uint64()
    _check(load().gbr_selftest_reciprocal(lo, hi, C.byref(n)), "gbr_selftest_reciprocal")
    return n.value


def gbr_selftest_division(seed=1, count=1 << 26):
    """Operand pairs whose time-step quotient differs from IEEE division (0)."""
    n = C.c_uint64()
    _check(load().gbr_selftest_division(seed, count, C.byref(n)), "gbr_selftest_division")
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
    _dims[h.value] = [(int(a), int(c)) for a, c in zip(arrs[0], arrs[1])]
    return h.value


def gbr_batch_destroy(b):
    _dims.pop(b, None)
    return _check(load().gbr_batch_destroy(b), "gbr_batch_destroy")


def gbr_batch_set_arrays(b, X, Y, Z):
    """X, Y, Z: sequences of device arrays (tensors or addresses), one per grid."""
    w = "gbr_batch_set_arrays"
    grids = _dims.get(b)
    if grids is None:
        _bad(w, "unknown or destroyed batch")
    if any(len(v) != len(grids) for v in (X, Y, Z)):
        _bad(w, f"every array set needs {len(grids)} arrays")
    tabs = [(C.c_void_p * len(v))(*[_dev(t, w, f"{nm}[{k}]", ("float64",), 4 * g[0] * g[1],
                                         exact=True) for k, (t, g) in enumerate(zip(v, grids))])
            for nm, v in (("X", X), ("Y", Y), ("Z", Z))]
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
    _dims[h.value] = (nx, ny, nz)
    return h.value


def gbr3_destroy(ctx):
    _dims.pop(ctx, None)
    return _check(load().gbr3_destroy(ctx), "gbr3_destroy")


def gbr3_set_geometry(ctx, x0, x1, y0, y1, z0, z1, bc_x, bc_y, bc_z):
    return _check(load().gbr3_set_geometry(ctx, x0, x1, y0, y1, z0, z1, bc_x, bc_y, bc_z),
                  "gbr3_set_geometry")


def gbr3_set_order(ctx, order):
    return _check(load().gbr3_set_order(ctx, order), "gbr3_set_order")


def gbr3_set_sweeps(ctx, form):
    return _check(load().gbr3_set_sweeps(ctx, form), "gbr3_set_sweeps")


def gbr3_residual(ctx, Q, Res, stream=None):
    w = "gbr3_residual"
    return _check(load().gbr3_residual(ctx, _state(ctx, Q, w, "Q", 5), _state(ctx, Res, w, "Res", 5),
                                       _stream(stream)), w)


def gbr3_rk_stage(ctx, stage, dt, Qn, Qk, Qout, stream=None):
    w = "gbr3_rk_stage"
    return _check(load().gbr3_rk_stage(ctx, stage, _scalar(dt, w, "dt"), _state(ctx, Qn, w, "Qn", 5),
                                       _state(ctx, Qk, w, "Qk", 5), _state(ctx, Qout, w, "Qout", 5),
                                       _stream(stream)), w)


def gbr3_compute_dt(ctx, Q, cfl, dt, stream=None):
    w = "gbr3_compute_dt"
    return _check(load().gbr3_compute_dt(ctx, _state(ctx, Q, w, "Q", 5), cfl, _scalar(dt, w, "dt"),
                                         _stream(stream)), w)


def gbr3_stage_dt(ctx, cfl, dt, stream=None):
    w = "gbr3_stage_dt"
    return _check(load().gbr3_stage_dt(ctx, cfl, _scalar(dt, w, "dt"), _stream(stream)), w)


def gbr3_export_flags(ctx, enable):
    return _check(load().gbr3_export_flags(ctx, 1 if enable else 0), "gbr3_export_flags")


def gbr3_get_flags(ctx, sig_x, sig_y, sig_z, stream=None):
    w = "gbr3_get_flags"
    nx, ny, nz = _dims.get(ctx) or _bad(w, "unknown or destroyed context")
    f = lambda x, nm, n: _dev(x, w, nm, ("uint8",), n, optional=True, host_ok=True)
    return _check(load().gbr3_get_flags(ctx, f(sig_x, "sig_x", nz * ny * (nx + 1)),
                                        f(sig_y, "sig_y", nz * (ny + 1) * nx),
                                        f(sig_z, "sig_z", (nz + 1) * ny * nx), _stream(stream)), w)


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
