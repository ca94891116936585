"""The binding rejects arguments the C entry points would access out of
bounds or on the wrong side (host memory, wrong element type, too few
elements, non-contiguous views) before anything is enqueued.  Host-only:
the context handles below are registered with the binding's size table but
never reach the library, since every call here must fail in the checks."""
import numpy as np
import pytest

from paper_2305_00762_amd import gbr


class FakeDev:
    """Stands in for a device tensor: what the checks read, nothing else."""

    def __init__(self, n, dtype="float64", contiguous=True, cuda=True, ok=False):
        self.n, self.dt, self.c, self.is_cuda, self.ok = n, dtype, contiguous, cuda, ok
        self.dtype = "torch." + dtype

    def numel(self):
        return self.n

    def is_contiguous(self):
        return self.c

    def data_ptr(self):
        # a valid argument yields a null address (the library would reject
        # it too); an invalid one must never get this far
        if not self.ok:
            raise AssertionError("a rejected argument must not reach the library")
        return 0


@pytest.fixture
def ctx():
    h = 0x7E57
    gbr._dims[h] = (16, 12)
    yield h
    gbr._dims.pop(h, None)


def rejects(fn, *a):
    with pytest.raises(gbr.GbrError) as e:
        fn(*a)
    assert e.value.code == gbr.GBR_EINVAL


def test_state_arrays_checked(ctx):
    good = FakeDev(4 * 16 * 12, ok=True)
    dt = FakeDev(1, ok=True)
    for bad in (np.zeros((4, 12, 16)), FakeDev(4 * 16 * 12, "float32"),
                FakeDev(4 * 16 * 12 - 1), FakeDev(4 * 16 * 12 + 4),
                FakeDev(4 * 16 * 12, contiguous=False), FakeDev(4 * 16 * 12, cuda=False)):
        rejects(gbr.gbr_residual, ctx, bad, good)
        rejects(gbr.gbr_residual, ctx, good, bad)
        rejects(gbr.gbr_rk_stage, ctx, 2, dt, good, bad, good)
        rejects(gbr.gbr_compute_dt, ctx, bad, 0.2, dt)
        rejects(gbr.gbr_autotune, ctx, bad)
    rejects(gbr.gbr_rk_stage, ctx, 1, FakeDev(1, "float32"), good, good, good)
    rejects(gbr.gbr_rk_stage, ctx, 1, np.zeros(1), good, good, good)
    rejects(gbr.gbr_compute_dt, ctx, good, 0.2, FakeDev(0))


def test_detector_buffers_checked(ctx):
    n = 16 * 12
    Q = FakeDev(4 * n, ok=True)
    rejects(gbr.gbr_mlp_features, ctx, Q, FakeDev(2 * n * 32 - 1, "int16"))
    rejects(gbr.gbr_mlp_features, ctx, Q, FakeDev(2 * n * 32, "float32"))
    rejects(gbr.gbr_mlp_features, ctx, Q, FakeDev(2 * n * 32, "int16", ok=True),
            FakeDev(2 * n - 1, "uint8"))
    rejects(gbr.gbr_mlp_forward, 1, FakeDev(32 * 100 - 1, "int16"), 100, FakeDev(100, "float32"))
    rejects(gbr.gbr_mlp_forward, 1, FakeDev(32 * 100, "int16", ok=True), 100,
            FakeDev(99, "float32"))
    feat, lab = FakeDev(3200, "int16", ok=True), FakeDev(100, "uint8", ok=True)
    rejects(gbr.gbr_mlp_grad, 1, feat, lab, FakeDev(63, "int32"), 64, FakeDev(2018, "float32"))
    rejects(gbr.gbr_mlp_grad, 1, feat, lab, FakeDev(64, "int32", ok=True), 64,
            FakeDev(2017, "float32"))


def test_flag_export_sizes_checked(ctx):
    rejects(gbr.gbr_get_flags, ctx, np.zeros((12, 16), np.uint8), None)
    rejects(gbr.gbr_get_flags, ctx, None, np.zeros((12, 16), np.uint8))
    rejects(gbr.gbr_get_flags, ctx, np.zeros((12, 17), np.float64), None)


def test_unknown_context_rejected():
    rejects(gbr.gbr_residual, 0xDEAD, FakeDev(4), FakeDev(4))


def test_batch_arrays_checked():
    b = 0xB47C
    gbr._dims[b] = [(16, 12), (20, 20)]
    try:
        ok = [FakeDev(4 * 16 * 12, ok=True), FakeDev(4 * 20 * 20, ok=True)]
        rejects(gbr.gbr_batch_set_arrays, b, ok, ok, ok[:1])
        rejects(gbr.gbr_batch_set_arrays, b, ok, ok,
                [FakeDev(4 * 20 * 20), FakeDev(4 * 16 * 12)])
        rejects(gbr.gbr_batch_set_arrays, b, ok, [ok[0], np.zeros(1600)], ok)
    finally:
        gbr._dims.pop(b, None)
