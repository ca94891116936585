"""Thin driver over the C ABI: device buffers from torch, SSP-RK3 steps.

All arithmetic of a step runs in the library's HIP kernels: this module only
allocates device memory, holds the stream and calls gbr_compute_dt and
gbr_rk_stage three times per step.
"""
import numpy as np

from . import gbr


class Solver:
    def __init__(self, problem, device="cuda", stream=None, export_flags=False,
                 precision=gbr.GBR_PREC_FP64, detector=gbr.GBR_DET_PLAIN,
                 recon=gbr.GBR_RECON_PRIM, order=7, mp_mode=gbr.GBR_MP_FLAGGED,
                 fused_dt=False):
        import torch
        # fused_dt: after the first step, take dt from the extrema the last
        # stage-3 kernel reduced (gbr_stage_dt) instead of another pass over Q
        self.fused_dt = fused_dt
        self._stage3_fresh = False
        self.torch = torch
        self.p = problem
        self.device = device
        self.stream = stream
        self.ctx = gbr.gbr_init(problem.nx, problem.ny, problem.gamma, problem.mu, problem.Pr)
        gbr.gbr_set_geometry(self.ctx, *problem.geometry())
        gbr.gbr_set_scheme(self.ctx, recon, mp_mode, precision, detector)
        if order != 7:
            gbr.gbr_set_order(self.ctx, order)
        if getattr(problem, "sides", None) is not None:
            gbr.gbr_set_sides(self.ctx, problem.sides)
        if getattr(problem, "riemann", 0):
            gbr.gbr_set_riemann(self.ctx, problem.riemann)
        if export_flags:
            gbr.gbr_export_flags(self.ctx, True)
        shape = (4, problem.ny, problem.nx)
        self.Q = torch.empty(shape, dtype=torch.float64, device=device)
        self.Q1 = torch.empty_like(self.Q)
        self.Q2 = torch.empty_like(self.Q)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        if problem.Q is not None:
            self.set_state(problem.Q)

    def close(self):
        if self.ctx:
            gbr.gbr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, Q):
        self.Q.copy_(self.torch.from_numpy(np.ascontiguousarray(Q, np.float64)))
        self._stage3_fresh = False

    def state(self):
        self.torch.cuda.synchronize()
        return self.Q.cpu().numpy()

    def residual(self, Q=None):
        Q = self.Q if Q is None else Q
        R = self.torch.empty_like(Q)
        gbr.gbr_residual(self.ctx, Q, R, self.stream)
        return R

    def compute_dt(self, cfl=None):
        cfl = self.p.cfl if cfl is None else cfl
        if self.fused_dt and self._stage3_fresh:
            gbr.gbr_stage_dt(self.ctx, cfl, self.dt, self.stream)
            self._stage3_fresh = False
        else:
            gbr.gbr_compute_dt(self.ctx, self.Q, cfl, self.dt, self.stream)
        return self.dt

    def step(self, cfl=None):
        """One SSP-RK3 step: dt from Q^n on the device, three stage kernels,
        the device clock advanced by dt.  Q holds Q^{n+1} afterwards; no host
        synchronisation."""
        self.compute_dt(cfl)
        gbr.gbr_rk_stage(self.ctx, 1, self.dt, self.Q, self.Q, self.Q1, self.stream)
        gbr.gbr_rk_stage(self.ctx, 2, self.dt, self.Q, self.Q1, self.Q2, self.stream)
        gbr.gbr_rk_stage(self.ctx, 3, self.dt, self.Q, self.Q2, self.Q1, self.stream)
        gbr.gbr_advance_time(self.ctx, self.dt, self.stream)
        self.Q, self.Q1 = self.Q1, self.Q
        self._stage3_fresh = True

    def time(self):
        self.torch.cuda.synchronize()
        return gbr.gbr_get_time(self.ctx)

    def flags(self):
        sx = np.zeros((self.p.ny, self.p.nx + 1), np.uint8)
        sy = np.zeros((self.p.ny + 1, self.p.nx), np.uint8)
        gbr.gbr_get_flags(self.ctx, sx, sy, self.stream)
        return sx, sy

    def check(self):
        return gbr.gbr_check(self.ctx, self.stream)


class BatchSolver:
    """Many grids advanced together through the batched entry points: three
    state arrays per grid, one launch per stage over all grids."""

    def __init__(self, problems, precision=gbr.GBR_PREC_FP32_BULK, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.problems = list(problems)
        self.stream = stream
        P = self.problems
        self.b = gbr.gbr_batch_init([p.nx for p in P], [p.ny for p in P],
                                    [[p.x0, p.x1, p.y0, p.y1] for p in P],
                                    [[p.bc_x, p.bc_y] for p in P], [p.gamma for p in P],
                                    [p.mu for p in P], [p.Pr for p in P], [p.cfl for p in P],
                                    precision)
        self.bufs = [[torch.empty((4, p.ny, p.nx), dtype=torch.float64, device=device)
                      for p in P] for _ in range(3)]
        for q, p in zip(self.bufs[0], P):
            q.copy_(torch.from_numpy(np.ascontiguousarray(p.Q, np.float64)))
        gbr.gbr_batch_set_arrays(self.b, *self.bufs)

    def step(self):
        gbr.gbr_batch_step(self.b, self.stream)

    def states(self):
        """The current state tensors, one per grid."""
        return self.bufs[gbr.gbr_batch_current(self.b)]

    def dt(self):
        return gbr.gbr_batch_get_dt(self.b, len(self.problems), self.stream)

    def check(self):
        return gbr.gbr_batch_check(self.b, self.stream)

    def close(self):
        if self.b:
            gbr.gbr_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver3:
    """3D Euler (inviscid) grid: three device state buffers, SSP-RK3 steps
    through gbr3_compute_dt and gbr3_rk_stage."""

    def __init__(self, problem, device="cuda", stream=None, export_flags=False, order=7,
                 sweeps=None, fused_dt=False):
        import torch
        self.torch = torch
        self.p = problem
        self.stream = stream
        # fused_dt: after the first step, the time step from the extrema the
        # last stage-3 call reduced (gbr3_stage_dt), bit-identical
        self.fused_dt = fused_dt
        self._stage3_fresh = False
        self.ctx = gbr.gbr3_init(problem.nx, problem.ny, problem.nz, problem.gamma)
        gbr.gbr3_set_geometry(self.ctx, *problem.geometry(), *problem.bc)
        if order != 7:
            gbr.gbr3_set_order(self.ctx, order)
        if sweeps is not None:
            gbr.gbr3_set_sweeps(self.ctx, sweeps)
        if export_flags:
            gbr.gbr3_export_flags(self.ctx, True)
        shape = (5, problem.nz, problem.ny, problem.nx)
        self.Q = torch.empty(shape, dtype=torch.float64, device=device)
        self.Q1 = torch.empty_like(self.Q)
        self.Q2 = torch.empty_like(self.Q)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        if problem.Q is not None:
            self.Q.copy_(torch.from_numpy(np.ascontiguousarray(problem.Q, np.float64)))

    def close(self):
        if self.ctx:
            gbr.gbr3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self):
        self.torch.cuda.synchronize()
        return self.Q.cpu().numpy()

    def residual(self, Q=None):
        Q = self.Q if Q is None else Q
        R = self.torch.empty_like(Q)
        gbr.gbr3_residual(self.ctx, Q, R, self.stream)
        return R

    def set_state(self, Q):
        """Copy a host or device state into Q; the next step takes its time
        step from that state."""
        self.Q.copy_(self.torch.as_tensor(np.ascontiguousarray(Q, np.float64)))
        self._stage3_fresh = False

    def compute_dt(self, cfl=None):
        cfl = self.p.cfl if cfl is None else cfl
        if self.fused_dt and self._stage3_fresh:
            gbr.gbr3_stage_dt(self.ctx, cfl, self.dt, self.stream)
            self._stage3_fresh = False
        else:
            gbr.gbr3_compute_dt(self.ctx, self.Q, cfl, self.dt, self.stream)
        return self.dt

    def step(self, cfl=None):
        self.compute_dt(cfl)
        gbr.gbr3_rk_stage(self.ctx, 1, self.dt, self.Q, self.Q, self.Q1, self.stream)
        gbr.gbr3_rk_stage(self.ctx, 2, self.dt, self.Q, self.Q1, self.Q2, self.stream)
        gbr.gbr3_rk_stage(self.ctx, 3, self.dt, self.Q, self.Q2, self.Q1, self.stream)
        self.Q, self.Q1 = self.Q1, self.Q
        self._stage3_fresh = True

    def flags(self):
        p = self.p
        sx = np.zeros((p.nz, p.ny, p.nx + 1), np.uint8)
        sy = np.zeros((p.nz, p.ny + 1, p.nx), np.uint8)
        sz = np.zeros((p.nz + 1, p.ny, p.nx), np.uint8)
        gbr.gbr3_get_flags(self.ctx, sx, sy, sz, self.stream)
        return sx, sy, sz

    def check(self):
        return gbr.gbr3_check(self.ctx, self.stream)
