"""Throughput of the MEG7 hot path on one MI355X: cell-stage updates/s.

A step is one SSP-RK3 time step of the whole hot path on one grid: the time
step (Sec. 2.5) and three stage calls, each the learned detector's per-cell
flag map (when selected and due) and the fused residual + stage-update
kernel.  The first step's time step is a reduction over Q^n; every later one
comes from the extrema the previous step's stage-3 kernel reduced while
writing Q^n (gbr_stage_dt, bit-identical).  Inputs are resident in HBM before
the timed region.

Default workload: the learned detector's evaluation field, the four-quadrant
Riemann problem at 4096^2 (seed 5000), whose state does not fit the 256 MB
Infinity Cache.  The headline path is FP32 bulk arithmetic with the learned
detector evaluated once per step on Q^n (FP64 state and stage update); the
plain FP64 path, the FP32-bulk path with the plain detector and the learned
detector evaluated every stage run the same steps from the same initial state
beside it, and the line reports their throughputs, the speedups and the
L1/Linf difference per conserved variable against the plain FP64 state.  The
shear layer at 4096^2 (seed 5001) is reported beside it the same way.  The
CPU oracle runs a bounded sample on all host threads and on one thread as
the cpu_baseline leg, and the headline path's state after the same number of
steps is compared with it (L1/Linf per variable).

Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload riemann4096]
                  [--path fp32_mlp_step|fp32_mlp|fp32|fp64|fp64_cons|fp64_g4|fp64_mpe]
                  [--no-cpu-baseline] [--no-compare] [--no-secondary]
"""
import hashlib
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-stage updates/s, FP32+MLP-detector vs FP64 plain, at stated L1 error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published

# Algorithmic HBM bytes per cell of one stage launch: read Q^(k) (32 B),
# write Q^(k+1) (32 B), and Q^n (32 B) in stages 2 and 3; 256/3 B on average.
BYTES_PER_CELL_STAGE = {1: 64.0, 2: 96.0, 3: 96.0}

# 3D (40 B per cell state): the x sweep reads Q^(k) and writes the residual
# accumulator (80 B), the y sweep reads Q^(k) and the accumulator and writes it
# (120 B), the z sweep reads Q^(k) and the accumulator, writes the result and
# reads Q^n (stage 1) or Q^n and Q^(k) (stages 2, 3) for the update:
# 120 + (40 + 80 + 80)/3 B.  Per cell-stage on average:
BYTES_PER_CELL_STAGE_3D = 80.0 + 120.0 + 120.0 + 200.0 / 3.0
# With the x and y sweeps fused over tiles of a z plane, the fused kernel
# reads Q^(k) and writes the accumulator (80 B) and the z sweep moves the
# 186.7 B above.
BYTES_PER_CELL_STAGE_3D_FUSED = 80.0 + 120.0 + 200.0 / 3.0
SWEEPS3 = {"lines": 0, "fused": 1, "fused_half": 2}

WORKLOADS = {
    # name: (family, n, seed, steps, description)
    "riemann1024": ("riemann", 1024, 0, 200,
                    "2D Euler four-quadrant Riemann problem, 1024x1024, quadrant states from "
                    "seed 0, transmissive, CFL 0.2"),
    "vortex64": ("vortex", 64, 0, 10, "2D Euler isentropic vortex 64x64 periodic, CFL 0.5"),
    "shear2048": ("shear", 2048, 0, 100,
                  "2D Navier-Stokes periodic shear layer 2048x2048, Re 1e4, Pr 0.72, Mach 0.3, "
                  "CFL 0.2"),
    "riemann4096": ("riemann", 4096, 5000, 50,
                    "2D Euler four-quadrant Riemann problem, 4096x4096, seed 5000, transmissive, "
                    "CFL 0.2 (the learned detector's evaluation field)"),
    "shear4096": ("shear", 4096, 5001, 50,
                  "2D Navier-Stokes periodic shear layer 4096x4096, seed 5001, Re 1e4, Pr 0.72, "
                  "Mach 0.3, CFL 0.2 (the learned detector's evaluation field)"),
    "double_mach": ("double_mach", 1024, 0, None,
                    "Double Mach reflection 1024x256 on [0,4]x[0,1] (Mach-10 shock at 60 degrees, "
                    "reflecting wall, inflow, exact moving top boundary, shock-stable HLLC), run "
                    "from t = 0 to t = 0.2, CFL 0.2"),
    "viscous_shock_tube": ("viscous_shock_tube", 1280, 0, None,
                           "Viscous shock tube 1280x640 on [0,1]x[0,0.5], Re 1000, Pr 0.73, "
                           "adiabatic no-slip walls and a symmetry plane, run from t = 0 to t = 1, "
                           "CFL 0.2"),
    "taylor_green3d": ("taylor_green3d", 64, 0, None,
                       "Inviscid Taylor-Green vortex 64^3 on [0, 2 pi)^3 (the paper's 3D case), "
                       "periodic, CFL 0.2, run from t = 0 to t = 10; kinetic energy and enstrophy "
                       "at t = 1..10"),
    "riemann3d128": ("riemann3d", 128, 0, 20,
                     "3D Euler eight-octant Riemann problem 128^3, octant states from seed 0, "
                     "transmissive, CFL 0.2"),
    "batch512": ("batch", 0, 0, 10,
                 "512 independent grids, side n ~ U{64..768} (seed 0), families uniform over "
                 "vortex / Riemann / shear layer, per-grid seed 10000 + index; one launch per "
                 "stage over all grids, steps replayed as a HIP graph"),
}

def _path(prec, mlp, dtype, kernel, cons=False, order=7, mp_everywhere=False, per_step=False):
    return {"prec": prec, "mlp": mlp, "dtype": dtype, "kernel": kernel, "cons": cons,
            "order": order, "mp_everywhere": mp_everywhere, "per_step": per_step}


PATHS = {
    # learned detector evaluated once per step on Q^n and reused by stages 2
    # and 3 (a change of the method; its L1 error is reported)
    "fp32_mlp_step": _path("fp32", True, "f32+f64", "meg7_stage_kernel_f32<mlp>", per_step=True),
    "fp32_mlp": _path("fp32", True, "f32+f64", "meg7_stage_kernel_f32<mlp>"),
    "fp32": _path("fp32", False, "f32+f64", "meg7_stage_kernel_f32"),
    "fp64": _path("fp64", False, "f64", "meg7_stage_kernel"),
    # MEG7-cons (Table 2): GRB and the MP procedure on conservative variables
    "fp64_cons": _path("fp64", False, "f64", "meg7_stage_kernel<cons>", cons=True),
    # the fourth-order GRB subset (alpha = 4, beta = 0; eq. fourth)
    "fp64_g4": _path("fp64", False, "f64", "meg7_stage_kernel<g4>", order=4),
    # the MEG7 states at every interface (the MP test everywhere)
    "fp64_mpe": _path("fp64", False, "f64", "meg7_stage_kernel<mpe>", mp_everywhere=True),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="riemann4096", choices=sorted(WORKLOADS))
    ap.add_argument("--path", default="fp32_mlp", choices=sorted(PATHS))
    ap.add_argument("--weights", default=None, help="detector weights (.npz)")
    ap.add_argument("--margin", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison paths beside the headline path")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the shear-layer field reported beside the 4096^2 Riemann field")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="host seconds of the all-threads oracle sample")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--sweeps3", default="lines", choices=sorted(SWEEPS3),
                    help="3D launch form: line sweeps, or x/y fused over z-plane tiles")
    ap.add_argument("--tiling", default="auto",
                    help="tile variant index, or 'auto' (gbr_autotune on the initial state)")
    return ap.parse_args()


def kernel_source_sha():
    """Hash of the HIP sources the kernels are built from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2305_00762_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, **launch):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if any
    (a line 'bytes_per_launch = <value>'), and only if the summary was taken
    on the current kernel sources (its 'source_sha = <hash>' line) and on the
    launch being reported (a 'key = value' line for every keyword, e.g. the
    tile shape): counters of another kernel or launch are not reported."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    keys = {}
    for line in open(path):
        t = line.strip()
        if "=" in t and not t.startswith(" "):
            k, v = t.split("=", 1)
            if k.strip() in ("bytes_per_launch", "source_sha") or k.strip() in launch:
                keys[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if keys.get("source_sha") != kernel_source_sha() or "bytes_per_launch" not in keys:
        return None
    if any(keys.get(k) != str(v) for k, v in launch.items()):
        return None
    return float(keys["bytes_per_launch"])


# VALU issue peak of the chip: 256 CUs x 4 SIMDs, each issuing one wave64
# VALU instruction per 4 cycles (16 lanes per cycle), at 2.4 GHz -- the FP64
# vector peak (78.6 TFLOP/s) counted in lane operations (one FMA each).
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def cpu_model():
    """The host CPU as /proc/cpuinfo describes it (model name, family, model,
    stepping, sockets, logical CPUs) and the CPUs this process may run on."""
    info = {}
    try:
        ids = set()
        nlog = 0
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k == "processor":
                nlog += 1
            elif k == "physical id":
                ids.add(v)
            elif k in ("model name", "cpu family", "model", "stepping", "cpu MHz", "cache size") \
                    and k not in info:
                info[k] = v
        info["sockets"] = len(ids) or None
        info["logical_cpus"] = nlog
    except OSError:
        pass
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        info["usable_cpus"] = os.cpu_count()
    return info


def load_valu(kernel_prefix, workload):
    """VALU wave-instructions per launch of a stage kernel from the committed
    rocprofv3 SQ-counter summary, if any (its SQ_INSTS_VALU line)."""
    path = os.path.join(ROOT, "profiles", f"meg7_stage_kernels_{workload}_sq_counters.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if len(f) >= 4 and f[0] == kernel_prefix and f[1] == "SQ_INSTS_VALU" and f[2] == "mean":
            return float(f[3])
    return None


def valu_roofline(kernel, workload, avg_us):
    prefix = {"meg7_stage_kernel_f32<mlp>": "meg7_stage_kernel_f32",
              "meg7_stage_kernel": "meg7_stage_kernel<"}.get(kernel)
    instr = load_valu(prefix, workload) if prefix else None
    if instr is None:
        return None
    achieved = instr * 64 / (avg_us * 1e-6)
    return {"bound": "alu", "achieved": achieved / 1e9, "peak": VALU_PEAK_LANE_OPS / 1e9,
            "unit": "G lane-op/s (issued)", "frac": achieved / VALU_PEAK_LANE_OPS,
            "valu_wave_instructions_per_launch": instr}


class Path:
    """One configured context and its three state buffers."""

    def __init__(self, P, path, stream, tiling, weights, margin):
        import torch
        from paper_2305_00762_amd import gbr
        self.gbr, self.P, self.stream = gbr, P, stream
        spec = PATHS[path]
        prec_name, mlp, self.dtype, self.kernel = spec["prec"], spec["mlp"], spec["dtype"], spec["kernel"]
        self.cons, order = spec["cons"], spec["order"]
        self.ctx = gbr.gbr_init(P.nx, P.ny, P.gamma, P.mu, P.Pr)
        gbr.gbr_set_geometry(self.ctx, *P.geometry())
        prec = gbr.GBR_PREC_FP32_BULK if prec_name == "fp32" else gbr.GBR_PREC_FP64
        self.net = None
        det = gbr.GBR_DET_PLAIN
        if mlp:
            from paper_2305_00762_amd import detector as D
            self.net = D.load(weights or D.DEFAULT_WEIGHTS)
            gbr.gbr_set_mlp_detector(self.ctx, self.net, D.DEFAULT_MARGIN if margin is None else margin,
                                     stream.cuda_stream)
            det = gbr.GBR_DET_MLP
        recon = gbr.GBR_RECON_CONS if self.cons else gbr.GBR_RECON_PRIM
        mp = gbr.GBR_MP_EVERYWHERE if spec["mp_everywhere"] else gbr.GBR_MP_FLAGGED
        gbr.gbr_set_scheme(self.ctx, recon, mp, prec, det)
        if spec["per_step"]:
            gbr.gbr_set_mlp_reuse(self.ctx, True)
        self.name = path
        # the next time step comes from the last stage-3 output's extrema
        self.fresh = False
        if order != 7:
            gbr.gbr_set_order(self.ctx, order)
        self.order = order
        if P.sides is not None:
            gbr.gbr_set_sides(self.ctx, P.sides)
        if P.riemann:
            gbr.gbr_set_riemann(self.ctx, P.riemann)
        dev = torch.device("cuda:0")
        self.Q = [torch.from_numpy(P.Q).to(dev) for _ in range(3)]
        self.Q0 = self.Q[0].clone()
        self.dt = torch.zeros(1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        if tiling == "auto":
            gbr.gbr_autotune(self.ctx, self.Q[0], 5, stream.cuda_stream)
        else:
            gbr.gbr_set_tiling(self.ctx, int(tiling))
        self.tile = gbr.gbr_get_tiling(self.ctx)

    def reset(self):
        import torch
        for q in self.Q:
            q.copy_(torch.from_numpy(self.P.Q))
        torch.cuda.synchronize()
        self.gbr.gbr_set_time(self.ctx, 0.0)
        self.fresh = False

    def step(self):
        """One SSP-RK3 step on self.stream; Q^{n+1} ends in self.Q[0]."""
        g, sh = self.gbr, self.stream.cuda_stream
        Q, Q1, Q2 = self.Q
        if self.fresh:
            g.gbr_stage_dt(self.ctx, self.P.cfl, self.dt, sh)
        else:
            g.gbr_compute_dt(self.ctx, Q, self.P.cfl, self.dt, sh)
        self.fresh = True
        g.gbr_rk_stage(self.ctx, 1, self.dt, Q, Q, Q1, sh)
        g.gbr_rk_stage(self.ctx, 2, self.dt, Q, Q1, Q2, sh)
        g.gbr_rk_stage(self.ctx, 3, self.dt, Q, Q2, Q1, sh)
        if self.P.sides is not None:
            g.gbr_advance_time(self.ctx, self.dt, sh)
        self.Q = [Q1, Q, Q2]

    def run(self, warmup, steps, timing=False):
        """warmup untimed steps, then `steps` timed ones; returns total ms of
        the timed steps (and the kernel timings when asked)."""
        import torch
        g, sh = self.gbr, self.stream.cuda_stream
        with torch.cuda.stream(self.stream):
            for _ in range(warmup):
                self.step()
        self.stream.synchronize()
        if g.gbr_check(self.ctx, sh) != g.GBR_OK:
            raise RuntimeError("device reported a bad state during warmup")
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        if timing:
            g.gbr_timing(self.ctx, True)
        with torch.cuda.stream(self.stream):
            start.record(self.stream)
            for _ in range(steps):
                self.step()
            stop.record(self.stream)
        self.stream.synchronize()
        torch.cuda.synchronize()
        kt = None
        if timing:
            kt = g.gbr_timing_read(self.ctx)
            g.gbr_timing(self.ctx, False)
        self.status = g.gbr_check(self.ctx, sh)
        return start.elapsed_time(stop), kt

    def run_to(self, t_final, chunk=250):
        """Whole steps from the current state until the device clock reaches
        t_final (the last step passes it by less than one dt).  The clock and
        the last dt are read after each batch of steps; a batch is at most
        `chunk` steps and at most the steps the last dt says remain, so the
        batches shrink to single steps near the end.  Returns (ms, steps)."""
        import torch
        g, sh = self.gbr, self.stream.cuda_stream
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        steps, batch = 0, chunk
        with torch.cuda.stream(self.stream):
            start.record(self.stream)
            while True:
                for _ in range(batch):
                    self.step()
                steps += batch
                self.stream.synchronize()
                t = g.gbr_get_time(self.ctx)
                if t >= t_final:
                    break
                dt = float(self.dt.item())
                batch = max(1, min(chunk, int((t_final - t) / dt)))
            stop.record(self.stream)
        self.stream.synchronize()
        torch.cuda.synchronize()
        self.status = g.gbr_check(self.ctx, sh)
        return start.elapsed_time(stop), steps

    def close(self):
        self.gbr.gbr_destroy(self.ctx)
        if self.net is not None:
            self.gbr.gbr_mlp_destroy(self.net)


def diff(Qa, Qb):
    d = (Qa - Qb).abs().reshape(4, -1)
    return ([float(v) for v in d.mean(dim=1).cpu()], [float(v) for v in d.max(dim=1).values.cpu()])


def cpu_baseline(P, seconds, max_steps=50, recon=0, order=7, mp_mode=0, one_thread=True):
    """The CPU oracle on a bounded sample of the same workload: whole SSP-RK3
    steps on the full grid from the initial state, on all host threads, until
    about `seconds` of host time have passed; and one thread on one stage-1
    call over the full grid (16.8M cell-stages at 4096^2, about 10 s).
    Returns (record, state after the all-threads sample, steps)."""
    import numpy as np
    import oracle as O
    cfg = O.make_cfg(P.nx, P.ny, *P.geometry(), gamma=P.gamma, mu=P.mu, Pr=P.Pr, recon=recon,
                     order=order, riemann=P.riemann, mp_mode=mp_mode,
                     sides=[O.side(*sd) for sd in P.sides] if P.sides is not None else None)
    O.set_threads(0)
    Q = np.ascontiguousarray(P.Q.copy())
    steps, t0 = 0, time.perf_counter()
    while True:
        O.step(cfg, Q, P.cfl)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= max_steps:
            break
    cells = P.nx * P.ny * 3 * steps
    rec = {"value": cells / el, "unit": "cell-stage updates/s", "cores": O.threads(),
           "cpu": cpu_model(), "kind": "oracle",
           "sample": f"{steps} whole SSP-RK3 steps of the same workload from its initial "
                     f"state ({cells} cell-stages) in {el:.1f} s, all host threads"}
    if one_thread:
        O.set_threads(1)
        Q0 = np.ascontiguousarray(P.Q.copy())
        dt = O.dt(cfg, Q0, P.cfl)
        t1 = time.perf_counter()
        O.rk_stage(cfg, 1, dt, Q0, Q0)
        el1 = time.perf_counter() - t1
        O.set_threads(0)
        rec["one_thread"] = {"value": P.nx * P.ny / el1, "unit": "cell-stage updates/s",
                             "cores": 1, "sample": f"one stage-1 call over the full grid "
                                                   f"({P.nx * P.ny} cell-stages) in {el1:.1f} s"}
    return rec, Q, steps


def calibration_copy(mib):
    """A plain device copy of known size (reads and writes `mib` MiB once), so
    rocprofv3 byte counters can be scaled against it."""
    import torch
    if not mib:
        return
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def batch_problems():
    from paper_2305_00762_amd import problems as PB
    out = []
    for fam, n, seed in PB.batch_spec(512, seed=0):
        out.append(PB.vortex(n, cfl=0.5) if fam == "vortex" else PB.make(fam, n, seed=seed))
    return out


def tg_diagnostics(Q, dx):
    """Kinetic energy <rho |u|^2 / 2> and enstrophy <rho |curl u|^2 / 2> of a
    periodic 3D state (host numpy; curl by second-order central differences)."""
    import numpy as np
    r = Q[0]
    u, v, w = Q[1] / r, Q[2] / r, Q[3] / r
    d = lambda f, ax: (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) / (2.0 * dx)
    # array axes (z, y, x) = (0, 1, 2)
    wx = d(w, 1) - d(v, 0)
    wy = d(u, 0) - d(w, 2)
    wz = d(v, 2) - d(u, 1)
    ke = float((0.5 * r * (u * u + v * v + w * w)).mean())
    ens = float((0.5 * r * (wx * wx + wy * wy + wz * wz)).mean())
    return ke, ens


def bench_3d(a, n):
    """The paper's 3D case: inviscid Taylor-Green vortex, 64^3, t = 0..10, at
    the requested GRB order with the other order run beside it: whole-run time,
    throughput, the sweep kernels' roofline, and the kinetic energy and
    enstrophy histories (the paper's comparison of fourth- and seventh-order
    GRB)."""
    import numpy as np
    import torch
    from paper_2305_00762_amd import gbr
    from paper_2305_00762_amd import problems as PB
    from paper_2305_00762_amd.solver import Solver3
    torch.cuda.set_device(0)
    s = torch.cuda.Stream()
    P = PB.taylor_green3d(n)
    cells = P.nx * P.ny * P.nz
    dx = 2.0 * np.pi / n
    head_order = 4 if a.path == "fp64_g4" else 7
    calibration_copy(a.calib_copy_mb)

    def history(order):
        """Steps to t = 10 with diagnostics at t = 1..10 (device time summed on
        the stream, read after batches that shrink near each target)."""
        with torch.cuda.stream(s):
            S = Solver3(P, stream=s, order=order, sweeps=SWEEPS3[a.sweeps3], fused_dt=True)
            tacc = torch.zeros(1, dtype=torch.float64, device="cuda")
        k0 = tg_diagnostics(P.Q, dx)
        hist, steps, batch = [], 0, 50
        for target in range(1, 11):
            while True:
                with torch.cuda.stream(s):
                    for _ in range(batch):
                        S.step()
                        tacc.add_(S.dt)
                steps += batch
                s.synchronize()
                t = float(tacc.item())
                if t >= target:
                    break
                batch = max(1, min(50, int((target - t) / float(S.dt.item()))))
            ke, ens = tg_diagnostics(S.state(), dx)
            hist.append({"t": t, "ke_ratio": ke / k0[0], "enstrophy_ratio": ens / k0[1]})
            batch = 50
        status = gbr.strerror(S.check())
        S.close()
        return hist, steps, status

    def timed(order, steps):
        return timed3(a, P, s, order, steps)

    out_orders = {}
    for order in ([head_order] + ([11 - head_order] if not a.no_compare else [])):
        hist, steps, st = history(order)
        ms, stage_ms, st2 = timed(order, steps)
        out_orders[order] = {"steps_to_t10": steps, "time_to_solution_s": ms * 1e-3,
                             "value": cells * 3 * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                             "stage_us": stage_ms * 1e3, "history": hist,
                             "status": st if st == st2 else f"{st}/{st2}"}
    h = out_orders[head_order]
    bpc = bytes_3d(a)
    achieved = bpc * cells / (h["stage_us"] * 1e-6) / 1e9
    out = {
        "metric": METRIC, "value": h["value"], "unit": "cell-stage updates/s", "n_gpus": 1,
        "steps": h["steps_to_t10"], "warmup": a.warmup, "ms_per_step": h["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "taylor_green3d", "description": WORKLOADS["taylor_green3d"][4],
                   "nx": n, "ny": n, "nz": n, "order": head_order, "sweeps": a.sweeps3,
                   "step": step_3d(a)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": kernel_3d(a), "avg_launch_us": h["stage_us"],
                     "bytes_per_cell_stage": bpc},
        "time_to_solution_s": h["time_to_solution_s"],
        "status": h["status"],
        "orders": {str(k): v for k, v in out_orders.items()},
    }
    if not a.no_cpu_baseline:
        import oracle as O
        cfg = O.make_cfg3(n, n, n, *P.geometry(), bc=P.bc, gamma=P.gamma, order=head_order)
        Q = np.ascontiguousarray(P.Q.copy())
        t0, k = time.perf_counter(), 0
        while time.perf_counter() - t0 < a.cpu_seconds and k < 50:
            O.step3(cfg, Q, P.cfl)
            k += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": cells * 3 * k / el, "unit": "cell-stage updates/s",
                               "cores": O.threads(), "cpu": cpu_model(), "kind": "oracle",
                               "sample": f"{k} whole SSP-RK3 steps of the same workload from its "
                                         f"initial state ({cells * 3 * k} cell-stages) in {el:.1f} s"}
        with torch.cuda.stream(s):
            S = Solver3(P, stream=s, order=head_order, sweeps=SWEEPS3[a.sweeps3], fused_dt=True)
            for _ in range(k):
                S.step()
        G = S.state()
        S.close()
        d = np.abs(G - Q).reshape(5, -1)
        out["error_vs_oracle"] = {"after_steps": k, "L1": d.mean(1).tolist(),
                                  "Linf": d.max(1).tolist(),
                                  "vars": ["rho", "rho_u", "rho_v", "rho_w", "E"]}
    print(json.dumps(out), flush=True)


def bytes_3d(a):
    return BYTES_PER_CELL_STAGE_3D if a.sweeps3 == "lines" else BYTES_PER_CELL_STAGE_3D_FUSED


def step_3d(a):
    dt = "dt (first step: reduction over Q^n; then from the stage-3 extrema)"
    if a.sweeps3 == "lines":
        return f"{dt} + 3 x (x, y, z line-sweep kernels)"
    return f"{dt} + 3 x (x/y kernel over z-plane tiles + z line-sweep kernel)"


def kernel_3d(a):
    if a.sweeps3 == "lines":
        return "meg7_sweep3_kernel (x, y, z per stage)"
    return "meg7_xy3_kernel + meg7_sweep3_kernel (z) per stage"


def timed3(a, P, s, order, steps):
    """Whole-step time of `steps` steps from the initial state (after warm-up
    steps), then the same steps again with events around every stage's
    kernels: (ms, ms per stage, status)."""
    import torch
    from paper_2305_00762_amd import gbr
    from paper_2305_00762_amd.solver import Solver3
    with torch.cuda.stream(s):
        S = Solver3(P, stream=s, order=order, sweeps=SWEEPS3[a.sweeps3], fused_dt=True)
        for _ in range(a.warmup):
            S.step()
    s.synchronize()
    S.set_state(P.Q)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        start.record(s)
        for _ in range(steps):
            S.step()
        stop.record(s)
    s.synchronize()
    ms = start.elapsed_time(stop)
    S.set_state(P.Q)
    torch.cuda.synchronize()
    gbr.gbr3_timing(S.ctx, True)
    with torch.cuda.stream(s):
        for _ in range(steps):
            S.step()
    sweep_ms, calls = gbr.gbr3_timing_read(S.ctx)
    gbr.gbr3_timing(S.ctx, False)
    st = gbr.strerror(S.check())
    S.close()
    return ms, sweep_ms / max(calls, 1), st


def bench_3d_fixed(a, n, steps):
    """The eight-octant 3D Riemann problem at n^3: a fixed number of steps from
    the initial state (whole-step throughput and the per-stage kernel time),
    the other launch form beside it, and the error against the oracle after a
    few steps."""
    import numpy as np
    import torch
    from paper_2305_00762_amd import problems as PB
    from paper_2305_00762_amd.solver import Solver3
    torch.cuda.set_device(0)
    s = torch.cuda.Stream()
    P = PB.riemann3d(n, seed=0)
    cells = P.nx * P.ny * P.nz
    calibration_copy(a.calib_copy_mb)
    ms, stage_ms, st = timed3(a, P, s, 7, steps)
    bpc = bytes_3d(a)
    achieved = bpc * cells / (stage_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": cells * 3 * steps / (ms * 1e-3), "unit": "cell-stage updates/s",
        "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "description": WORKLOADS[a.workload][4],
                   "nx": n, "ny": n, "nz": n, "order": 7, "sweeps": a.sweeps3,
                   "step": step_3d(a)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel_3d(a),
                     "avg_launch_us": stage_ms * 1e3, "bytes_per_cell_stage": bpc},
        "status": st,
    }
    if not a.no_compare:
        other = "lines" if a.sweeps3 != "lines" else "fused"
        b = argparse.Namespace(**vars(a))
        b.sweeps3 = other
        ms2, stage2, st2 = timed3(b, P, s, 7, steps)
        out["other_form"] = {"sweeps": other, "value": cells * 3 * steps / (ms2 * 1e-3),
                             "ms_per_step": ms2 / steps, "stage_us": stage2 * 1e3, "status": st2}
    if not a.no_cpu_baseline:
        import oracle as O
        cfg = O.make_cfg3(n, n, n, *P.geometry(), bc=P.bc, gamma=P.gamma, order=7)
        Q = np.ascontiguousarray(P.Q.copy())
        k = 3
        t0 = time.perf_counter()
        for _ in range(k):
            O.step3(cfg, Q, P.cfl)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": cells * 3 * k / el, "unit": "cell-stage updates/s",
                               "cores": O.threads(), "cpu": cpu_model(), "kind": "oracle",
                               "sample": f"{k} whole SSP-RK3 steps of the same workload from its "
                                         f"initial state ({cells * 3 * k} cell-stages) in {el:.1f} s"}
        with torch.cuda.stream(s):
            S = Solver3(P, stream=s, sweeps=SWEEPS3[a.sweeps3], fused_dt=True)
            for _ in range(k):
                S.step()
        G = S.state()
        S.close()
        d = np.abs(G - Q).reshape(5, -1)
        out["error_vs_oracle"] = {"after_steps": k, "L1": d.mean(1).tolist(),
                                  "Linf": d.max(1).tolist(),
                                  "vars": ["rho", "rho_u", "rho_v", "rho_w", "E"]}
    print(json.dumps(out), flush=True)


def bench_batch(a, steps):
    """The batched workload: FP32 bulk + FP64 state (plain detector), every
    stage of all 512 grids in one launch, steps replayed as a HIP graph."""
    import numpy as np
    import torch
    from paper_2305_00762_amd import gbr
    from paper_2305_00762_amd.solver import BatchSolver
    t0 = time.time()
    calibration_copy(a.calib_copy_mb)
    ps = batch_problems()
    cells = sum(p.nx * p.ny for p in ps)
    torch.cuda.set_device(0)
    s = torch.cuda.Stream()
    spec = PATHS[a.path]
    if spec["cons"] or spec["order"] != 7 or spec["mp_everywhere"]:
        print("bench.py: batched grids run seventh-order MEG7-prim; use --path fp64 or fp32",
              file=sys.stderr)
        sys.exit(2)
    prec = gbr.GBR_PREC_FP64 if a.path == "fp64" else gbr.GBR_PREC_FP32_BULK
    with torch.cuda.stream(s):
        B = BatchSolver(ps, precision=prec, stream=s)
    s.synchronize()
    for p in ps:
        p.Q = None if p.nx > 128 else p.Q        # keep only the initial states the oracle needs
    form = gbr.gbr_batch_autotune(B.b, 3, s) if a.tiling == "auto" else None
    if form is None:
        gbr.gbr_batch_set_tiling(B.b, int(a.tiling))
    form, tx, ty, total, wg = gbr.gbr_batch_info(B.b)
    with torch.cuda.stream(s):
        for _ in range(a.warmup):
            B.step()
    s.synchronize()
    if B.check() != gbr.GBR_OK:
        raise RuntimeError("device reported a bad state during warmup")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        start.record(s)
        for _ in range(steps):
            B.step()
        stop.record(s)
    s.synchronize()
    total_ms = start.elapsed_time(stop)
    status = gbr.strerror(B.check())
    value = cells * 3 * steps / (total_ms * 1e-3)
    # kernel durations: the same steps launched directly with per-stage events
    gbr.gbr_batch_timing(B.b, True)
    with torch.cuda.stream(s):
        for _ in range(steps):
            B.step()
    stage_ms, launches = gbr.gbr_batch_timing_read(B.b)
    gbr.gbr_batch_timing(B.b, False)
    done = a.warmup + 2 * steps
    avg_ms = stage_ms / max(launches, 1)
    achieved = 256.0 / 3.0 * cells / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "cell-stage updates/s", "n_gpus": 1,
        "steps": steps, "warmup": a.warmup, "ms_per_step": total_ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == gbr.GBR_PREC_FP32_BULK else "f64", "data": "synthetic",
        "config": {"workload": "batch512", "description": WORKLOADS["batch512"][4],
                   "grids": len(ps), "cells": cells, "path": "fp32" if prec else "fp64",
                   "launch_form": form, "tile": f"{tx}x{ty}", "tiles": total,
                   "workgroups_per_stage_launch": wg, "graph": True,
                   "setup_s": round(time.time() - t0, 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": load_traffic("meg7_batch_kernel", "batch512",
                                             path="fp32" if prec else "fp64",
                                             launch_form=form,
                                             tile=f"{tx}x{ty}"),
                     "kernel": "meg7_batch_kernel", "avg_launch_us": avg_ms * 1e3,
                     "bytes_per_cell_stage": 256.0 / 3.0},
        "status": status,
    }
    # the smallest grids against the oracle after the same number of steps
    small = sorted(range(len(ps)), key=lambda k: ps[k].nx * ps[k].ny)[:4]
    if not a.no_cpu_baseline:
        import oracle as O
        errs, t_cpu, cs = [], 0.0, 0
        st = B.states()
        for k in small:
            P = ps[k]
            cfg = O.make_cfg(P.nx, P.ny, *P.geometry(), gamma=P.gamma, mu=P.mu, Pr=P.Pr)
            Q = np.ascontiguousarray(P.Q.copy())
            t1 = time.perf_counter()
            for _ in range(done):
                O.step(cfg, Q, P.cfl)
            t_cpu += time.perf_counter() - t1
            cs += P.nx * P.ny * 3 * done
            d = np.abs(st[k].cpu().numpy() - Q).reshape(4, -1)
            errs.append({"grid": k, "family": P.family, "n": P.nx, "L1": d.mean(1).tolist(),
                         "Linf": d.max(1).tolist()})
        out["cpu_baseline"] = {"value": cs / t_cpu, "unit": "cell-stage updates/s",
                               "cores": O.threads(), "cpu": cpu_model(), "kind": "oracle",
                               "sample": f"the {len(small)} smallest grids of the batch, {done} "
                                         f"whole steps each ({cs} cell-stages) in {t_cpu:.1f} s"}
        out["error_vs_oracle"] = {"after_steps": done, "grids": errs}
    B.close()
    print(json.dumps(out), flush=True)


def run_path(P, path, stream, a, steps, t_final, weights=None, margin=None):
    """One path over the workload: a kernel pass with HIP events around every
    launch (per-kernel durations for the roofline; the events add gaps
    between launches), then the same work from the same initial state
    without them for the throughput.  Returns (record, final state, Path)."""
    from paper_2305_00762_amd import gbr
    cells = P.nx * P.ny
    h = Path(P, path, stream, a.tiling, weights, margin)
    if t_final is not None:
        # the whole run of the test case: warm-up steps, then from the
        # initial state at t = 0 until the device clock reaches t_final,
        # timed; the kernel pass repeats the same number of steps
        h.run(a.warmup, 0)
        h.reset()
        total_ms, steps = h.run_to(t_final)
        Qf = h.Q[0].clone()
        t_reached = gbr.gbr_get_time(h.ctx)
        status = h.status
        h.reset()
        ev_ms, (det_ms, stage_ms, launches) = h.run(0, steps, timing=True)
    else:
        ev_ms, (det_ms, stage_ms, launches) = h.run(a.warmup, steps, timing=True)
        h.reset()
        total_ms, _ = h.run(a.warmup, steps)
        Qf = h.Q[0].clone()
        status = h.status
        t_reached = None
    rec = {"value": cells * 3 * steps / (total_ms * 1e-3), "ms_per_step": total_ms / steps,
           "steps": steps, "tile": f"{h.tile[1]}x{h.tile[2]}", "status": gbr.strerror(status),
           "ms_per_step_with_kernel_events": ev_ms / steps,
           "kernels_us_per_launch": {
               "stage": stage_ms * 1e3 / max(launches, 1),
               # per stage call: the flag map's time summed over the step's
               # evaluations, divided by the three stage calls
               "detector_flag_map": (det_ms * 1e3 / max(launches, 1) if h.net is not None
                                     else None)},
           "_stage_ms": stage_ms, "_det_ms": det_ms, "_launches": launches,
           "_total_ms": total_ms}
    if t_final is not None:
        rec["time_to_solution_s"] = total_ms * 1e-3
        rec["t_final"] = t_final
        rec["t_reached"] = t_reached
    if h.net is not None:
        ev, fb = gbr.gbr_mlp_stats(h.ctx, reset=True)
        rec["detector_fallback_rate"] = fb / max(ev, 1)
        rec["detector_evaluations_per_step"] = (2 if PATHS[path]["per_step"] else 6) * cells
    return rec, Qf, h


def detector_vs_plain(P, h, Q):
    """Interface flags of the path's learned detector against the plain
    detector's (Sec. 2.4) on the same state Q: the fraction of x and y
    interfaces that differ, and the fraction the plain detector flags."""
    import numpy as np
    import torch
    from paper_2305_00762_amd import gbr
    R = torch.empty_like(Q)
    sx = np.zeros((P.ny, P.nx + 1), np.uint8)
    sy = np.zeros((P.ny + 1, P.nx), np.uint8)
    gbr.gbr_export_flags(h.ctx, True)
    gbr.gbr_residual(h.ctx, Q, R, h.stream.cuda_stream)
    gbr.gbr_get_flags(h.ctx, sx, sy, h.stream.cuda_stream)
    gbr.gbr_export_flags(h.ctx, False)
    ctx = gbr.gbr_init(P.nx, P.ny, P.gamma, P.mu, P.Pr)
    gbr.gbr_set_geometry(ctx, *P.geometry())
    gbr.gbr_set_scheme(ctx, gbr.GBR_RECON_PRIM, gbr.GBR_MP_FLAGGED, gbr.GBR_PREC_FP32_BULK,
                       gbr.GBR_DET_PLAIN)
    gbr.gbr_export_flags(ctx, True)
    gbr.gbr_residual(ctx, Q, R, h.stream.cuda_stream)
    px = np.zeros_like(sx)
    py = np.zeros_like(sy)
    gbr.gbr_get_flags(ctx, px, py, h.stream.cuda_stream)
    gbr.gbr_destroy(ctx)
    tot = px.size + py.size
    return {"interface_flag_mismatch": (int((px != sx).sum()) + int((py != sy).sum())) / tot,
            "plain_flagged_fraction": (int((px == 0).sum()) + int((py == 0).sum())) / tot,
            "on": "the final state of the timed steps"}


def public(rec):
    return {k: v for k, v in rec.items() if not k.startswith("_")}


def compare_paths(head_path):
    """Paths run beside the headline one: the plain FP64 path always (first:
    the others' errors are taken against it); the FP32-bulk path with the
    plain detector for an FP32-bulk headline; the learned detector once per
    step beside the per-stage one and the reverse."""
    out = ["fp64"] if head_path != "fp64" else []
    if PATHS[head_path]["prec"] == "fp32" and head_path != "fp32":
        out.append("fp32")
    if head_path == "fp32_mlp_step":
        out.append("fp32_mlp")
    if head_path == "fp32_mlp":
        out.append("fp32_mlp_step")
    return out


COMPARE_KEY = {"fp64": "fp64_plain", "fp32": "fp32_plain", "fp32_mlp": "fp32_mlp_per_stage",
               "fp32_mlp_step": "fp32_mlp_per_step"}


def bench_2d(a, workload, steps_arg, stream, cpu=True, secondary=False):
    """The record of one 2D workload: the headline path, its roofline, the
    comparison paths and (cpu) the oracle baseline."""
    import torch
    from paper_2305_00762_amd import problems as PB
    fam, n, seed, wsteps, desc = WORKLOADS[workload]
    steps = steps_arg if steps_arg is not None else wsteps
    P = PB.make(fam, n, seed=seed) if fam != "vortex" else PB.vortex(n, cfl=0.5)
    cells = P.nx * P.ny
    t_final = P.t_final if steps is None else None
    head_rec, Qhead, head = run_path(P, a.path, stream, a, steps, t_final, a.weights, a.margin)
    steps = head_rec["steps"]
    stage_ms, launches = head_rec["_stage_ms"], head_rec["_launches"]
    # roofline of the dominant kernel (the stage kernel): algorithmic bytes of
    # the timed launches over their summed duration from the library's events
    alg_bytes = sum(BYTES_PER_CELL_STAGE.values()) * cells * steps
    achieved = alg_bytes / (stage_ms * 1e-3) / 1e9
    kname = head.kernel.replace("<", "_").replace(">", "")
    out = {
        "value": head_rec["value"],
        "ms_per_step": head_rec["ms_per_step"],
        "steps": steps,
        "config": {"workload": workload, "description": desc, "nx": P.nx, "ny": P.ny,
                   "path": a.path, "tile": head_rec["tile"],
                   "detector": ("learned, evaluated once per step on Q^n and reused by stages 2 "
                                "and 3 (a change of the method; its error is reported)"
                                if PATHS[a.path]["per_step"] else
                                "learned, evaluated at every stage" if PATHS[a.path]["mlp"]
                                else "plain (Sec. 2.4)"),
                   "step": "dt (first step: reduction over Q^n; then from the stage-3 extrema) + "
                           "3 x (learned-detector flag map if selected and due + fused "
                           "residual/stage kernel)"},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": load_traffic(kname, workload, tile=head_rec["tile"]),
            "kernel": head.kernel,
            "avg_launch_us": stage_ms * 1e3 / max(launches, 1),
            "bytes_per_cell_stage": 256.0 / 3.0,
        },
        # the same kernel against the VALU issue roofline (its intensity, ~1500
        # lane-operations per 85 B, lies far right of the ridge): issued lane
        # operations (SQ_INSTS_VALU x 64, from the committed counter summary)
        # over the live launch duration
        "roofline_valu": valu_roofline(head.kernel, workload, stage_ms * 1e3 / max(launches, 1)),
        "status": head_rec["status"],
    }
    out.update({k: v for k, v in public(head_rec).items()
                if k not in ("value", "ms_per_step", "steps", "tile", "status")})
    if head.net is not None and head_rec["_det_ms"] > 0:
        # flag map: reads Q (32 B) and writes one byte per cell, per evaluation;
        # evaluated once per step, it reads after the first step the float32
        # (rho, p) the previous stage 3 stored (8 B)
        per_step = PATHS[a.path]["per_step"]
        evals = steps * (1 if per_step else 3)
        nbytes = (33.0 + 9.0 * (steps - 1)) if per_step else 33.0 * evals
        out["detector_flag_map_GBs"] = nbytes * cells / (head_rec["_det_ms"] * 1e-3) / 1e9
        out["detector_vs_plain"] = detector_vs_plain(P, head, Qhead)
    head.close()

    if not a.no_compare:
        base_Q = None
        for cp in compare_paths(a.path):
            rec, Qc, h = run_path(P, cp, stream, a, steps if t_final is None else None, t_final)
            h.close()
            key = COMPARE_KEY.get(cp, cp)
            out[key] = public(rec)
            out[f"speedup_vs_{key}"] = out["value"] / rec["value"]
            if t_final is not None:
                out[f"time_to_solution_ratio_vs_{key}"] = (head_rec["_total_ms"] /
                                                          rec["_total_ms"])
            if cp == "fp64":
                base_Q = Qc
            else:
                if base_Q is not None:
                    l1, linf = diff(Qc, base_Q)
                    out[key]["error_vs_fp64_plain"] = {"L1": l1, "Linf": linf}
                del Qc
        if base_Q is not None:
            l1, linf = diff(Qhead, base_Q)
            after = f"t = {t_final}" if t_final is not None else a.warmup + steps
            out["error_vs_fp64_plain"] = {"after_steps": after, "L1": l1, "Linf": linf,
                                          "vars": ["rho", "rho_u", "rho_v", "E"]}
            del base_Q
    del Qhead
    torch.cuda.empty_cache()

    if cpu:
        rec, Qo, osteps = cpu_baseline(P, a.cpu_seconds, recon=1 if PATHS[a.path]["cons"] else 0,
                                       order=PATHS[a.path]["order"],
                                       mp_mode=1 if PATHS[a.path]["mp_everywhere"] else 0)
        out["cpu_baseline"] = rec
        h = Path(P, a.path, stream, a.tiling, a.weights, a.margin)
        h.run(osteps, 0)
        l1, linf = diff(h.Q[0].cpu(), torch.from_numpy(Qo))
        h.close()
        out["error_vs_oracle"] = {"after_steps": osteps, "L1": l1, "Linf": linf,
                                  "vars": ["rho", "rho_u", "rho_v", "E"],
                                  "oracle": "plain method (Sec. 2.4 detector), FP64"}
    return out


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; the decomposition over several GPUs (halo "
              "exchange per stage, one min-reduction of the time step) is designed, not "
              "built; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    fam, n, seed, wsteps, desc = WORKLOADS[a.workload]
    steps = a.steps if a.steps is not None else wsteps
    if fam == "batch":
        return bench_batch(a, steps)
    if fam == "taylor_green3d":
        return bench_3d(a, n)
    if fam == "riemann3d":
        return bench_3d_fixed(a, n, steps)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    calibration_copy(a.calib_copy_mb)
    rec = bench_2d(a, a.workload, a.steps, stream, cpu=not a.no_cpu_baseline)
    out = {"metric": METRIC, "value": rec.pop("value"), "unit": "cell-stage updates/s",
           "n_gpus": 1, "steps": rec.pop("steps"), "warmup": a.warmup,
           "ms_per_step": rec.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": PATHS[a.path]["dtype"], "data": "synthetic"}
    out.update(rec)
    if a.workload == "riemann4096" and not a.no_secondary:
        # the other evaluation field of the learned detector, reported beside
        out["shear4096"] = bench_2d(a, "shear4096", a.steps, stream, cpu=False)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
