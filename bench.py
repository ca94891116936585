"""Throughput of the MEG7 hot path on one MI355X: cell-stage updates/s.

A step is one SSP-RK3 time step of the whole hot path on the workload: the
device time step (CFL reduction) and three fused residual + stage-update
launches.  Inputs are resident in HBM before the timed region.  Prints ONE
JSON line (see the keys below).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload riemann1024]
                  [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-stage updates/s, FP32+MLP-detector vs FP64 plain, at stated L1 error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_VECTOR_PEAK_TF = 78.6     # MI355X FP64 vector, published

# algorithmic HBM bytes per cell and launch: read Q^(k) (32 B), write Q^(k+1)
# (32 B), and Q^n (32 B) in stages 2 and 3.
BYTES_PER_CELL_STAGE = {1: 64.0, 2: 96.0, 3: 96.0}

WORKLOADS = {
    # name: (family, n, seed, description)
    "riemann1024": ("riemann", 1024, 0,
                    "2D Euler four-quadrant Riemann problem, 1024x1024, seed 0, transmissive, "
                    "FP64 plain method, CFL 0.2"),
    "vortex64": ("vortex", 64, 0, "2D Euler isentropic vortex 64x64 periodic, CFL 0.5"),
    "shear2048": ("shear", 2048, 0,
                  "2D Navier-Stokes periodic shear layer 2048x2048, Re 1e4, Pr 0.72, CFL 0.2"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="riemann1024", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--tiling", default="auto",
                    help="tile variant index, or 'auto' (gbr_autotune on the initial state)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    return ap.parse_args()


def load_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if any."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and line.strip().startswith("bytes_per_launch"):
            k, v = line.split("=", 1)
            vals[k.strip()] = float(v.split()[0])
    return vals.get("bytes_per_launch")


def cpu_baseline(P, seconds):
    """The CPU oracle on a bounded sample of the same workload: whole SSP-RK3
    steps on the full grid until about `seconds` of host time have passed."""
    import numpy as np
    import oracle as O
    cfg = O.make_cfg(P.nx, P.ny, *P.geometry(), gamma=P.gamma, mu=P.mu, Pr=P.Pr)
    Q = np.ascontiguousarray(P.Q.copy())
    steps, t0 = 0, time.perf_counter()
    while True:
        O.step(cfg, Q, P.cfl)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    cells = P.nx * P.ny * 3 * steps
    return {"value": cells / el, "unit": "cell-stage updates/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps ({cells} cell-stages) of the same workload, "
                      f"{el:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU decomposition is "
              "a design in DESIGN.md, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2305_00762_amd import gbr
    from paper_2305_00762_amd import problems as PB

    fam, n, seed, desc = WORKLOADS[a.workload]
    P = PB.make(fam, n, seed=seed) if fam != "vortex" else PB.vortex(n, cfl=0.5)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    ctx = gbr.gbr_init(P.nx, P.ny, P.gamma, P.mu, P.Pr)
    gbr.gbr_set_geometry(ctx, *P.geometry())
    prec = gbr.GBR_PREC_FP32_BULK if a.precision == "fp32" else gbr.GBR_PREC_FP64
    gbr.gbr_set_scheme(ctx, gbr.GBR_RECON_PRIM, gbr.GBR_MP_FLAGGED, prec, gbr.GBR_DET_PLAIN)
    Qs = [torch.from_numpy(P.Q).to(dev) for _ in range(3)]
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    if a.tiling == "auto":
        gbr.gbr_autotune(ctx, Qs[0], 5, sh)
    else:
        gbr.gbr_set_tiling(ctx, int(a.tiling))
    tiling = gbr.gbr_get_tiling(ctx)
    if a.calib_copy_mb:
        # a plain copy of known size: reads and writes calib_copy_mb MiB once
        src = torch.ones(a.calib_copy_mb << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def one_step(Q, Q1, Q2, ev=None):
        gbr.gbr_compute_dt(ctx, Q, P.cfl, dt, sh)
        for st, (src, dst) in enumerate(((Q, Q1), (Q1, Q2), (Q2, Q1)), start=1):
            if ev is not None:
                ev[st][0].record(stream)
            gbr.gbr_rk_stage(ctx, st, dt, Q, src, dst, sh)
            if ev is not None:
                ev[st][1].record(stream)
        return Q1, Q, Q2        # Q^{n+1} is in Q1

    Q, Q1, Q2 = Qs
    with torch.cuda.stream(stream):
        for _ in range(a.warmup):
            Q, Q1, Q2 = one_step(Q, Q1, Q2)
    stream.synchronize()
    if gbr.gbr_check(ctx, sh) != gbr.GBR_OK:
        raise RuntimeError("device reported a bad state during warmup")

    # timed region: K whole steps, events around every stage launch
    evs = [[None, None]] + [[[torch.cuda.Event(enable_timing=True) for _ in range(2)]
                             for _ in range(a.steps)] for _ in range(3)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        start.record(stream)
        for k in range(a.steps):
            ev = [None] + [evs[s][k] for s in (1, 2, 3)]
            Q, Q1, Q2 = one_step(Q, Q1, Q2, ev)
        stop.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    status = gbr.gbr_check(ctx, sh)
    cells = P.nx * P.ny
    value = cells * 3 * a.steps / (total_ms * 1e-3)

    stage_ms = {s: sum(e[0].elapsed_time(e[1]) for e in evs[s]) / a.steps for s in (1, 2, 3)}
    launches = 3 * a.steps
    stage_total_s = sum(stage_ms.values()) * a.steps * 1e-3
    alg_bytes = sum(BYTES_PER_CELL_STAGE[s] for s in (1, 2, 3)) * cells * a.steps
    achieved = alg_bytes / stage_total_s / 1e9
    traffic = load_traffic("meg7_stage_fp64", a.workload)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": total_ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "description": desc, "nx": P.nx, "ny": P.ny,
                   "precision": a.precision, "detector": "plain",
                   "step": "device dt + 3 fused residual/stage launches",
                   "tile": f"{tiling[1]}x{tiling[2]}"},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "meg7_stage_kernel" + ("_f32" if a.precision == "fp32" else "") + f" ({a.precision})",
            "avg_launch_ms": stage_total_s * 1e3 / launches,
            "stage_ms": stage_ms,
            "bytes_per_cell_stage": 256.0 / 3.0,
        },
        "status": gbr.strerror(status),
    }
    gbr.gbr_destroy(ctx)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
