"""Throughput benchmark: TVD-RK3 steps of the FP64 WENO5-JS/HLLC/viscous
right-hand side on decaying isotropic turbulence at 256^3 (one MI355X).

python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line: Mcell-updates/s over exactly K steps (inputs resident in
HBM, timed between device synchronisations), the roofline of the dominant
kernel (its duration measured live with HIP events inside the library, its
algorithmic flops from the operation-count table paper_2203_13760_amd/opcounts.json,
written by oracle/write_opcounts.py), and the CPU oracle
timed on a bounded slab of the same field on one host core.

--copy-bytes N runs only a plain device-to-device copy of N bytes (the
calibration of the HBM traffic counters) and exits.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X_FP64_VECTOR_PEAK = 78.6e12  # 256 CUs x 2.4 GHz x 128 FP64 flops/clock (FMA = 2)
MI355X_HBM_PEAK = 8.0e12
# per cell, per axis: R -= (G+ - G-)/dx for 5 variables (3 flops each); per
# cell: the stage combination a Un + b (Uk + dt R) for 5 variables (4 each)
DIVERGENCE_FLOPS_PER_CELL_AXIS = 15
RK_FLOPS_PER_CELL = 20
KERNELS = ("k_prim", "k_grad", "k_sweep_x", "k_sweep_y", "k_sweep_z")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="grid side (the headline case is 256)")
    ap.add_argument("--reps", type=int, default=5, help="kernel-timing repetitions")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slab", type=int, default=24, help="z-planes of the oracle's timed slab")
    ap.add_argument("--copy-bytes", type=int, default=0)
    return ap.parse_args()


def copy_calibration(nbytes):
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "read_KiB": n * 8 / 1024, "write_KiB": n * 8 / 1024}),
          flush=True)


def cpu_baseline(case, W, nz):
    """The oracle as it stands, one TVD-RK3 step on a periodic slab of the
    benchmark field (full x-y planes, nz z-planes), single-threaded."""
    import numpy as np
    import oracle
    sub = dict(case)
    n = case["n"]
    dz = (case["hi"][2] - case["lo"][2]) / n[2]
    sub["n"] = (n[0], n[1], nz)
    sub["hi"] = (case["hi"][0], case["hi"][1], case["lo"][2] + dz * nz)
    Ws = np.ascontiguousarray(W[:, :nz])
    U = oracle.state_init(sub, Ws)
    dt = oracle.cfl_dt(sub, U)
    t0 = time.perf_counter()
    oracle.rk3_step(sub, U, dt)
    sec = time.perf_counter() - t0
    cells = n[0] * n[1] * nz
    return {"value": cells / sec / 1e6, "unit": "Mcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 TVD-RK3 step of the serial oracle on a {n[0]}x{n[1]}x{nz} periodic slab "
                      f"of the same field ({cells} cell-updates, {sec:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is a "
              "design, not a build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    from paper_2203_13760_amd import cfd
    from paper_2203_13760_amd import workloads as wl
    from paper_2203_13760_amd.solver import Solver

    torch.cuda.set_device(0)
    n = args.n
    case, W = wl.isotropic_turbulence(n, seed=2203)
    print(f"bench: HIT {n}^3 seed 2203, mu={case['mu']:.6g}, p0={case['stats']['p0']:.6g}", flush=True)
    s = Solver(case)
    U = s.init(W)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    if args.warmup:
        s.advance(U, args.warmup, t=t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(U, args.steps, t=t)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    health = s.check()
    cells = n ** 3
    value = cells * args.steps / sec / 1e6
    ms_per_step = sec / args.steps * 1e3
    print(f"bench: {args.steps} steps in {sec:.4f} s, {value:.1f} Mcell-updates/s, health {health}",
          flush=True)

    # live per-kernel durations (HIP events around each kernel of one stage)
    ms = cfd.cfd_profile_stage(s.h, U, args.reps)
    dom = int(np.argmax(ms))
    with open(os.path.join(ROOT, "paper_2203_13760_amd", "opcounts.json")) as f:
        parts = json.load(f)["3d_viscous_heat"]
    face = parts["face_flux"]
    faces_per_axis = (n + 1) * n * n
    flops = {
        0: parts["prim_per_cell"] * (n + 6) ** 3,
        1: 45.0 * (n + 6) ** 3,  # 9 fourth-order centred derivatives, 5 flops each
        2: face * faces_per_axis + DIVERGENCE_FLOPS_PER_CELL_AXIS * cells,
        3: face * faces_per_axis + DIVERGENCE_FLOPS_PER_CELL_AXIS * cells,
        4: face * faces_per_axis + (DIVERGENCE_FLOPS_PER_CELL_AXIS + RK_FLOPS_PER_CELL) * cells,
    }[dom]
    achieved = flops / (ms[dom] * 1e-3)
    roofline = {"bound": "alu", "kernel": KERNELS[dom], "achieved": achieved / 1e12,
                "peak": MI355X_FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / MI355X_FP64_VECTOR_PEAK, "traffic": None,
                "kernel_ms": {k: round(v, 4) for k, v in zip(KERNELS, ms)},
                "flops_per_launch": flops}
    # whole-step view: algorithmic flops per cell-update over the measured step time
    step_flops = 3 * (3 * face * (n + 1) / n + parts["prim_per_cell"] * ((n + 6) / n) ** 3
                      + 45.0 * ((n + 6) / n) ** 3 + 3 * DIVERGENCE_FLOPS_PER_CELL_AXIS + RK_FLOPS_PER_CELL)
    s.close()
    del U
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, W, args.cpu_slab)
        print(f"bench: cpu oracle {cpu['value']:.4f} Mcell-updates/s", flush=True)

    out = {
        "metric": "Mcell-updates/s per RK3 step FP64 at 256^3",
        "value": value,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"decaying compressible isotropic turbulence {n}^3, periodic, "
                               "E(k)~k^4 exp(-2(k/4)^2), Mt 0.3, Re_lambda 100, seed 2203; "
                               "WENO5-JS + HLLC/Einfeldt + 4th-order viscous/heat + TVD-RK3, CFL 0.5",
                   "grid": [n, n, n], "cells": cells, "parallelism": "single GPU"},
        "roofline": roofline,
        "step_flops_per_cell_update": step_flops,
        "step_tflops": step_flops * cells * args.steps / sec / 1e12,
        "fused_min_traffic_GBps": 320.0 * value * 1e6 / 1e9,
        "cpu_baseline": cpu,
        "paper_context": {"value": 1000.0 / 92.76, "unit": "Mcell-updates/s",
                          "workload": "Taylor-Green vortex 256^3, HLLC float64, JAX on one RTX A6000"},
        "health": health,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
