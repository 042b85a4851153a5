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
GRADIENT_FLOPS_PER_CELL = 45  # 9 fourth-order centred velocity derivatives, 5 flops each
KERNELS = ("k_prim", "k_sweep_x", "k_sweep_y", "k_sweep_z", "k_prim_halo")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hit256_traffic.txt")


def kernel_sources_hash():
    """sha256 over the kernel sources (file name + bytes, sorted by name)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2203_13760_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n):
    """Calibrated HBM bytes per dispatch from the committed rocprofv3 counter
    summary, or None when it does not describe this grid or these kernels."""
    if n != 256 or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    out = {}
    for k in KERNELS:
        if f"{k}.read_bytes" in vals:
            out[k] = (float(vals[f"{k}.read_bytes"]), float(vals[f"{k}.write_bytes"]))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="grid side (the headline case is 256)")
    ap.add_argument("--reps", type=int, default=30, help="kernel-timing repetitions (stages 1, 2, 3 in turn)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slab", type=int, default=48, help="z-planes of the oracle's timed slab")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation measurement")
    ap.add_argument("--adj-n", type=int, default=128)
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--no-roe", action="store_true", help="skip the ROE setup and WENO5-Z legs")
    ap.add_argument("--no-implosion", action="store_true", help="skip the implosion (Rusanov vs HLLC) leg")
    ap.add_argument("--nn-epochs", type=int, default=1,
                    help="epochs of the Rusanov-NN training in the implosion leg (0 skips it)")
    ap.add_argument("--roe-steps", type=int, default=10)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg (batched vs one at a time)")
    ap.add_argument("--serving", action="store_true",
                    help="run the serving benchmark (batched vs one at a time) instead")
    ap.add_argument("--serving-requests", type=int, default=400)
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--serving-steps", type=int, default=200)
    ap.add_argument("--serving-sweep", type=str, default="",
                    help="comma-separated extra arrival rates for a load sweep (batched only)")
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
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": cells / sec / 1e6, "unit": "Mcell-updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"1 TVD-RK3 step of the serial oracle on a {n[0]}x{n[1]}x{nz} periodic slab "
                      f"of the same field ({cells} cell-updates, {sec:.1f} s)"}


def differentiation(n, nsteps, ckpt_every=20, reps=5):
    """Cost of the discrete adjoint on the Taylor-Green vortex with seeded noise
    (sigma 1e-3) at n^3: one fixed-dt TVD-RK3 step vs one step adjoint applied
    to a seeded Gaussian cotangent, the adjoint either recomputing its two
    inner stages or taking the primitives of its three stage inputs from a
    step that kept them (cfd_rk3_step_prims), each timed with
    torch events on the stream the library launches on; and the full gradient
    of the final kinetic energy through an n_steps rollout with checkpoints
    every ckpt_every steps (kept stages, and recomputed stages)."""
    import torch
    from paper_2203_13760_amd import workloads as wl
    from paper_2203_13760_amd.autograd import rollout, state_init
    from paper_2203_13760_amd.experiments import kinetic_energy
    from paper_2203_13760_amd.solver import Solver
    case, W = wl.taylor_green_noisy(n, sigma=1e-3, seed=4)
    s = Solver(case)
    U = s.init(W)
    dt = float(s.compute_dt(U).item())
    # a dense seeded cotangent (a uniform one has zero face differences)
    gen = torch.Generator(device="cuda").manual_seed(4)
    Ub = torch.randn(U.shape, generator=gen, dtype=torch.float64, device="cuda")
    out = torch.empty_like(U)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    s.step(U, dt)
    s.step_adjoint(U, dt, Ub, out)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        s.step(U, dt)
    ev[1].record()
    for _ in range(reps):
        s.step_adjoint(U, dt, Ub, out)
    ev[2].record()
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / reps
    adj = ev[1].elapsed_time(ev[2]) / reps
    # the rollout's kept stages: the primitives of the three stage inputs
    Pk = s.empty_stage_prims()
    s.step_prims(U, dt, Pk)
    s.step_adjoint_prims(Pk, dt, Ub, out)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        s.step_prims(U, dt, Pk)
    ev[1].record()
    for _ in range(reps):
        s.step_adjoint_prims(Pk, dt, Ub, out)
    ev[2].record()
    torch.cuda.synchronize()
    fwd_keep = ev[0].elapsed_time(ev[1]) / reps
    adj_kept = ev[1].elapsed_time(ev[2]) / reps
    del Pk
    tgrad = {}
    for keep in (True, False):
        Wt = torch.from_numpy(W).cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = kinetic_energy(s, rollout(state_init(s, Wt), s, dt, nsteps, ckpt_every,
                                      keep_stages=keep))
        L.backward()
        torch.cuda.synchronize()
        tgrad[keep] = time.perf_counter() - t0
        if keep:
            gnorm = float(Wt.grad[1:4].norm().item())
    s.close()
    # the paper's gradient check: d(Delta S)/dM_S of a Mach 2 shock after 5 steps,
    # adjoint against central differences (least-squares order over the steps)
    import numpy as np
    from paper_2203_13760_amd.experiments import shock_entropy_gradient
    sg = shock_entropy_gradient()
    sg["fd_order"] = float(np.polyfit(np.log(sg["eps"]), np.log(sg["fd_error"]), 1)[0])
    return {"workload": f"Taylor-Green vortex {n}^3 + Gaussian noise 1e-3 (seed 4), fixed dt {dt:.4g}",
            "step_ms": fwd, "step_adjoint_ms": adj, "adjoint_over_step": adj / fwd,
            "step_keeping_stages_ms": fwd_keep, "step_adjoint_kept_stages_ms": adj_kept,
            "adjoint_kept_stages_over_step": adj_kept / fwd,
            "gradient_steps": nsteps, "checkpoint_every": ckpt_every, "gradient_s": tgrad[True],
            "gradient_recomputing_stages_s": tgrad[False],
            "loss": float(L.item()), "grad_norm": gnorm, "shock_gradient": sg}


def implosion_leg(nn_epochs=1):
    """The implosion of §7.4 (the Rusanov-NN experiment's data): the 128^2
    ground truth (WENO3-JS, TVD-RK2, HLLC, dt 2.5e-4) coarse-grained onto 32^2
    every 1e-3, against the 32^2 solvers with the classical Rusanov flux and
    with HLLC, over the paper's 2500 coarse steps: relative L1 errors of
    density and pressure (the quantity of the paper's error figure)."""
    import numpy as np
    from paper_2203_13760_amd.experiments import implosion_trajectories
    out = implosion_trajectories(n_cg_steps=2500, every=100)
    keys = ("rusanov_rho", "rusanov_p", "hllc_rho", "hllc_p")
    pick = {}
    for t in (0.1, 1.0, 2.5):
        i = int(np.argmin(np.abs(np.array(out["t"]) - t)))
        pick[f"t={t}"] = {k: out[k][i] for k in keys}
    res = {"workload": "implosion of §7.4 as printed, 128^2 truth coarse-grained to 32^2, 2500 coarse steps",
           "coarse_steps": 2500, "seconds": out["seconds"], "health": out["health"],
           "mean": {k: float(np.mean(out[k])) for k in keys}, "at": pick}
    if nn_epochs > 0:
        # the Rusanov-NN flux trained on the first 1000 coarse steps (windows of 15
        # steps, batches of 20, Adam 5e-4; the paper trains 200 epochs)
        from paper_2203_13760_amd.experiments import train_rusanov_nn
        nn = train_rusanov_nn(epochs=nn_epochs, n_eval=2500, every=100, log=None)
        at = {}
        for t in (0.1, 1.0, 2.5):
            i = int(np.argmin(np.abs(np.array(nn["after"]["step"]) * 1e-3 - t)))
            at[f"t={t}"] = {"nn_rho": nn["after"]["rho"][i], "nn_p": nn["after"]["p"][i],
                            "rusanov_rho": nn["rusanov"]["rho"][i], "rusanov_p": nn["rusanov"]["p"][i]}
        res["rusanov_nn"] = {
            "epochs": nn_epochs, "batches": nn["batches"], "train_seconds": nn["train_seconds"],
            "seconds_per_batch": nn["seconds_per_batch"], "epoch_loss": nn["epoch_loss"],
            "at": at, "health": nn["after"]["health"],
            "mean": {"nn_rho": float(np.mean(nn["after"]["rho"])), "nn_p": float(np.mean(nn["after"]["p"])),
                     "untrained_rho": float(np.mean(nn["before"]["rho"])),
                     "rusanov_rho": float(np.mean(nn["rusanov"]["rho"])),
                     "rusanov_p": float(np.mean(nn["rusanov"]["p"]))}}
    return res


def scheme_leg(case, W, steps, reps, hllc_ms_per_step, flag):
    """Another convective scheme (a configuration flag) on the same field and
    grid: CFL steps per second and the stage kernels' durations."""
    import torch
    from paper_2203_13760_amd import cfd
    from paper_2203_13760_amd.solver import Solver
    case = dict(case)
    case["flags"] = case["flags"] | flag
    n = case["n"][0]
    s = Solver(case)
    try:
        U = s.init(W)
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        s.advance(U, 2, t=t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(U, steps, t=t)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ms = cfd.cfd_profile_stage(s.h, U, reps)
        health = s.check()
    finally:
        s.close()
    ms_per_step = sec / steps * 1e3
    return {"value": n ** 3 * steps / sec / 1e6, "unit": "Mcell-updates/s", "steps": steps,
            "ms_per_step": ms_per_step, "over_hllc": ms_per_step / hllc_ms_per_step,
            "kernel_ms": {k: round(v, 4) for k, v in zip(KERNELS, ms)}, "health": health}


def roe_leg(case, W, steps, reps, hllc_ms_per_step):
    """The paper's ROE setup (Roe flux splitting, WENO5-JS in characteristic
    space) on the same field and grid."""
    from paper_2203_13760_amd import workloads as wl
    out = scheme_leg(case, W, steps, reps, hllc_ms_per_step, wl.ROE)
    out["paper_context"] = {"value": 1000.0 / 760.09, "unit": "Mcell-updates/s",
                            "workload": "256^3, ROE float64, JAX on one RTX A6000 (8.2 x its HLLC step)"}
    return out


def serving_leg(requests, rate, steps):
    """The serving workload (seeded Poisson arrivals of mixed 2D Kelvin-Helmholtz /
    3D Taylor-Green solves): continuous batching against the same server with
    one resident solve at a time; p50/p99 time to solution and throughput."""
    from paper_2203_13760_amd import serving
    srv = serving.BatchServer(max_grids=256, arena_bytes=96 << 30)
    try:
        srv.run(serving.mixed_workload(8, 1000.0, seed=99, steps=3, kh_range=(64, 96), tgv_range=(32, 40)))
        mk = lambda: serving.mixed_workload(requests, rate, seed=3, steps=steps)
        batched = srv.run(mk())
        single = srv.run(mk(), max_resident=1)
    finally:
        srv.close()
    return {"workload": f"{requests} requests, Poisson {rate}/s (seed 3), 60% KH 2D n in [64,1024], "
                        f"40% TGV 3D n in [32,128], {steps} TVD-RK3 CFL steps each",
            "p50_s": batched["p50_s"], "p99_s": batched["p99_s"],
            "throughput_ratio": batched["throughput_req_s"] / single["throughput_req_s"],
            "batched": batched, "one_at_a_time": single}


def serving_bench(args):
    """Continuous-batching serving of mixed 2D Kelvin-Helmholtz / 3D Taylor-Green
    solves (seeded Poisson arrivals): batched persistent launches vs the same
    kernels and graph with one resident solve, p50/p99 time to solution."""
    import torch
    from paper_2203_13760_amd import serving
    torch.cuda.set_device(0)
    srv = serving.BatchServer(max_grids=256, arena_bytes=96 << 30)
    # warm-up: a handful of small requests through both paths
    srv.run(serving.mixed_workload(8, 1000.0, seed=99, steps=3, kh_range=(64, 96), tgv_range=(32, 40)))
    mk = lambda rate: serving.mixed_workload(args.serving_requests, rate, seed=3, steps=args.serving_steps)
    log = lambda m: print(m, flush=True)
    batched = srv.run(mk(args.serving_rate), log=log)
    print(f"serving: batched {batched}", flush=True)
    single = srv.run(mk(args.serving_rate), max_resident=1, log=log)
    print(f"serving: one at a time {single}", flush=True)
    sweep = []
    for r in [float(x) for x in args.serving_sweep.split(",") if x]:
        res = srv.run(mk(r), log=log)
        res["rate"] = r
        sweep.append(res)
        print(f"serving: rate {r} {res}", flush=True)
    srv.close()
    out = {
        "metric": "p99 solve latency (s), serving, mixed 2D KH / 3D TGV FP64 solves",
        "value": batched["p99_s"], "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.serving_requests} requests, Poisson {args.serving_rate}/s (seed 3), "
                               f"60% KH 2D n in [64,1024], 40% TGV 3D n in [32,128], "
                               f"{args.serving_steps} TVD-RK3 CFL steps each"},
        "batched": batched, "one_at_a_time": single,
        "throughput_ratio": batched["throughput_req_s"] / single["throughput_req_s"],
        "load_sweep": sweep,
    }
    print(json.dumps(out), flush=True)


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
    if args.serving:
        serving_bench(args)
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
    # the sweeps also form the tangential velocity derivatives they need; the
    # nine fourth-order central derivatives of a cell (5 flops each) are
    # credited a third to each sweep
    grad = GRADIENT_FLOPS_PER_CELL / 3.0
    # the sweeps run z, y, x; the x sweep, the last, also applies the stage
    # update and forms the primitives of the updated cells
    flops = {
        0: parts["prim_per_cell"] * (n + 6) ** 3,
        1: face * faces_per_axis + (DIVERGENCE_FLOPS_PER_CELL_AXIS + grad + RK_FLOPS_PER_CELL
                                    + parts["prim_per_cell"]) * cells,
        2: face * faces_per_axis + (DIVERGENCE_FLOPS_PER_CELL_AXIS + grad) * cells,
        3: face * faces_per_axis + (DIVERGENCE_FLOPS_PER_CELL_AXIS + grad) * cells,
        4: 0.0,
    }[dom]
    achieved = flops / (ms[dom] * 1e-3)
    roofline = {"bound": "alu", "kernel": KERNELS[dom], "achieved": achieved / 1e12,
                "peak": MI355X_FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / MI355X_FP64_VECTOR_PEAK, "traffic": None,
                "kernel_ms": {k: round(v, 4) for k, v in zip(KERNELS, ms)},
                "flops_per_launch": flops}
    traffic = measured_traffic(n)
    if traffic and KERNELS[dom] in traffic:
        rd, wr = traffic[KERNELS[dom]]
        roofline["traffic"] = rd + wr
        roofline["traffic_GBps"] = (rd + wr) / (ms[dom] * 1e-3) / 1e9
        roofline["traffic_hbm_frac"] = (rd + wr) / (ms[dom] * 1e-3) / MI355X_HBM_PEAK
        # a stage of a run of steps: the sweeps and the primitives' halo refresh
        # (the primitive pass runs once per run, before the first step)
        stage = KERNELS[1:]
        if all(k in traffic for k in stage):
            stage_bytes = sum(sum(traffic[k]) for k in stage)
            roofline["stage_traffic_bytes"] = stage_bytes
            roofline["stage_traffic_GBps"] = stage_bytes / (sum(ms[1:]) * 1e-3) / 1e9
    # whole-step view: algorithmic flops per cell-update over the measured step time
    step_flops = 3 * (3 * face * (n + 1) / n + parts["prim_per_cell"] * ((n + 6) / n) ** 3
                      + GRADIENT_FLOPS_PER_CELL + 3 * DIVERGENCE_FLOPS_PER_CELL_AXIS + RK_FLOPS_PER_CELL)
    s.close()
    del U
    torch.cuda.empty_cache()

    roe = None
    if not args.no_roe:
        roe = roe_leg(case, W, args.roe_steps, args.reps, ms_per_step)
        print(f"bench: ROE setup {roe['value']:.1f} Mcell-updates/s, {roe['ms_per_step']:.3f} ms per step "
              f"({roe['over_hllc']:.2f} x the HLLC step)", flush=True)
        torch.cuda.empty_cache()

    wenoz = None
    if not args.no_roe:
        wenoz = scheme_leg(case, W, args.roe_steps, args.reps, ms_per_step, wl.WENOZ)
        print(f"bench: WENO5-Z {wenoz['value']:.1f} Mcell-updates/s ({wenoz['over_hllc']:.2f} x the WENO5-JS step)",
              flush=True)
        torch.cuda.empty_cache()

    implosion = None
    if not args.no_implosion:
        implosion = implosion_leg(args.nn_epochs)
        print(f"bench: implosion 128^2 -> 32^2 over {implosion['coarse_steps']} coarse steps in "
              f"{implosion['seconds']:.1f} s; mean relative L1 density error Rusanov "
              f"{implosion['mean']['rusanov_rho']:.4f}, HLLC {implosion['mean']['hllc_rho']:.4f}", flush=True)
        if "rusanov_nn" in implosion:
            r = implosion["rusanov_nn"]
            print(f"bench: Rusanov-NN trained {r['epochs']} epoch(s), {r['batches']} batches at "
                  f"{r['seconds_per_batch']:.3f} s/batch; mean relative L1 density error "
                  f"{r['mean']['nn_rho']:.4f} (classical Rusanov {r['mean']['rusanov_rho']:.4f})", flush=True)
        torch.cuda.empty_cache()

    adjoint = None
    if not args.no_adjoint:
        adjoint = differentiation(args.adj_n, args.adj_steps)
        print(f"bench: adjoint step / step = {adjoint['adjoint_over_step']:.3f} recomputing the stages, "
              f"{adjoint['adjoint_kept_stages_over_step']:.3f} with kept stages, at {args.adj_n}^3, "
              f"gradient through {args.adj_steps} steps in {adjoint['gradient_s']:.2f} s", flush=True)
        torch.cuda.empty_cache()

    serving_out = None
    if not args.no_serving:
        serving_out = serving_leg(args.serving_requests, args.serving_rate, args.serving_steps)
        print(f"bench: serving p50 {serving_out['p50_s']:.2f} s, p99 {serving_out['p99_s']:.2f} s, batched "
              f"{serving_out['batched']['throughput_req_s']:.1f} req/s = {serving_out['throughput_ratio']:.2f} x "
              f"one at a time", flush=True)
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
        "p99_solve_latency_s": serving_out["p99_s"] if serving_out else None,
        "serving": serving_out,
        "differentiation": adjoint,
        "roe_setup": roe,
        "wenoz": wenoz,
        "implosion": implosion,
        "paper_context": {"value": 1000.0 / 92.76, "unit": "Mcell-updates/s",
                          "workload": "Taylor-Green vortex 256^3, HLLC float64, JAX on one RTX A6000"},
        "health": health,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
