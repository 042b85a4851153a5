"""Parity at the full sizes of the benchmark configurations, against the live
oracle (its long runs start in background threads at collection; see
oracle_jobs.py) or against a stored oracle result:

  - the Taylor-Green vortex at 64^3 through 100 CFL steps, whole field;
  - the 256^3 headline field after one step, on 8 full z-planes;
  - the gradient of the differentiation workload at 16^3 through 200 steps
    with checkpoints every 20, against the oracle's reverse mode (stored by
    tests/golden/make_tgv16_gradient.py);
  - a serving mix whose x-sweep phase takes the batch kernel's dynamic work
    distribution (per-XCD counters, stealing, counter reset), 3 steps.

Error measure as in test_gpu_parity.py: normwise per variable, 1e-12 after
one step, 1e-10 after 100 steps or through a rollout gradient.
"""
import math
import os

import numpy as np
import pytest

import oracle
import oracle_jobs
from paper_2203_13760_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def normwise(a, b):
    err = 0.0
    for v in range(a.shape[0]):
        den = float(np.max(np.abs(b[v])))
        num = float(np.max(np.abs(a[v] - b[v])))
        if num:
            err = max(err, num / den if den > 0 else math.inf)
    return err


@pytest.fixture(scope="module")
def Solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_13760_amd.solver import Solver as S
    return S


@pytest.mark.oracle_job("tgv64_100")
def test_tgv64_hundred_cfl_steps_match_oracle(Solver):
    case, W = wl.taylor_green(64)
    print("full-size parity: TGV 64^3, 100 CFL steps, whole field", flush=True)
    s = Solver(case)
    U = s.init(W)
    t = s.advance(U, 100)
    Ug = U.cpu().numpy()
    tg = float(t.item())
    assert s.check() == 0
    s.close()
    ref = oracle_jobs.result("tgv64_100")
    assert ref["steps"] == 100
    assert abs(tg - ref["t"]) <= 1e-12 * ref["t"]
    e = normwise(oracle.interior(case, Ug), oracle.interior(case, ref["U"]))
    assert e <= 1e-10, e


@pytest.mark.oracle_job("hit256_planes")
def test_hit256_step_on_eight_full_planes(Solver):
    case, W = wl.isotropic_turbulence(256, seed=2203)
    print("full-size parity: HIT 256^3, one step, 8 full z-planes", flush=True)
    ref = oracle_jobs.result("hit256_planes")
    s = Solver(case)
    U = s.init(W)
    dtg = s.compute_dt(U)
    assert abs(float(dtg.item()) - ref["dt"]) <= 1e-14 * ref["dt"]
    s.step(U, ref["dt"])
    k0, nk = oracle_jobs.HIT_PLANES
    h = case["nh"]
    got = U[:, h + k0:h + k0 + nk, h:h + 256, h:h + 256].cpu().numpy()
    assert s.check() == 0
    s.close()
    e = normwise(got, ref["planes"])
    assert e <= 1e-12, e


def test_rollout_gradient_16_cubed_200_steps_matches_oracle(Solver):
    from paper_2203_13760_amd.autograd import rollout, state_init
    from paper_2203_13760_amd.experiments import kinetic_energy
    gold = np.load(os.path.join(GOLDEN, "tgv16_gradient_200.npz"))
    case, W = wl.taylor_green_noisy(int(gold["n"]), sigma=float(gold["sigma"]), seed=int(gold["seed"]))
    dt = float(gold["dt"])
    assert dt == oracle.cfl_dt(case, oracle.state_init(case, W))
    print("rollout gradient vs oracle reverse mode: 16^3, 200 steps, checkpoints every 20", flush=True)
    s = Solver(case)
    Wt = torch.from_numpy(W).cuda().requires_grad_(True)
    L = kinetic_energy(s, rollout(state_init(s, Wt), s, dt, int(gold["steps"]), 20))
    L.backward()
    g = Wt.grad[1:4].cpu().numpy()
    s.close()
    assert abs(float(L.item()) - float(gold["loss"])) <= 1e-12 * abs(float(gold["loss"]))
    e = normwise(g, gold["grad"])
    assert e <= 1e-10, e


@pytest.mark.oracle_job("serving_large")
def test_serving_mix_on_the_dynamic_path_matches_oracle(Solver):
    from paper_2203_13760_amd import cfd
    from paper_2203_13760_amd.solver import padded_shape
    grids = oracle_jobs.serving_large_mix()
    steps = oracle_jobs.SERVING_STEPS
    print(f"serving parity: TGV 128^3 + 2 x KH 1024^2, {steps} steps, dynamic work distribution", flush=True)

    def run(sel):
        b = cfd.cfd_batch_create(8, 3 << 30)
        slots = [cfd.cfd_batch_add(b, grids[k][0], torch.from_numpy(np.ascontiguousarray(grids[k][1])).cuda())
                 for k in sel]
        assert None not in slots
        for _ in range(steps):
            cfd.cfd_batch_step(b)
        out = []
        for k, sl in zip(sel, slots):
            cfd.cfd_batch_finish(b, sl)
            U = torch.empty(padded_shape(grids[k][0]), dtype=torch.float64, device="cuda")
            cfd.cfd_batch_copy_state(b, sl, U)
            out.append(U.cpu().numpy())
        torch.cuda.synchronize()
        cfd.cfd_batch_destroy(b)
        return out

    # the x-sweep phase of the mix holds more blocks than the dynamic threshold
    # (8 per workgroup of the 2048-workgroup persistent launch); each grid
    # alone stays below it and takes the fixed stride
    def x_blocks(case):
        n = case["n"]
        slots = (n[0] + 4) * n[1] * n[2]
        return ((slots + 59) // 60 + 3) // 4

    assert sum(x_blocks(c) for c, _ in grids) >= 8 * 2048
    assert all(x_blocks(c) < 8 * 2048 for c, _ in grids)
    mix = run([0, 1, 2])
    alone = [run([k])[0] for k in range(3)]
    for k in range(3):
        assert np.array_equal(mix[k], alone[k]), k
    ref = oracle_jobs.result("serving_large")
    for k, (case, _) in enumerate(grids):
        e = normwise(oracle.interior(case, mix[k]), oracle.interior(case, ref[k]))
        assert e <= 1e-10, (k, e)
