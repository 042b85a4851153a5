"""Write tests/golden/tgv16_gradient_200.npz: the oracle's reverse-mode
gradient of the final kinetic energy with respect to the initial velocities,
for the differentiation workload at 16^3 (Taylor-Green vortex with Gaussian
noise sigma = 1e-3, seed 4; fixed dt = the CFL step of the noisy initial
state; 200 TVD-RK3 steps). Calls only the oracle (taped reverse mode, one step
at a time); about ten minutes on one core.

    python tests/golden/make_tgv16_gradient.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_13760_amd import workloads as wl  # noqa: E402

N, STEPS, SEED, SIGMA = 16, 200, 4, 1e-3


def main():
    case, W = wl.taylor_green_noisy(N, sigma=SIGMA, seed=SEED)
    dt = oracle.cfl_dt(case, oracle.state_init(case, W))
    t0 = time.perf_counter()
    loss, grad = oracle.grad_kinetic_energy(case, W, STEPS, dt)
    sec = time.perf_counter() - t0
    out = os.path.join(HERE, "tgv16_gradient_200.npz")
    np.savez(out, loss=np.float64(loss), grad=grad, dt=np.float64(dt), n=N, steps=STEPS, seed=SEED,
             sigma=SIGMA)
    print(f"wrote {out}: loss {loss!r}, |grad| {np.linalg.norm(grad):.6e}, dt {dt!r}, {sec:.0f} s")


if __name__ == "__main__":
    main()
