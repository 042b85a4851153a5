"""Write paper_2203_13760_amd/opcounts.json: algorithmic FP64 operation counts
(add + mul + div + sqrt, each one flop) of the parts of one right-hand side,
counted by the oracle's OpCount instantiation. The benchmark reads this table
to price kernels against the FP64 vector peak; it never runs the oracle for it.

Usage: python oracle/write_opcounts.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402


def case(n, flags, dims):
    ext = [n if d < dims else 1 for d in range(3)]
    return {"n": ext, "nh": 3, "lo": [0, 0, 0], "hi": [1, 1, 1], "gamma": 1.4, "mu": 0.01,
            "prandtl": 0.72, "cfl": 0.5, "bc": [0] * 6, "flags": flags}


def main():
    out = {"definition": "flops = add + mul + div + sqrt of the oracle's operations; "
                         "face = one numerical flux G = F - F^d at one face",
           "divergence_per_cell_axis": 15, "rk_stage_per_cell": 20}
    rng = np.random.default_rng(0)
    for name, flags, dims in (("3d_viscous_heat", 7, 3), ("3d_inviscid", 1, 3), ("2d_inviscid", 1, 2),
                              ("1d_inviscid", 1, 1)):
        c = case(12, flags, dims)
        shape = oracle.padded_shape(c)
        W = np.empty((5,) + tuple(shape[1:]))
        W[0] = 1.0 + 0.1 * rng.random(shape[1:])
        W[1:4] = 0.1 * rng.standard_normal((3,) + tuple(shape[1:]))
        W[4] = 1.0 + 0.1 * rng.random(shape[1:])
        U = np.empty(shape)
        g = c["gamma"]
        U[0] = W[0]
        U[1:4] = W[0] * W[1:4]
        U[4] = W[4] / (g - 1) + 0.5 * W[0] * (W[1:4] ** 2).sum(0)
        parts = oracle.opcount_parts(c, U)
        out[name] = {"prim_per_cell": parts["prim_per_cell"], "face_flux": parts["face"][0]}
    path = os.path.join(ROOT, "paper_2203_13760_amd", "opcounts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
