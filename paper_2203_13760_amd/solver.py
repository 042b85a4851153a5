"""Solver: a thin owner of one libcfd handle plus torch-allocated states.

Device memory and streams come from PyTorch; all arithmetic runs in libcfd.
"""
from __future__ import annotations

import numpy as np
import torch

from . import cfd


def padded_shape(case):
    nh = int(case.get("nh", 3))
    ext = [int(n) + 2 * nh if int(n) > 1 else 1 for n in case["n"]]
    return (5, ext[2], ext[1], ext[0])


def interior(case, U):
    """View of the interior cells of a padded state (5, Z, Y, X)."""
    nh = int(case.get("nh", 3))
    sl = []
    for d in (2, 1, 0):
        n = int(case["n"][d])
        sl.append(slice(nh, nh + n) if n > 1 else slice(0, 1))
    return U[(slice(None),) + tuple(sl)]


class Solver:
    def __init__(self, case, device="cuda"):
        self.case = dict(case)
        self.device = torch.device(device)
        self.shape = padded_shape(case)
        self.h = cfd.cfd_create(case)
        assert cfd.cfd_state_numel(self.h) == int(np.prod(self.shape))
        self._scalar = torch.zeros(2, dtype=torch.float64, device=self.device)

    def close(self):
        if self.h:
            cfd.cfd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_state(self):
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def init(self, W):
        """Padded conservative state from interior primitives W (5, nz, ny, nx)."""
        W = torch.as_tensor(np.ascontiguousarray(W), dtype=torch.float64).to(self.device).contiguous()
        U = self.empty_state()
        cfd.cfd_state_init(self.h, W, U)
        return U

    def state_init(self, W, U):
        """cfd_state_init of device primitives W (5, nz, ny, nx) into U."""
        cfd.cfd_state_init(self.h, W, U)
        return U

    def state_init_adjoint(self, W, Ubar, Wbar):
        """Wbar += (dU/dW)^T Ubar for U = state_init(W) (cfd_state_init_adjoint)."""
        cfd.cfd_state_init_adjoint(self.h, W, Ubar, Wbar)
        return Wbar

    def fill_halo(self, U):
        cfd.cfd_fill_halo(self.h, U)
        return U

    def rhs(self, U, R=None):
        R = self.empty_state() if R is None else R
        cfd.cfd_rhs(self.h, U, R)
        return R

    def compute_dt(self, U):
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        cfd.cfd_compute_dt(self.h, U, out)
        return out

    def step(self, U, dt=0.0):
        """One TVD-RK3 step in place; returns the device scalar holding dt."""
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        cfd.cfd_rk3_step(self.h, U, float(dt), out)
        return out

    def advance(self, U, n_steps, t_end=0.0, t=None):
        """n_steps CFL steps in place (stopping at t_end > 0); t is a device scalar."""
        if t is None:
            t = torch.zeros(1, dtype=torch.float64, device=self.device)
        cfd.cfd_advance(self.h, U, int(n_steps), float(t_end), t)
        return t

    def advance_fixed(self, U, n_steps, dt):
        cfd.cfd_advance_fixed(self.h, U, int(n_steps), float(dt))
        return U

    def rhs_adjoint(self, U, Rbar, Ubar=None):
        Ubar = self.empty_state() if Ubar is None else Ubar
        cfd.cfd_rhs_adjoint(self.h, U, Rbar, Ubar)
        return Ubar

    def step_adjoint(self, Un, dt, Ubar_np1, Ubar_n=None):
        Ubar_n = self.empty_state() if Ubar_n is None else Ubar_n
        cfd.cfd_rk3_step_adjoint(self.h, Un, float(dt), Ubar_np1, Ubar_n)
        return Ubar_n

    def step_stages(self, U, dt, U1, U2):
        """One fixed-dt step in place, keeping its stage states in U1 and U2."""
        cfd.cfd_rk3_step_stages(self.h, U, float(dt), U1, U2)
        return U

    def step_adjoint_stages(self, Un, U1, U2, dt, Ubar_np1, Ubar_n=None):
        Ubar_n = self.empty_state() if Ubar_n is None else Ubar_n
        cfd.cfd_rk3_step_adjoint_stages(self.h, Un, U1, U2, float(dt), Ubar_np1, Ubar_n)
        return Ubar_n

    def empty_stage_prims(self):
        """Buffer for the primitives of a step's three stage inputs (cfd_rk3_step_prims)."""
        return torch.empty((3, 6) + self.shape[1:], dtype=torch.float64, device=self.device)

    def step_prims(self, U, dt, P):
        """One fixed-dt step in place, keeping the primitives of its stage inputs in P."""
        cfd.cfd_rk3_step_prims(self.h, U, float(dt), P)
        return U

    def step_adjoint_prims(self, P, dt, Ubar_np1, Ubar_n=None):
        Ubar_n = self.empty_state() if Ubar_n is None else Ubar_n
        cfd.cfd_rk3_step_adjoint_prims(self.h, P, float(dt), Ubar_np1, Ubar_n)
        return Ubar_n

    def set_nn_weights(self, theta, theta_bar=None):
        """Rusanov-NN weights (a device float64 tensor of cfd.CFD_NN_PARAMS values,
        read at every launch, so it may be updated in place) and an optional
        accumulator that every later adjoint call adds the weight gradient to.
        The solver keeps references to both."""
        for t in (theta, theta_bar):
            if t is not None:
                assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == cfd.CFD_NN_PARAMS
        cfd.cfd_set_nn_weights(self.h, theta, theta_bar)
        self._nn = (theta, theta_bar)

    def check(self):
        return cfd.cfd_check(self.h)
