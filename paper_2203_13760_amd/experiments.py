"""Two experiments of the paper on libcfd: the validation of reverse-mode
gradients (§6.1, "Validation of Automatic Differentiation Gradients"),
single-phase case, on the discrete adjoint; and the implosion of §6.2 that
the Rusanov-NN flux is trained on, with the classical Rusanov flux and HLLC
on the coarse grid against the coarse-grained ground truth (the network and its
training are not part of this library).

Gradient validation:

A shock of Mach number M_S runs to the right into gas at rest
(rho = p = 1, u = 0); the state behind it follows from the Rankine-Hugoniot
relations. After n fixed-dt TVD-RK3 steps (HLLC setup, inviscid) the integral
entropy has grown by

    Delta S = sum_i (rho_i s_i - rho0_i s0_i) dx,   s = ln(p / rho^gamma) / (gamma - 1)

(specific entropy in units of c_v, up to a constant that cancels), and its
derivative with respect to M_S is obtained by reverse mode: the derivative of
Delta S with respect to the final state, pulled back through the n step
adjoints (RK3Rollout), contracted with the derivative of the initial state with
respect to M_S (torch autograd of the Rankine-Hugoniot state). The paper
compares it with second-order central differences
(Delta S(M + e) - Delta S(M - e)) / 2e, which converge to it at second order.

The paper fixes M_S = 2, dt = 1e-2, n = 5 and gamma = 1.4 but not the grid:
here x in [0, 2] with 40 cells (dx = 0.05, so the CFL number of the post-shock
state is about 0.6), the shock at x = 0.5, zero-gradient ends.
"""
from __future__ import annotations

import time

import torch

from . import workloads as wl
from .autograd import conservative_from_primitive, rollout
from .solver import Solver, interior

SHOCK_M = 2.0
SHOCK_DT = 1e-2
SHOCK_STEPS = 5
SHOCK_EPS = (1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4)


def shock_case(n=40, length=2.0, gamma=1.4):
    return wl.make_case((n, 1, 1), hi=(length, 1.0, 1.0), gamma=gamma, bc=(wl.ZERO_GRADIENT,) * 6,
                        flags=wl.INVISCID, cfl=0.5)


def post_shock(M, gamma=1.4, rho_r=1.0, p_r=1.0):
    """Rankine-Hugoniot state behind a shock of Mach number M (torch scalar)
    moving right into gas at rest (rho_r, u = 0, p_r): (rho, u, p)."""
    c_r = (gamma * p_r / rho_r) ** 0.5
    M2 = M * M
    rho = rho_r * (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
    p = p_r * (2.0 * gamma * M2 - (gamma - 1.0)) / (gamma + 1.0)
    u = M * c_r * (1.0 - rho_r / rho)
    return rho, u, p


def initial_W(case, M, x_shock=0.5):
    """Primitive initial state (5, 1, 1, n) as a differentiable function of M."""
    x = torch.as_tensor(wl.cell_centres(case, 0), dtype=torch.float64, device=M.device)
    left = (x < x_shock).to(torch.float64)
    rho_l, u_l, p_l = post_shock(M, case["gamma"])
    rho = left * rho_l + (1.0 - left) * 1.0
    u = left * u_l
    p = left * p_l + (1.0 - left) * 1.0
    zero = torch.zeros_like(x)
    return torch.stack([rho, u, zero, zero, p]).reshape(5, 1, 1, -1)


def integral_entropy(case, U):
    """sum_i rho_i s_i dx over the interior cells of a padded conservative state."""
    g = case["gamma"]
    Ui = interior(case, U)
    rho = Ui[0]
    p = (g - 1.0) * (Ui[4] - 0.5 * (Ui[1] ** 2 + Ui[2] ** 2 + Ui[3] ** 2) / rho)
    s = (torch.log(p) - g * torch.log(rho)) / (g - 1.0)
    dx = (case["hi"][0] - case["lo"][0]) / case["n"][0]
    return (rho * s).sum() * dx


def delta_entropy(solver: Solver, M, dt=SHOCK_DT, n_steps=SHOCK_STEPS):
    """Delta S after n_steps from the shock of Mach number M (differentiable in M)."""
    case = solver.case
    U0 = conservative_from_primitive(solver, initial_W(case, M))
    Un = rollout(U0, solver, dt, n_steps, ckpt_every=n_steps)
    return integral_entropy(case, Un) - integral_entropy(case, U0)


def shock_entropy_gradient(M0=SHOCK_M, eps=SHOCK_EPS, n=40):
    """g_AD = d(Delta S)/dM_S by the discrete adjoint, and the central
    differences g_FD(e) for each e in eps, on one GPU."""
    case = shock_case(n)
    s = Solver(case)
    try:
        M = torch.tensor(M0, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dS = delta_entropy(s, M)
        dS.backward()
        torch.cuda.synchronize()
        t_ad = time.perf_counter() - t0
        g_ad = float(M.grad.item())
        fd = []
        with torch.no_grad():
            for e in eps:
                up = delta_entropy(s, torch.tensor(M0 + e, dtype=torch.float64, device="cuda"))
                dn = delta_entropy(s, torch.tensor(M0 - e, dtype=torch.float64, device="cuda"))
                fd.append(float((up - dn).item()) / (2.0 * e))
        return {"M_S": M0, "dt": SHOCK_DT, "steps": SHOCK_STEPS, "cells": n, "delta_S": float(dS.item()),
                "g_ad": g_ad, "eps": list(eps), "g_fd": fd, "fd_error": [abs(x - g_ad) for x in fd],
                "ad_seconds": t_ad}
    finally:
        s.close()


# ---------------------------------------------------------------- §6.2 implosion
def coarse_grain(U_fine, case_fine, n_cg):
    """Block averages of the fine interior conservative state onto n_cg x n_cg
    cells (reading: the paper's coarse-graining of the 128^2 trajectory onto
    32^2 points, done finite-volume consistently on the conserved variables)."""
    Ui = interior(case_fine, U_fine)  # (5, 1, n, n)
    n = case_fine["n"][0]
    r = n // n_cg
    return Ui.reshape(5, 1, n_cg, r, n_cg, r).mean(dim=(3, 5))


def _set_interior(solver, U, Ui):
    interior(solver.case, U).copy_(Ui)
    solver.fill_halo(U)


def _rho_p(Ui, gamma):
    rho = Ui[0]
    p = (gamma - 1.0) * (Ui[4] - 0.5 * (Ui[1] ** 2 + Ui[2] ** 2 + Ui[3] ** 2) / rho)
    return rho, p


def implosion_trajectories(n_fine=128, n_cg=32, dt=2.5e-4, dt_cg=1e-3, n_cg_steps=2500, every=100):
    """The implosion of §6.2: the ground truth on n_fine^2 (WENO3-JS, TVD-RK2,
    HLLC, fixed dt), coarse-grained onto n_cg^2 every dt_cg, and the coarse
    solvers with the Rusanov flux and with HLLC (WENO3-JS, TVD-RK2, dt_cg) run
    from the coarse-grained initial state. Returns the relative L1 errors of
    density and pressure against the coarse-grained truth every `every` coarse
    steps (the quantity of the paper's error figure), on one GPU."""
    case_f, W = wl.implosion(n_fine)
    fine = Solver(case_f)
    coarse = {}
    try:
        Uf = fine.init(W)
        r = int(round(dt_cg / dt))
        cg0 = coarse_grain(Uf, case_f, n_cg)
        states = {}
        for name, flux in (("rusanov", wl.RUSANOV), ("hllc", 0)):
            case_c, Wc = wl.implosion(n_cg, flags=wl.INVISCID | wl.WENO3 | wl.RK2 | flux)
            s = Solver(case_c)
            coarse[name] = s
            Uc = s.init(Wc)
            _set_interior(s, Uc, cg0)
            states[name] = Uc
        g = case_f["gamma"]
        out = {"step": [], "t": [], "rusanov_rho": [], "rusanov_p": [], "hllc_rho": [], "hllc_p": []}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, n_cg_steps + 1):
            fine.advance_fixed(Uf, r, dt)
            for name, s in coarse.items():
                s.advance_fixed(states[name], 1, dt_cg)
            if k % every == 0 or k == n_cg_steps:
                rho_t, p_t = _rho_p(coarse_grain(Uf, case_f, n_cg), g)
                out["step"].append(k)
                out["t"].append(k * dt_cg)
                for name, s in coarse.items():
                    rho, p = _rho_p(interior(s.case, states[name]), g)
                    out[f"{name}_rho"].append(float((rho - rho_t).abs().sum() / rho_t.abs().sum()))
                    out[f"{name}_p"].append(float((p - p_t).abs().sum() / p_t.abs().sum()))
        torch.cuda.synchronize()
        out["seconds"] = time.perf_counter() - t0
        out["health"] = {"fine": fine.check(), **{n: s.check() for n, s in coarse.items()}}
        return out
    finally:
        fine.close()
        for s in coarse.values():
            s.close()
