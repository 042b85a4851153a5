"""Two experiments of the paper on libcfd: the validation of reverse-mode
gradients (§7.3, "Validation of Automatic Differentiation Gradients"),
single-phase case, on the discrete adjoint; and the implosion of §7.4 that
the Rusanov-NN flux is trained on, with the classical Rusanov flux and HLLC
on the coarse grid against the coarse-grained ground truth, and the supervised
training of the Rusanov-NN dissipation through the discrete adjoint.

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
from .autograd import rollout, state_init
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


def kinetic_energy(solver: Solver, U):
    """Total kinetic energy sum 1/2 |rho u|^2 / rho dV over interior cells: the
    loss of the differentiation workload (a Taylor-Green vortex's final
    kinetic energy as a function of its initial velocities)."""
    Ui = interior(solver.case, U)
    dV = 1.0
    for d in range(3):
        dV *= (solver.case["hi"][d] - solver.case["lo"][d]) / solver.case["n"][d]
    return (0.5 * (Ui[1] ** 2 + Ui[2] ** 2 + Ui[3] ** 2) / Ui[0]).sum() * dV


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
    U0 = state_init(solver, initial_W(case, M))
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


# ---------------------------------------------------------------- §7.4 implosion
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
    """The implosion of §7.4: the ground truth on n_fine^2 (WENO3-JS, TVD-RK2,
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


# ---------------------------------------------------------------------------
# Rusanov-NN training (§7.4)

NN_FLAGS = wl.INVISCID | wl.WENO3 | wl.RK2 | wl.RUSANOV_NN


def cg_trajectory(n_fine=128, n_cg=32, dt=2.5e-4, dt_cg=1e-3, n_cg_steps=1000):
    """The coarse-grained ground truth of §7.4: the n_fine^2 implosion (WENO3-JS,
    TVD-RK2, HLLC, fixed dt) block-averaged onto n_cg^2 every dt_cg. Returns a
    device tensor (n_cg_steps + 1, 5, 1, n_cg, n_cg) of interior conservative
    states, snapshot 0 the initial state."""
    case_f, W = wl.implosion(n_fine)
    fine = Solver(case_f)
    try:
        Uf = fine.init(W)
        r = int(round(dt_cg / dt))
        out = torch.empty((n_cg_steps + 1, 5, 1, n_cg, n_cg), dtype=torch.float64, device=Uf.device)
        out[0] = coarse_grain(Uf, case_f, n_cg)
        for k in range(1, n_cg_steps + 1):
            fine.advance_fixed(Uf, r, dt)
            out[k] = coarse_grain(Uf, case_f, n_cg)
        if fine.check() != 0:
            raise RuntimeError("ground-truth run left the admissible states")
        return out
    finally:
        fine.close()


def primitives_2d(Ui, gamma):
    """(rho, u, v, p) of interior conservative states (5, ...): the primitive
    state vector W of the §7.4 loss (the flow is two-dimensional)."""
    rho = Ui[0]
    u = Ui[1] / rho
    v = Ui[2] / rho
    p = (gamma - 1.0) * (Ui[4] - 0.5 * (Ui[1] * u + Ui[2] * v + Ui[3] * Ui[3] / rho))
    return torch.stack((rho, u, v, p))


def _interior_slices(case):
    """Slices of the interior cells over the last three (z, y, x) dimensions."""
    nh = int(case.get("nh", 3))
    return tuple(slice(nh, nh + int(case["n"][d])) if int(case["n"][d]) > 1 else slice(0, 1) for d in (2, 1, 0))


def primitive_mse_grad(Ui, Wt, gamma, scale):
    """Gradient with respect to interior conservative states Ui (5, ...) of
    scale * mean((W(Ui) - Wt)^2), W = (rho, u, v, p) as in primitives_2d and Wt
    the target primitives (4, ...), written out by the chain rule (elementwise,
    so it can be captured in a graph without reductions)."""
    rho = Ui[0]
    ir = 1.0 / rho
    u, v, w = Ui[1] * ir, Ui[2] * ir, Ui[3] * ir
    gm1 = gamma - 1.0
    p = gm1 * (Ui[4] - 0.5 * (Ui[1] * u + Ui[2] * v + Ui[3] * w))
    c = 2.0 * scale / (4.0 * rho.numel())
    rr, ru, rv, rp = c * (rho - Wt[0]), c * (u - Wt[1]), c * (v - Wt[2]), c * (p - Wt[3])
    return torch.stack((rr - (ru * u + rv * v) * ir + rp * (0.5 * gm1) * (u * u + v * v + w * w),
                        ru * ir - rp * (gm1 * u),
                        rv * ir - rp * (gm1 * v),
                        -rp * (gm1 * w),
                        rp * gm1))


class RusanovNNTrainer:
    """Supervised training of the Rusanov-NN dissipation on a coarse-grained
    trajectory (§7.4): from snapshot s the coarse solver (WENO3-JS, TVD-RK2,
    Rusanov-NN, fixed dt_cg) is unrolled for n_unroll steps; the loss is the
    mean over the unrolled steps of the mean squared error between predicted
    and coarse-grained primitive states (rho, u, v, p); its gradient with
    respect to the network weights comes from the step adjoints of the library
    (the state adjoint pulled back step by step, the weight gradient
    accumulated by the library), and Adam updates the weights in place on the
    device, where every later launch reads them."""

    def __init__(self, traj, theta0, dt_cg=1e-3, n_unroll=15, lr=5e-4, betas=(0.9, 0.999), eps=1e-8, graph=False):
        n_cg = traj.shape[-1]
        self.case, _ = wl.implosion(n_cg, flags=NN_FLAGS)
        self.gamma = float(self.case["gamma"])
        self.solver = Solver(self.case)
        self.traj = traj
        self.dt = float(dt_cg)
        self.n_unroll = int(n_unroll)
        self.theta = torch.as_tensor(theta0, dtype=torch.float64).to(traj.device).contiguous()
        self.theta_bar = torch.zeros_like(self.theta)
        self.solver.set_nn_weights(self.theta, self.theta_bar)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.t = 0
        shape = tuple(self.solver.shape)
        self.S = torch.zeros((self.n_unroll + 1,) + shape, dtype=torch.float64, device=traj.device)  # states
        self.T = torch.zeros((self.n_unroll, 4) + tuple(traj.shape[2:]), dtype=torch.float64, device=traj.device)
        self.ubar = [self.solver.empty_state() for _ in range(2)]
        self.graph = None
        if graph:
            self._capture()

    def close(self):
        self.graph = None
        self.solver.close()

    def _body(self):
        """The window on the static buffers: n_unroll fixed steps from S[0],
        then the reverse, each step adjoint seeded with the loss gradient of its
        output against the targets T; the library adds the weight gradient
        (loss scale 1) to theta_bar. A fixed launch sequence with no host
        synchronisation and no allocation (capturable)."""
        sv, case = self.solver, self.case
        for k in range(1, self.n_unroll + 1):
            self.S[k].copy_(self.S[k - 1])
            sv.step(self.S[k], self.dt)
        ub, ub_prev = self.ubar
        ub.zero_()
        for k in range(self.n_unroll, 0, -1):
            g = primitive_mse_grad(interior(case, self.S[k]), self.T[k - 1], self.gamma, 1.0 / self.n_unroll)
            interior(case, ub).add_(g)
            sv.step_adjoint(self.S[k - 1], self.dt, ub, ub_prev)
            ub, ub_prev = ub_prev, ub

    def _load(self, s0):
        """The window from snapshot s0 into the static buffers: S[0] (with its
        halo) and the target primitives T."""
        case = self.case
        U = self.S[0]
        interior(case, U).copy_(self.traj[s0])
        self.solver.fill_halo(U)
        Tc = self.traj[s0 + 1:s0 + 1 + self.n_unroll]          # (n_unroll, 5, 1, n, n)
        self.T.copy_(primitives_2d(Tc.transpose(0, 1), self.gamma).transpose(0, 1))

    def _capture(self):
        """Record _body as one HIP graph (torch's graph capture over the
        library's launches on the current stream). One eager run on the first
        window first allocates the library's adjoint scratch and warms the
        allocator; the weight gradient it adds is cleared, and so is the
        solver's health word."""
        self._load(0)
        self._body()
        torch.cuda.synchronize()
        self.theta_bar.zero_()
        self.solver.check()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._body()
        torch.cuda.synchronize()
        self.theta_bar.zero_()
        self.graph = g

    def _window(self, s0):
        """Loss of the window from snapshot s0 (a device scalar); adds its
        weight gradient to theta_bar."""
        case = self.case
        self._load(s0)
        if self.graph is not None:
            self.graph.replay()
        else:
            self._body()
        Si = self.S[1:][(Ellipsis,) + _interior_slices(case)]  # (n_unroll, 5, 1, n, n)
        Wp = primitives_2d(Si.transpose(0, 1), self.gamma)
        return torch.mean((Wp - self.T.transpose(0, 1)) ** 2)

    def train_batch(self, starts):
        """One Adam step on the mean loss of the windows from `starts`; returns
        that loss."""
        self.theta_bar.zero_()
        loss = sum(self._window(int(s0)) for s0 in starts) / len(starts)
        self.theta_bar.mul_(1.0 / len(starts))
        g = self.theta_bar
        b1, b2 = self.betas
        self.t += 1
        self.m.mul_(b1).add_(g, alpha=1.0 - b1)
        self.v.mul_(b2).addcmul_(g, g, value=1.0 - b2)
        mh = self.m / (1.0 - b1 ** self.t)
        vh = self.v / (1.0 - b2 ** self.t)
        self.theta.sub_(self.lr * mh / (vh.sqrt() + self.eps))
        return float(loss)

    def rollout_errors(self, traj_eval, every=100):
        """Relative L1 errors of density and pressure of the coarse Rusanov-NN
        solver run from snapshot 0 over the whole of traj_eval (the quantity of
        the paper's error figure)."""
        sv, case = self.solver, self.case
        U = sv.empty_state()
        interior(case, U).copy_(traj_eval[0])
        sv.fill_halo(U)
        out = {"step": [], "rho": [], "p": []}
        n = traj_eval.shape[0] - 1
        for k in range(1, n + 1):
            sv.advance_fixed(U, 1, self.dt)
            if k % every == 0 or k == n:
                rho, p = _rho_p(interior(case, U), self.gamma)
                rho_t, p_t = _rho_p(traj_eval[k], self.gamma)
                out["step"].append(k)
                out["rho"].append(float((rho - rho_t).abs().sum() / rho_t.abs().sum()))
                out["p"].append(float((p - p_t).abs().sum() / p_t.abs().sum()))
        out["health"] = sv.check()
        return out


def train_rusanov_nn(epochs=1, n_train=1000, n_unroll=15, batch=20, lr=5e-4, seed=0, n_eval=2500, every=100,
                     theta0=None, log=print, graph=True):
    """The §7.4 training on one GPU: ground truth (128^2 -> 32^2, n_eval coarse
    steps), training windows from the first n_train coarse steps, unroll
    n_unroll, batches of `batch` windows, Adam with learning rate lr, `epochs`
    passes (the paper: 200), then the trained coarse solver and the classical
    Rusanov flux evaluated over the whole trajectory. With graph set, each
    window replays one captured HIP graph. Returns the loss per epoch, the
    errors and the timings."""
    t0 = time.perf_counter()
    traj = cg_trajectory(n_cg_steps=max(n_eval, n_train))
    torch.cuda.synchronize()
    t_truth = time.perf_counter() - t0
    th0 = wl.nn_weights(seed=seed, alpha0=1.2, scale=0.1) if theta0 is None else theta0
    tr = RusanovNNTrainer(traj, th0, n_unroll=n_unroll, lr=lr, graph=graph)
    g = torch.Generator().manual_seed(seed)
    starts = torch.arange(0, n_train - n_unroll + 1)
    out = {"epochs": epochs, "n_train": n_train, "n_unroll": n_unroll, "batch": batch, "lr": lr, "graph": graph,
           "truth_seconds": t_truth, "epoch_loss": [], "batches": 0}
    try:
        out["before"] = tr.rollout_errors(traj[: n_eval + 1], every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for ep in range(epochs):
            perm = starts[torch.randperm(len(starts), generator=g)]
            tot, nb = 0.0, 0
            for b in range(0, len(perm), batch):
                tot += tr.train_batch(perm[b:b + batch].tolist())
                nb += 1
            out["epoch_loss"].append(tot / nb)
            out["batches"] += nb
            if log:
                log(f"epoch {ep + 1}/{epochs}: loss {tot / nb:.6e}")
        torch.cuda.synchronize()
        out["train_seconds"] = time.perf_counter() - t1
        out["seconds_per_batch"] = out["train_seconds"] / max(out["batches"], 1)
        out["after"] = tr.rollout_errors(traj[: n_eval + 1], every)
        out["theta"] = tr.theta.cpu().numpy().tolist()
    finally:
        tr.close()
    # the classical Rusanov flux from the same coarse-grained initial state
    case_r, _ = wl.implosion(traj.shape[-1], flags=wl.INVISCID | wl.WENO3 | wl.RK2 | wl.RUSANOV)
    sr = Solver(case_r)
    try:
        U = sr.empty_state()
        interior(case_r, U).copy_(traj[0])
        sr.fill_halo(U)
        rus = {"step": [], "rho": [], "p": []}
        gmm = float(case_r["gamma"])
        for k in range(1, n_eval + 1):
            sr.advance_fixed(U, 1, 1e-3)
            if k % every == 0 or k == n_eval:
                rho, p = _rho_p(interior(case_r, U), gmm)
                rho_t, p_t = _rho_p(traj[k], gmm)
                rus["step"].append(k)
                rus["rho"].append(float((rho - rho_t).abs().sum() / rho_t.abs().sum()))
                rus["p"].append(float((p - p_t).abs().sum() / p_t.abs().sum()))
        out["rusanov"] = rus
    finally:
        sr.close()
    return out


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="Rusanov-NN training on the implosion of §7.4")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--n-eval", type=int, default=2500)
    ap.add_argument("--n-train", type=int, default=1000)
    ap.add_argument("--no-graph", action="store_true", help="run each training window eagerly")
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    res = train_rusanov_nn(epochs=a.epochs, n_train=a.n_train, n_eval=a.n_eval, lr=a.lr,
                           log=lambda m: print(m, flush=True), graph=not a.no_graph)
    summary = {k: v for k, v in res.items() if k != "theta"}
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)
