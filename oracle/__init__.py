"""ctypes front end of the serial FP64 reference solver ("oracle").

TEST INFRASTRUCTURE ONLY: imported by the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``. The product package never imports it.

A case is described by a plain mapping with the keys ``n`` (3 interior extents,
1 = inactive axis), ``nh`` (halo width), ``lo``/``hi`` (box), ``gamma``, ``mu``,
``prandtl``, ``cfl``, ``bc`` (6 boundary codes, 0 periodic, 1 zero gradient,
2 reflecting wall, order x-, x+, y-, y+, z-, z+) and ``flags`` (1 inviscid,
2 viscous, 4 heat, 8 WENO5-Z, 16 Roe flux splitting, 32 WENO3-JS, 64 Rusanov,
128 TVD-RK2, 256 Rusanov-NN with the weights given to ``set_nn``).
States are float64 numpy arrays of shape (5, Z, Y, X) with halos (x fastest).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleCfg(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("nh", C.c_int32),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("gamma", C.c_double),
        ("mu", C.c_double),
        ("prandtl", C.c_double),
        ("cfl", C.c_double),
        ("bc", C.c_int32 * 6),
        ("flags", C.c_uint32),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: F401  (build on first use)
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    d = C.c_double
    dp = P(d)
    cfgp = P(OracleCfg)
    lib.oracle_state_numel.argtypes = [cfgp]
    lib.oracle_state_numel.restype = C.c_long
    lib.oracle_state_init.argtypes = [cfgp, dp, dp]
    lib.oracle_fill_halo.argtypes = [cfgp, dp]
    lib.oracle_rhs.argtypes = [cfgp, dp, dp]
    lib.oracle_dt.argtypes = [cfgp, dp, d, d]
    lib.oracle_dt.restype = d
    lib.oracle_rk3_step.argtypes = [cfgp, dp, d, dp]
    lib.oracle_advance.argtypes = [cfgp, dp, C.c_int, d, d, dp]
    lib.oracle_weno5.argtypes = [d, d, d, d, d]
    lib.oracle_weno5.restype = d
    lib.oracle_weno5z.argtypes = [d, d, d, d, d]
    lib.oracle_weno5z.restype = d
    lib.oracle_hllc.argtypes = [d, dp, dp, C.c_int, dp]
    lib.oracle_hllc.restype = None
    lib.oracle_einfeldt.argtypes = [d, dp, dp, C.c_int, dp]
    lib.oracle_einfeldt.restype = None
    lib.oracle_roe_eigen.argtypes = [d, dp, dp, C.c_int, dp, dp, dp]
    lib.oracle_roe_eigen.restype = None
    lib.oracle_roe_flux.argtypes = [d, dp, C.c_int, dp]
    lib.oracle_roe_flux.restype = None
    lib.oracle_euler_flux.argtypes = [d, dp, C.c_int, dp]
    lib.oracle_euler_flux.restype = None
    lib.oracle_weno3.argtypes = [d, d, d]
    lib.oracle_weno3.restype = d
    lib.oracle_rusanov.argtypes = [d, dp, dp, C.c_int, dp]
    lib.oracle_rusanov.restype = None
    lib.oracle_opcount.argtypes = [cfgp, dp, dp]
    lib.oracle_opcount_parts.argtypes = [cfgp, dp, dp]
    lib.oracle_vjp_rhs.argtypes = [cfgp, dp, dp, dp]
    lib.oracle_status.argtypes = [C.c_int]
    lib.oracle_status.restype = C.c_int
    lib.oracle_vjp_state_init.argtypes = [cfgp, dp, dp, dp]
    lib.oracle_vjp_rk3_step.argtypes = [cfgp, dp, d, dp, dp]
    lib.oracle_grad_ke.argtypes = [cfgp, dp, C.c_int, d, dp, dp]
    lib.oracle_vjp_rhs_theta.argtypes = [cfgp, dp, dp, dp, dp]
    lib.oracle_vjp_step_theta.argtypes = [cfgp, dp, d, dp, dp, dp]
    lib.oracle_set_nn.argtypes = [dp]
    lib.oracle_nn_alpha.argtypes = [dp]
    lib.oracle_nn_alpha.restype = d
    lib.oracle_rusanov_nn.argtypes = [d, dp, dp, C.c_int, dp]
    _lib = lib
    return lib


def make_cfg(case) -> OracleCfg:
    c = OracleCfg()
    for i in range(3):
        c.n[i] = int(case["n"][i])
        c.lo[i] = float(case["lo"][i])
        c.hi[i] = float(case["hi"][i])
    c.nh = int(case.get("nh", 3))
    c.gamma = float(case["gamma"])
    c.mu = float(case.get("mu", 0.0))
    c.prandtl = float(case.get("prandtl", 0.72))
    c.cfl = float(case.get("cfl", 0.5))
    for i in range(6):
        c.bc[i] = int(case["bc"][i])
    c.flags = int(case["flags"])
    return c


def padded_shape(case):
    nh = int(case.get("nh", 3))
    ext = []
    for d in range(3):
        n = int(case["n"][d])
        ext.append(n + 2 * nh if n > 1 else n)
    return (5, ext[2], ext[1], ext[0])


def interior(case, U):
    """View of the interior cells of a padded state (5, nz, ny, nx)."""
    nh = int(case.get("nh", 3))
    sl = []
    for d in (2, 1, 0):
        n = int(case["n"][d])
        sl.append(slice(nh, nh + n) if n > 1 else slice(0, 1))
    return U[(slice(None),) + tuple(sl)]


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ok(rc):
    if rc != 0:
        raise ValueError("oracle rejected the configuration")


def state_init(case, W):
    """Padded conservative state from interior primitive point values W (5, nz, ny, nx)."""
    lib = _load()
    cfg = make_cfg(case)
    W = np.ascontiguousarray(W, dtype=np.float64)
    U = np.zeros(padded_shape(case))
    _ok(lib.oracle_state_init(C.byref(cfg), _ptr(W), _ptr(U)))
    return U


def fill_halo(case, U):
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64).copy()
    _ok(lib.oracle_fill_halo(C.byref(cfg), _ptr(U)))
    return U


def rhs(case, U):
    """Right-hand side R(U) (padded, halo entries zero)."""
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64).copy()
    R = np.zeros_like(U)
    _ok(lib.oracle_rhs(C.byref(cfg), _ptr(U), _ptr(R)))
    return R


def cfl_dt(case, U, t=0.0, t_end=0.0):
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64)
    return float(lib.oracle_dt(C.byref(cfg), _ptr(U), float(t), float(t_end)))


def rk3_step(case, U, dt=0.0):
    """One TVD-RK3 step (dt <= 0: CFL step). Returns (U_new, dt_used)."""
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64).copy()
    dtu = C.c_double(0.0)
    _ok(lib.oracle_rk3_step(C.byref(cfg), _ptr(U), float(dt), C.byref(dtu)))
    return U, dtu.value


def advance(case, U, n_steps, t_end=0.0, fixed_dt=0.0, t=0.0):
    """Up to n_steps steps, stopping at t_end (> 0). Returns (U, t, steps_taken)."""
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64).copy()
    tt = C.c_double(float(t))
    n = lib.oracle_advance(C.byref(cfg), _ptr(U), int(n_steps), float(t_end), float(fixed_dt),
                           C.byref(tt))
    if n < 0:
        raise ValueError("oracle rejected the configuration")
    return U, tt.value, int(n)


def status(clear=True):
    """Health word of the calling thread since the last clear: bit 0 a
    non-finite conservative value, bit 1 rho <= 0, bit 2 p <= 0 in a step's
    input, stage or output state; bit 3 a reconstructed face state with
    rho <= 0 or p <= 0."""
    return int(_load().oracle_status(1 if clear else 0))


def weno5(a, b, c, d, e):
    return float(_load().oracle_weno5(float(a), float(b), float(c), float(d), float(e)))


def weno5z(a, b, c, d, e):
    return float(_load().oracle_weno5z(float(a), float(b), float(c), float(d), float(e)))


def hllc(gamma, WL, WR, axis):
    lib = _load()
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(5)
    lib.oracle_hllc(float(gamma), _ptr(WL), _ptr(WR), int(axis), _ptr(F))
    return F


def einfeldt(gamma, WL, WR, axis):
    """The Einfeldt signal speeds of the HLLC flux at a face: (ubar, dbar, S_L, S_R)."""
    lib = _load()
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    out = np.zeros(4)
    lib.oracle_einfeldt(float(gamma), _ptr(WL), _ptr(WR), int(axis), _ptr(out))
    return out


def roe_eigen(gamma, wl, wr, axis):
    """Roe average of primitive states wl | wr along `axis`: (R, L, lam) with
    the right eigenvectors as the columns of R, L = R^-1 (by elimination)."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    R = np.zeros(25)
    L = np.zeros(25)
    lam = np.zeros(5)
    _load().oracle_roe_eigen(float(gamma), _ptr(wl), _ptr(wr), int(axis), _ptr(R), _ptr(L), _ptr(lam))
    return R.reshape(5, 5), L.reshape(5, 5), lam


def roe_flux(gamma, w6, axis):
    """Roe flux-splitting convective flux at the face between the third and
    fourth of six primitive states w6 (6 x 5)."""
    w6 = np.ascontiguousarray(w6, dtype=np.float64).reshape(30)
    F = np.zeros(5)
    _load().oracle_roe_flux(float(gamma), _ptr(w6), int(axis), _ptr(F))
    return F


def weno3(a, b, c):
    return float(_load().oracle_weno3(float(a), float(b), float(c)))


def rusanov(gamma, WL, WR, axis):
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(5)
    _load().oracle_rusanov(float(gamma), _ptr(WL), _ptr(WR), int(axis), _ptr(F))
    return F


def euler_flux(gamma, w, axis):
    w = np.ascontiguousarray(w, dtype=np.float64)
    F = np.zeros(5)
    _load().oracle_euler_flux(float(gamma), _ptr(w), int(axis), _ptr(F))
    return F


def opcount(case, U):
    """Operation counts of one right-hand side: dict add/mul/div/sqrt/cmp."""
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros(5)
    _ok(lib.oracle_opcount(C.byref(cfg), _ptr(U), _ptr(out)))
    return dict(zip(("add", "mul", "div", "sqrt", "cmp"), out.tolist()))


def opcount_parts(case, U):
    """Flops (add+mul+div+sqrt) of the parts of one right-hand side:
    {"prim_per_cell", "face": [x, y, z]} (one face flux each)."""
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros(4)
    _ok(lib.oracle_opcount_parts(C.byref(cfg), _ptr(U), _ptr(out)))
    return {"prim_per_cell": float(out[0]), "face": [float(x) for x in out[1:]]}


def vjp_rhs(case, U, Rbar):
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64)
    Rbar = np.ascontiguousarray(Rbar, dtype=np.float64)
    Ubar = np.zeros_like(U)
    _ok(lib.oracle_vjp_rhs(C.byref(cfg), _ptr(U), _ptr(Rbar), _ptr(Ubar)))
    return Ubar


def vjp_state_init(case, W, Ubar):
    """Wbar = (dU/dW)^T Ubar for U = state_init(case, W) (halo entries of Ubar count)."""
    lib = _load()
    cfg = make_cfg(case)
    W = np.ascontiguousarray(W, dtype=np.float64)
    Ubar = np.ascontiguousarray(Ubar, dtype=np.float64)
    Wbar = np.zeros_like(W)
    _ok(lib.oracle_vjp_state_init(C.byref(cfg), _ptr(W), _ptr(Ubar), _ptr(Wbar)))
    return Wbar


def vjp_rk3_step(case, Un, dt, Ubar_np1):
    lib = _load()
    cfg = make_cfg(case)
    Un = np.ascontiguousarray(Un, dtype=np.float64)
    Ubar_np1 = np.ascontiguousarray(Ubar_np1, dtype=np.float64)
    Ubar_n = np.zeros_like(Un)
    _ok(lib.oracle_vjp_rk3_step(C.byref(cfg), _ptr(Un), float(dt), _ptr(Ubar_np1), _ptr(Ubar_n)))
    return Ubar_n


def grad_kinetic_energy(case, W0, n_steps, dt):
    """Loss = total kinetic energy after n_steps fixed-dt steps from primitive W0,
    and its gradient with respect to the initial (u, v, w). Returns (L, grad(3, nz, ny, nx))."""
    lib = _load()
    cfg = make_cfg(case)
    W0 = np.ascontiguousarray(W0, dtype=np.float64)
    g = np.zeros((3,) + W0.shape[1:])
    L = C.c_double(0.0)
    _ok(lib.oracle_grad_ke(C.byref(cfg), _ptr(W0), int(n_steps), float(dt), C.byref(L), _ptr(g)))
    return L.value, g


def rhs_rounding_bound(case, U, k=16.0):
    """Per-variable absolute tolerance for comparing two evaluations of the
    right-hand side that differ only in rounding (operation order, fused
    multiply-adds). R_i is a difference of face fluxes whose magnitude is
    bounded by |F_d| + (|u_d| + c)|U| (physical flux plus the Riemann solver's
    dissipation), so rounding errors of relative size eps in those fluxes give
    errors up to about eps * sum_d 2 (|F_d| + (|u_d| + c)|U|)/dx_d in R_i,
    however small R_i itself is. Returns k * eps * max_i of that scale, per
    conservative variable (k covers the few roundings per flux)."""
    Ui = interior(case, np.asarray(U, dtype=np.float64))
    g = float(case["gamma"])
    rho = Ui[0]
    u = Ui[1:4] / rho
    E = Ui[4]
    p = (g - 1.0) * (E - 0.5 * (Ui[1] * u[0] + Ui[2] * u[1] + Ui[3] * u[2]))
    c = np.sqrt(np.abs(g * p / rho))
    cons = [rho, Ui[1], Ui[2], Ui[3], E]
    scale = np.zeros(5)
    acc = [np.zeros_like(rho) for _ in range(5)]
    for d in range(3):
        if int(case["n"][d]) <= 1:
            continue
        dx = (case["hi"][d] - case["lo"][d]) / case["n"][d]
        ud = u[d]
        F = [rho * ud, Ui[1] * ud, Ui[2] * ud, Ui[3] * ud, ud * (E + p)]
        F[1 + d] = F[1 + d] + p
        for v in range(5):
            acc[v] += 2.0 * (np.abs(F[v]) + (np.abs(ud) + c) * np.abs(cons[v])) / dx
    for v in range(5):
        scale[v] = float(acc[v].max())
    return k * np.finfo(np.float64).eps * scale


# --------------------------------------------------------------------------
# Rusanov-NN flux (§7.4): Rusanov with alpha = exp(MLP(|du|, u_M, c_M, |ds|)),
# three hidden ReLU layers of 32 units; NN_PARAMS weights in the order
# W1 (32x4), b1, W2 (32x32), b2, W3 (32x32), b3, W4 (1x32), b4.
NN_PARAMS = 2305


def set_nn(theta):
    """Network weights used by every later call whose flags carry the Rusanov-NN
    flux (256); None clears them."""
    lib = _load()
    if theta is None:
        lib.oracle_set_nn(None)
        return
    th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    if th.size != NN_PARAMS:
        raise ValueError(f"expected {NN_PARAMS} weights, got {th.size}")
    lib.oracle_set_nn(_ptr(th))


def nn_alpha(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return float(_load().oracle_nn_alpha(_ptr(f)))


def rusanov_nn(gamma, WL, WR, axis):
    lib = _load()
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(5)
    _ok(lib.oracle_rusanov_nn(float(gamma), _ptr(WL), _ptr(WR), int(axis), _ptr(F)))
    return F


def vjp_rhs_theta(case, U, Rbar):
    """(Ubar, theta_bar) for R = rhs(U) with the Rusanov-NN flux."""
    lib = _load()
    cfg = make_cfg(case)
    U = np.ascontiguousarray(U, dtype=np.float64)
    Rbar = np.ascontiguousarray(Rbar, dtype=np.float64)
    Ubar = np.zeros_like(U)
    tb = np.zeros(NN_PARAMS)
    _ok(lib.oracle_vjp_rhs_theta(C.byref(cfg), _ptr(U), _ptr(Rbar), _ptr(Ubar), _ptr(tb)))
    return Ubar, tb


def vjp_step_theta(case, Un, dt, Ubar_np1):
    """(Ubar_n, theta_bar) for one fixed-dt step with the Rusanov-NN flux."""
    lib = _load()
    cfg = make_cfg(case)
    Un = np.ascontiguousarray(Un, dtype=np.float64)
    Ub = np.ascontiguousarray(Ubar_np1, dtype=np.float64)
    out = np.zeros_like(Un)
    tb = np.zeros(NN_PARAMS)
    _ok(lib.oracle_vjp_step_theta(C.byref(cfg), _ptr(Un), float(dt), _ptr(Ub), _ptr(out), _ptr(tb)))
    return out, tb
