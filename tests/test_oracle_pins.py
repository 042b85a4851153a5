"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(no GPU). Each test would fail under a plausible mistake in the oracle: a
dropped term, a wrong sign or index, a transposed operand, a wrong coefficient.

  P1  Sod's shock tube vs the exact Riemann solution (§5.1.2)
  P2  fifth-order convergence on the advected entropy wave (§5.1.1)
  P3  discrete conservation on periodic grids (§3.1, Eq. FVD telescopes)
  P4  free-stream preservation, bitwise
  P5  dissipative operator against closed forms (§2 stresses/heat flux, §3.4 stencils)
  P6  HLLC special cases (consistency, upwinding, stationary contact, symmetry)
  P7  WENO5-JS and WENO5-Z special cases (constants, exact on quadratics, ENO at a jump)
  P8  TVD-RK3 third order in time (§3.2)
  P9  the taped reverse-mode derivative against central finite differences
"""
import math

import numpy as np
import pytest

import oracle
from exact_riemann import ExactRiemann
from paper_2203_13760_amd import workloads as wl

GOLDEN = __file__.rsplit("/", 1)[0] + "/golden/"


def _golden(name):
    rows = {}
    for line in open(GOLDEN + name):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v, tol = line.split()
        rows[k] = (float(v), float(tol))
    return rows


# ---------------------------------------------------------------- P1 -------
def test_exact_riemann_solver_matches_published_star_state():
    e = ExactRiemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma=1.4)
    g = _golden("sod_star_state.txt")
    got = {"p_star": e.p_star, "u_star": e.u_star, "rho_star_L": e.rho_star_L,
           "rho_star_R": e.rho_star_R, "shock_speed": e.shock_speed_right()}
    for k, (v, tol) in g.items():
        assert abs(got[k] - v) <= tol, (k, got[k], v)


def _sod_run(n):
    case, W = wl.sod(n)
    U = oracle.state_init(case, W)
    U, t, steps = oracle.advance(case, U, 100000, t_end=case["t_end"])
    assert abs(t - 0.2) < 1e-14
    Ui = oracle.interior(case, U).reshape(5, n)
    rho = Ui[0]
    u = Ui[1] / rho
    p = 0.4 * (Ui[4] - 0.5 * Ui[1] * u)
    return rho, u, p, steps


def test_sod_shock_tube_against_exact_solution():
    e = ExactRiemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    l1 = {}
    for n in (100, 200, 400):
        rho, u, p, steps = _sod_run(n)
        ra, _, _ = e.cell_average_profile(n, 0.2)
        l1[n] = float(np.mean(np.abs(rho - ra)))
        x = (np.arange(n) + 0.5) / n
        if n == 200:
            assert 120 <= steps <= 200
            # plateaus: between rarefaction tail (0.486) and contact (0.685), and
            # between contact and shock (0.850)
            m1 = (x > 0.52) & (x < 0.66)
            m2 = (x > 0.71) & (x < 0.83)
            assert np.max(np.abs(rho[m1] - e.rho_star_L)) < 2e-3
            assert np.max(np.abs(rho[m2] - e.rho_star_R)) < 2e-3
            assert np.max(np.abs(p[m1 | m2] - e.p_star)) < 2e-3
            assert np.max(np.abs(u[m1 | m2] - e.u_star)) < 3e-3
            # untouched far field
            assert np.all(np.abs(rho[x < 0.1] - 1.0) < 1e-10)
            assert np.all(np.abs(rho[x > 0.95] - 0.125) < 1e-10)
    assert l1[200] <= 5e-3
    assert l1[100] > l1[200] > l1[400]


def test_lax_shock_tube_against_exact_solution():
    """Lax's shock tube at t = 0.14 (§5.1.2, N = 100 on [0,1] in the paper):
    the density error against the exact solution falls with the grid, the
    plateau between contact and shock sits at the exact star density, and
    the undisturbed ends are untouched."""
    e = ExactRiemann((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))
    l1 = {}
    for n in (100, 200, 400):
        case, W = wl.lax(n)
        U = oracle.state_init(case, W)
        U, t, steps = oracle.advance(case, U, 100000, t_end=case["t_end"])
        assert abs(t - 0.14) < 1e-14
        Ui = oracle.interior(case, U).reshape(5, n)
        rho = Ui[0]
        ra, _, _ = e.cell_average_profile(n, 0.14)
        l1[n] = float(np.mean(np.abs(rho - ra)))
        x = (np.arange(n) + 0.5) / n
        if n == 400:
            # contact at 0.714, shock at 0.847
            m = (x > 0.74) & (x < 0.83)
            assert np.max(np.abs(rho[m] - e.rho_star_R)) < 2e-2
            assert np.all(np.abs(rho[x > 0.95] - 0.5) < 1e-10)
    assert l1[100] <= 0.015
    assert l1[100] > l1[200] > l1[400]


# ---------------------------------------------------------------- P2 -------
def _entropy_error(n, dt=1e-4, t_end=1.0):
    case, W = wl.entropy_wave(n)
    U0 = oracle.state_init(case, W)
    U, t, _ = oracle.advance(case, U0, 10 ** 7, t_end=t_end, fixed_dt=dt)
    assert abs(t - t_end) < 1e-10
    return float(np.mean(np.abs(oracle.interior(case, U)[0] - oracle.interior(case, U0)[0])))


def test_entropy_wave_fifth_order_convergence():
    ns = (20, 40, 80, 160, 320)
    err = np.array([_entropy_error(n) for n in ns])
    order = np.log2(err[:-1] / err[1:])
    assert np.all(order[-2:] >= 4.7), order
    assert err[-1] < 5e-9


# ---------------------------------------------------------------- P8 -------
def test_tvd_rk3_third_order_in_time():
    # same grid, dt halved: the spatial error cancels in the difference to a
    # fine-dt reference, leaving the temporal error of the RK3 scheme
    n, t_end = 40, 0.5
    case, W = wl.entropy_wave(n)
    U0 = oracle.state_init(case, W)
    ref, _, _ = oracle.advance(case, U0, 10 ** 7, t_end=t_end, fixed_dt=0.01 / 64)
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        U, t, _ = oracle.advance(case, U0, 10 ** 7, t_end=t_end, fixed_dt=dt)
        errs.append(float(np.max(np.abs(U - ref))))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 3.0) < 0.25), order


# ---------------------------------------------------------------- P3 -------
def test_discrete_conservation_periodic():
    case, W = wl.taylor_green(0, shape=(12, 10, 8))
    U = oracle.state_init(case, W)
    R = oracle.interior(case, oracle.rhs(case, U))
    for v in range(5):
        s = math.fsum(R[v].ravel().tolist())
        assert abs(s) <= 1e-13 * np.abs(R[v]).sum() + 1e-300, (v, s)
    U2, _, _ = oracle.advance(case, U, 20)
    a, b = oracle.interior(case, U), oracle.interior(case, U2)
    scale = [np.abs(a[0]).sum(), np.abs(a[1:4]).sum(), np.abs(a[1:4]).sum(), np.abs(a[1:4]).sum(),
             np.abs(a[4]).sum()]
    for v in range(5):
        s0 = math.fsum(a[v].ravel().tolist())
        s1 = math.fsum(b[v].ravel().tolist())
        assert abs(s1 - s0) <= 1e-13 * scale[v], (v, s0, s1)


# ---------------------------------------------------------------- P4 -------
@pytest.mark.parametrize("bc", [wl.PERIODIC, wl.ZERO_GRADIENT])
def test_free_stream_preserved_bitwise(bc):
    case = wl.make_case((9, 7, 6), bc=(bc,) * 6, mu=0.05, flags=wl.ALL_PHYSICS)
    W = np.empty((5, 6, 7, 9))
    for v, val in enumerate((1.3, 0.3, -0.2, 0.1, 0.8)):
        W[v] = val
    U = oracle.state_init(case, W)
    R = oracle.rhs(case, U)
    assert np.all(R == 0.0)
    U2, _, _ = oracle.advance(case, U, 10)
    assert np.array_equal(U2, U)


# ---------------------------------------------------------------- P5 -------
def test_viscous_shear_wave_closed_form():
    # u = 0, v = sin 2 pi x (point values), rho = p = 1, viscous flux only:
    # d(rho v)/dt = mu (v'(x_{i+1/2}) - v'(x_{i-1/2})) / dx, fourth order
    mu = 0.1
    errs = []
    for n in (16, 32, 64):
        case = wl.make_case((n, 1, 1), mu=mu, flags=wl.VISCOUS)
        x = wl.cell_centres(case, 0)
        W = np.zeros((5, 1, 1, n))
        W[0] = 1.0
        W[2] = np.sin(2 * np.pi * x)
        W[4] = 1.0
        R = oracle.interior(case, oracle.rhs(case, oracle.state_init(case, W))).reshape(5, n)
        dx = 1.0 / n
        exact = mu * 2 * np.pi * (np.cos(2 * np.pi * (x + dx / 2)) - np.cos(2 * np.pi * (x - dx / 2))) / dx
        errs.append(np.max(np.abs(R[2] - exact)))
        assert np.all(R[0] == 0.0) and np.max(np.abs(R[1])) < 1e-14
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 3.8), order


def test_heat_conduction_closed_form():
    # rho = 1 + 0.1 sin 2 pi x, p = 1, u = 0, heat flux only: the energy
    # right-hand side is kappa (T'(x_{i+1/2}) - T'(x_{i-1/2}))/dx with T = p/rho,
    # kappa = gamma mu / ((gamma-1) Pr)
    mu, pr, g = 0.05, 0.72, 1.4
    kappa = g * mu / ((g - 1) * pr)
    errs = []
    for n in (16, 32, 64):
        case = wl.make_case((n, 1, 1), mu=mu, prandtl=pr, gamma=g, flags=wl.HEAT)
        x = wl.cell_centres(case, 0)
        W = np.zeros((5, 1, 1, n))
        W[0] = 1.0 + 0.1 * np.sin(2 * np.pi * x)
        W[4] = 1.0
        R = oracle.interior(case, oracle.rhs(case, oracle.state_init(case, W))).reshape(5, n)
        dx = 1.0 / n
        dT = lambda s: -0.2 * np.pi * np.cos(2 * np.pi * s) / (1 + 0.1 * np.sin(2 * np.pi * s)) ** 2
        exact = kappa * (dT(x + dx / 2) - dT(x - dx / 2)) / dx
        errs.append(np.max(np.abs(R[4] - exact)))
        assert np.all(R[:4] == 0.0)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 3.7), order


def test_viscous_tgv_momentum_is_minus_three_mu_u():
    # divergence-free TGV velocity, uniform rho and p, viscous flux only: the
    # momentum right-hand side approaches mu lap(u) = -3 mu u (second order,
    # since point values are compared with face-flux differences)
    mu = 0.01
    errs = []
    for n in (16, 32, 64):
        case, W = wl.taylor_green(n)
        case["mu"] = mu
        case["flags"] = wl.VISCOUS
        W[4] = 1.0
        R = oracle.interior(case, oracle.rhs(case, oracle.state_init(case, W)))
        err = max(np.max(np.abs(R[1] + 3 * mu * W[1])), np.max(np.abs(R[2] + 3 * mu * W[2])),
                  np.max(np.abs(R[3])))
        errs.append(err)
        assert np.all(R[0] == 0.0)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 1.9), order


# ---------------------------------------------------------------- P6 -------
def _phys_flux(W, d, g=1.4):
    rho, u, p = W[0], W[1:4], W[4]
    E = p / (g - 1) + 0.5 * rho * np.dot(u, u)
    F = np.zeros(5)
    F[0] = rho * u[d]
    F[1:4] = rho * u[d] * u
    F[1 + d] += p
    F[4] = u[d] * (E + p)
    return F


def test_hllc_special_cases():
    rng = np.random.default_rng(1)
    for _ in range(20):
        W = np.array([rng.uniform(0.2, 2), *rng.uniform(-1, 1, 3), rng.uniform(0.2, 2)])
        for d in range(3):
            F = oracle.hllc(1.4, W, W, d)
            np.testing.assert_allclose(F, _phys_flux(W, d), rtol=1e-13, atol=1e-13)
    # supersonic to the right: exactly the left physical flux; to the left: the right one
    WL = np.array([1.0, 5.0, 0.1, -0.2, 1.0])
    WR = np.array([0.5, 4.0, 0.0, 0.3, 0.8])
    assert np.array_equal(oracle.hllc(1.4, WL, WR, 0), oracle.hllc(1.4, WL, WL, 0)) or \
        np.allclose(oracle.hllc(1.4, WL, WR, 0), _phys_flux(WL, 0), rtol=1e-14)
    np.testing.assert_allclose(oracle.hllc(1.4, WL, WR, 0), _phys_flux(WL, 0), rtol=1e-14)
    WL2 = np.array([1.0, -5.0, 0.1, -0.2, 1.0])
    WR2 = np.array([0.5, -4.0, 0.0, 0.3, 0.8])
    np.testing.assert_allclose(oracle.hllc(1.4, WL2, WR2, 0), _phys_flux(WR2, 0), rtol=1e-14)
    # stationary contact: density jump, equal pressure, no motion
    F = oracle.hllc(1.4, np.array([1.0, 0, 0, 0, 0.7]), np.array([0.2, 0, 0, 0, 0.7]), 0)
    assert abs(F[0]) < 1e-15 and abs(F[4]) < 1e-15
    assert abs(F[1] - 0.7) < 1e-15 and abs(F[2]) < 1e-15 and abs(F[3]) < 1e-15
    # mirror symmetry: reflecting x -> -x swaps the states and negates normal velocity
    for _ in range(20):
        WL = np.array([rng.uniform(0.2, 2), *rng.uniform(-2, 2, 3), rng.uniform(0.2, 2)])
        WR = np.array([rng.uniform(0.2, 2), *rng.uniform(-2, 2, 3), rng.uniform(0.2, 2)])
        F = oracle.hllc(1.4, WL, WR, 0)
        m = lambda W: np.array([W[0], -W[1], W[2], W[3], W[4]])
        Fm = oracle.hllc(1.4, m(WR), m(WL), 0)
        np.testing.assert_allclose([-Fm[0], Fm[1], -Fm[2], -Fm[3], -Fm[4]], F, rtol=1e-12, atol=1e-12)
        # rotation: the y-face flux of states with (u,v,w) -> (w,u,v) equals the
        # x-face flux with the momentum slots rotated the same way
        rot = lambda W: np.array([W[0], W[3], W[1], W[2], W[4]])
        Fy = oracle.hllc(1.4, rot(WL), rot(WR), 1)
        np.testing.assert_allclose(Fy, [F[0], F[3], F[1], F[2], F[4]], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- P7 -------
def test_weno5_special_cases():
    for c in (0.0, 1.0, -3.7, 1e5, 2.5e-3):
        assert abs(oracle.weno5(c, c, c, c, c) - c) <= 2 * np.spacing(abs(c) + 1e-300)
    # exact for cell averages of any quadratic, whatever the nonlinear weights
    rng = np.random.default_rng(2)
    for _ in range(20):
        a0, a1, a2 = rng.uniform(-1, 1, 3)
        h = rng.uniform(0.05, 1.0)
        P = lambda x: a0 * x + a1 * x ** 2 / 2 + a2 * x ** 3 / 3  # primitive of q
        q = lambda x: a0 + a1 * x + a2 * x ** 2
        avg = [(P((m + 0.5) * h) - P((m - 0.5) * h)) / h for m in (-2, -1, 0, 1, 2)]
        assert abs(oracle.weno5(*avg) - q(0.5 * h)) < 1e-12
    # essentially non-oscillatory at a jump right of the centre cell
    assert abs(oracle.weno5(0, 0, 0, 1, 1)) < 1e-10
    assert abs(oracle.weno5(1, 1, 1, 0, 0) - 1) < 1e-10
    # smooth data: approaches the fifth-order linear combination (2a-13b+47c+27d-3e)/60
    for h in (0.1, 0.05, 0.025):
        avg = [(-np.cos(2 * (m + 0.5) * h) + np.cos(2 * (m - 0.5) * h)) / (2 * h) for m in (-2, -1, 0, 1, 2)]
        lin = (2 * avg[0] - 13 * avg[1] + 47 * avg[2] + 27 * avg[3] - 3 * avg[4]) / 60
        assert abs(oracle.weno5(*avg) - lin) < 50 * h ** 4


def test_weno5z_special_cases():
    """WENO5-Z (Borges et al. 2008): the same candidates as WENO5-JS, so the
    same exactness on constants and quadratics and the same ENO property; on
    smooth data its weights lie closer to the linear ones, so it sits closer
    to the fifth-order linear combination than WENO5-JS (an order of h
    better: the weights deviate by O(h^3) instead of O(h^2) at a smooth
    extremum-free point)."""
    # (the weights stay the linear ones here, so only the candidates' rounding remains)
    for c in (0.0, 1.0, -3.7, 1e5, 2.5e-3):
        assert abs(oracle.weno5z(c, c, c, c, c) - c) <= 4 * np.spacing(abs(c) + 1e-300)
    rng = np.random.default_rng(3)
    for _ in range(20):
        a0, a1, a2 = rng.uniform(-1, 1, 3)
        h = rng.uniform(0.05, 1.0)
        P = lambda x: a0 * x + a1 * x ** 2 / 2 + a2 * x ** 3 / 3
        q = lambda x: a0 + a1 * x + a2 * x ** 2
        avg = [(P((m + 0.5) * h) - P((m - 0.5) * h)) / h for m in (-2, -1, 0, 1, 2)]
        assert abs(oracle.weno5z(*avg) - q(0.5 * h)) < 1e-12
    assert abs(oracle.weno5z(0, 0, 0, 1, 1)) < 1e-10
    assert abs(oracle.weno5z(1, 1, 1, 0, 0) - 1) < 1e-10
    dz, djs = [], []
    for h in (0.1, 0.05, 0.025):
        avg = [(-np.cos(2 * (m + 0.5) * h + 0.3) + np.cos(2 * (m - 0.5) * h + 0.3)) / (2 * h)
               for m in (-2, -1, 0, 1, 2)]
        lin = (2 * avg[0] - 13 * avg[1] + 47 * avg[2] + 27 * avg[3] - 3 * avg[4]) / 60
        dz.append(abs(oracle.weno5z(*avg) - lin))
        djs.append(abs(oracle.weno5(*avg) - lin))
    assert all(z < j for z, j in zip(dz, djs)), (dz, djs)
    assert math.log2(dz[1] / dz[2]) > math.log2(djs[1] / djs[2]) + 0.5, (dz, djs)


def test_weno5z_entropy_wave_fifth_order_and_shock_tubes():
    """WENO5-Z through the whole oracle: fifth order on the entropy wave, and
    Sod and Lax against their exact solutions."""
    errs = []
    for n in (20, 40, 80, 160):
        case, W = wl.entropy_wave(n)
        case["flags"] |= wl.WENOZ
        U0 = oracle.state_init(case, W)
        U, t, _ = oracle.advance(case, U0, 10 ** 7, t_end=1.0, fixed_dt=1e-4)
        errs.append(float(np.mean(np.abs(oracle.interior(case, U)[0] - oracle.interior(case, U0)[0]))))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= 4.7, order
    for make, left, right, t_end in ((wl.sod, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2),
                                      (wl.lax, (0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.14)):
        e = ExactRiemann(left, right)
        l1 = []
        for n in (100, 200):
            case, W = make(n)
            case["flags"] |= wl.WENOZ
            U, t, _ = oracle.advance(case, oracle.state_init(case, W), 100000, t_end=t_end)
            rho = oracle.interior(case, U).reshape(5, n)[0]
            l1.append(float(np.mean(np.abs(rho - e.cell_average_profile(n, t_end)[0]))))
        assert l1[0] > l1[1] and l1[0] < 0.015, (make.__name__, l1)


# ---------------------------------------------------------------- ROE ------
def _cons(w, g=1.4):
    return np.array([w[0], w[0] * w[1], w[0] * w[2], w[0] * w[3],
                     w[4] / (g - 1) + 0.5 * w[0] * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2)])


def _prim(U, g=1.4):
    u = U[1:4] / U[0]
    return np.array([U[0], *u, (g - 1) * (U[4] - 0.5 * U[0] * np.dot(u, u))])


def test_roe_decomposition_pins():
    """The Roe matrix A = R Lambda R^-1 (§3.3 flux splitting, step 2): R^-1 R = I;
    the eigenvalues are u_d - a, u_d, u_d, u_d, u_d + a; A (U_R - U_L) =
    F(U_R) - F(U_L) exactly for any two states (Roe's defining property); for
    equal states A is the flux Jacobian (central differences of the Euler flux
    in the conservative variables)."""
    rng = np.random.default_rng(7)
    g = 1.4
    for t in range(60):
        d = t % 3
        wl = np.array([rng.uniform(0.2, 3), *rng.uniform(-2, 2, 3), rng.uniform(0.1, 4)])
        wr = np.array([rng.uniform(0.2, 3), *rng.uniform(-2, 2, 3), rng.uniform(0.1, 4)])
        R, L, lam = oracle.roe_eigen(g, wl, wr, d)
        assert np.allclose(L @ R, np.eye(5), rtol=0, atol=1e-12)
        # eigenvalues from the Roe-averaged state, computed here independently
        sl, sr = np.sqrt(wl[0]), np.sqrt(wr[0])
        Hl = g / (g - 1) * wl[4] / wl[0] + 0.5 * np.dot(wl[1:4], wl[1:4])
        Hr = g / (g - 1) * wr[4] / wr[0] + 0.5 * np.dot(wr[1:4], wr[1:4])
        u = (sl * wl[1:4] + sr * wr[1:4]) / (sl + sr)
        H = (sl * Hl + sr * Hr) / (sl + sr)
        a = np.sqrt((g - 1) * (H - 0.5 * np.dot(u, u)))
        assert np.allclose(lam, [u[d] - a, u[d], u[d], u[d], u[d] + a], rtol=0, atol=1e-13)
        A = R @ np.diag(lam) @ L
        dU = _cons(wr) - _cons(wl)
        dF = oracle.euler_flux(g, wr, d) - oracle.euler_flux(g, wl, d)
        assert np.max(np.abs(A @ dU - dF)) <= 1e-12 * np.max(np.abs(dF)), t
        # equal states: the Jacobian dF/dU by central differences
        R0, L0, lam0 = oracle.roe_eigen(g, wl, wl, d)
        A0 = R0 @ np.diag(lam0) @ L0
        U0 = _cons(wl)
        J = np.empty((5, 5))
        for k in range(5):
            h = 1e-6 * max(1.0, abs(U0[k]))
            e = np.zeros(5)
            e[k] = h
            J[:, k] = (oracle.euler_flux(g, _prim(U0 + e), d) - oracle.euler_flux(g, _prim(U0 - e), d)) / (2 * h)
        assert np.allclose(A0, J, rtol=1e-7, atol=1e-7), t


def test_roe_flux_special_cases():
    """A constant stencil gives the exact Euler flux; mirroring the stencil and
    flipping the normal velocity flips the mass and energy flux (reflection
    symmetry of the split scheme)."""
    rng = np.random.default_rng(8)
    g = 1.4
    for d in range(3):
        w = np.array([1.3, 0.4, -0.7, 0.2, 2.1])
        F = oracle.roe_flux(g, np.tile(w, (6, 1)), d)
        assert np.allclose(F, oracle.euler_flux(g, w, d), rtol=1e-14, atol=1e-14)
        w6 = np.column_stack([rng.uniform(0.3, 2, 6), rng.uniform(-1, 1, (6, 3)), rng.uniform(0.3, 2, 6)])
        m6 = w6[::-1].copy()
        m6[:, 1 + d] *= -1.0
        F1 = oracle.roe_flux(g, w6, d)
        F2 = oracle.roe_flux(g, m6, d)
        sign = np.ones(5)
        sign[[0, 4]] = -1.0
        t = [a for a in range(3) if a != d]
        sign[1 + t[0]] = sign[1 + t[1]] = -1.0
        assert np.allclose(F2, sign * F1, rtol=1e-11, atol=1e-12), (d, F1, F2)


def test_roe_setup_through_the_oracle():
    """The ROE setup through the whole oracle: fifth order on the entropy wave,
    Sod and Lax against their exact solutions, conservation on a periodic grid
    and bitwise free-stream preservation."""
    errs = []
    for n in (20, 40, 80, 160):
        case, W = wl.entropy_wave(n)
        case["flags"] |= wl.ROE
        U0 = oracle.state_init(case, W)
        U, t, _ = oracle.advance(case, U0, 10 ** 7, t_end=1.0, fixed_dt=1e-4)
        errs.append(float(np.mean(np.abs(oracle.interior(case, U)[0] - oracle.interior(case, U0)[0]))))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= 4.7, order
    for make, left, right, t_end in ((wl.sod, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2),
                                      (wl.lax, (0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.14)):
        e = ExactRiemann(left, right)
        l1 = []
        for n in (100, 200, 400):
            case, W = make(n)
            case["flags"] |= wl.ROE
            U, t, _ = oracle.advance(case, oracle.state_init(case, W), 100000, t_end=t_end)
            rho = oracle.interior(case, U).reshape(5, n)[0]
            l1.append(float(np.mean(np.abs(rho - e.cell_average_profile(n, t_end)[0]))))
        assert l1[0] > l1[1] > l1[2] and l1[0] < 0.015, (make.__name__, l1)
    case, W = wl.taylor_green(0, shape=(12, 10, 8))
    case["flags"] |= wl.ROE
    R = oracle.interior(case, oracle.rhs(case, oracle.state_init(case, W)))
    for v in range(5):
        s = math.fsum(R[v].ravel().tolist())
        assert abs(s) <= 1e-13 * np.abs(R[v]).sum() + 1e-300, (v, s)
    for bc in (wl.PERIODIC, wl.ZERO_GRADIENT):
        case = wl.make_case((9, 7, 6), bc=(bc,) * 6, mu=0.05, flags=wl.ALL_PHYSICS | wl.ROE)
        W = np.empty((5, 6, 7, 9))
        for v, val in enumerate((1.3, 0.3, -0.2, 0.1, 0.8)):
            W[v] = val
        U = oracle.state_init(case, W)
        assert np.all(oracle.rhs(case, U) == 0.0)


# ---------------------------------------------------------------- implosion substrate (§7.4)
def _mirror_pair(axis, n=24, steps=30, flags=wl.INVISCID, dt=2e-3):
    """A state on [0,1] along `axis` with reflecting walls at both ends, and the
    same state mirrored onto [0,2] with periodic ends (density and pressure
    even about x = 1, the normal velocity odd): the walled run must equal the
    first half of the periodic one."""
    other = 7 if axis == 1 else 1
    nw = [1, 1, 1]
    nw[axis] = n
    if axis == 1:
        nw[0] = other
    bcw = [wl.PERIODIC] * 6
    bcw[2 * axis] = bcw[2 * axis + 1] = wl.REFLECT
    hi = [1.0, 1.0, 1.0]
    cw = wl.make_case(tuple(nw), bc=tuple(bcw), flags=flags)
    nf = list(nw)
    nf[axis] = 2 * n
    hi[axis] = 2.0
    cf = wl.make_case(tuple(nf), hi=tuple(hi), bc=(wl.PERIODIC,) * 6, flags=flags)
    shape = (nw[2], nw[1], nw[0])
    x = (np.arange(n) + 0.5) / n
    prof = lambda a, k: a + 0.3 * np.sin(np.pi * k * x) + 0.2 * (x > 0.4 + 0.1 * k)
    Ww = np.empty((5,) + shape)
    cols = [prof(1.0, 1), 0.4 * np.sin(np.pi * x) * (1.0 + 0.5 * x), 0.2 * np.cos(3 * x), 0.1 * x, prof(1.5, 2)]
    for v in range(5):
        f = cols[v]
        f = f.reshape((1, n, 1)) if axis == 1 else f.reshape((1, 1, n))
        Ww[v] = np.broadcast_to(f, shape)
    Wf = np.concatenate([Ww, np.flip(Ww, axis=3 - axis)], axis=3 - axis)
    Wf[1 + axis] = np.concatenate([Ww[1 + axis], -np.flip(Ww[1 + axis], axis=2 - axis)], axis=2 - axis)
    Uw, _, _ = oracle.advance(cw, oracle.state_init(cw, Ww), steps, fixed_dt=dt)
    Uf, _, _ = oracle.advance(cf, oracle.state_init(cf, Wf), steps, fixed_dt=dt)
    iw = oracle.interior(cw, Uw)
    i_f = oracle.interior(cf, Uf)
    half = [slice(None)] * 4
    half[3 - axis] = slice(0, n)
    return iw, i_f[tuple(half)]


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("flags", [wl.INVISCID, wl.INVISCID | wl.WENO3 | wl.RK2 | wl.RUSANOV])
def test_reflecting_wall_equals_mirrored_periodic_domain(axis, flags):
    """Reflecting walls (the implosion of §7.4): the walled run equals the
    first half of the run on the mirrored domain twice as long, for a jump and
    a smooth profile, along x and along y (the sign flip must hit the wall's
    normal momentum and only it)."""
    a, b = _mirror_pair(axis, flags=flags)
    scale = np.abs(b).reshape(5, -1).max(axis=1) + 1e-300
    err = np.abs(a - b).reshape(5, -1).max(axis=1) / scale
    assert np.all(err <= 1e-13), err


def test_weno3_special_cases():
    """WENO3-JS: exact on linear data (both candidates are), the smooth side's
    candidate at a jump, and third order on smooth monotone data (the weights
    approach (1/3, 2/3) to O(h))."""
    for a, b, c in ((1.0, 2.0, 3.0), (-4.0, -1.5, 1.0)):
        assert abs(oracle.weno3(a, b, c) - (b + 0.5 * (c - b))) < 1e-14
    assert abs(oracle.weno3(0.0, 1.0, 1.0) - 1.0) < 1e-6
    assert abs(oracle.weno3(0.0, 0.0, 1.0) - 0.0) < 1e-6
    errs = []
    for n in (40, 80, 160, 320):
        h = 1.0 / n
        xl = 0.3 + np.arange(n) * h * 0.5
        avg = lambda x0: (np.exp(x0 + h) - np.exp(x0)) / h
        e = max(abs(oracle.weno3(avg(x - h), avg(x), avg(x + h)) - np.exp(x + h)) for x in xl[5:-5])
        errs.append(e)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= 2.8, order


def test_tvd_rk2_second_order_in_time():
    n, t_end = 40, 0.5
    case, W = wl.entropy_wave(n)
    case["flags"] |= wl.RK2
    U0 = oracle.state_init(case, W)
    ref, _, _ = oracle.advance(case, U0, 10 ** 7, t_end=t_end, fixed_dt=0.01 / 64)
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        U, t, _ = oracle.advance(case, U0, 10 ** 7, t_end=t_end, fixed_dt=dt)
        errs.append(float(np.max(np.abs(U - ref))))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 2.0) < 0.2), order


def test_rusanov_flux_pins():
    """Rusanov (§7.4): equal states give the physical flux; alpha is the
    largest |u -+ c| of the two states; at a stationary contact (u = 0, equal
    pressures) HLLC gives the exact flux (0, p, 0, 0, 0) and Rusanov adds the
    dissipation -alpha (U_R - U_L)/2."""
    g = 1.4
    w = np.array([1.2, 0.3, -0.1, 0.2, 0.9])
    for d in range(3):
        assert np.allclose(oracle.rusanov(g, w, w, d), oracle.euler_flux(g, w, d), rtol=1e-15, atol=1e-15)
    wl_ = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
    wr_ = np.array([0.25, 0.0, 0.0, 0.0, 1.0])
    a = max(math.sqrt(g * 1.0 / 1.0), math.sqrt(g * 1.0 / 0.25))
    F = oracle.rusanov(g, wl_, wr_, 0)
    Fh = oracle.hllc(g, wl_, wr_, 0)
    assert np.allclose(Fh, [0.0, 1.0, 0.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(F, [-0.5 * a * (0.25 - 1.0), 1.0, 0.0, 0.0, 0.0], rtol=1e-14)
    assert abs(F[4] - (-0.5 * a * (1.0 / 0.4 - 1.0 / 0.4))) < 1e-14


def test_implosion_scheme_sod_and_walled_conservation():
    """The implosion's scheme (WENO3-JS + TVD-RK2, HLLC or Rusanov): Sod
    converges to the exact solution, Rusanov more diffusively than HLLC; on the
    walled implosion mass and energy are conserved to rounding (the wall
    fluxes of mirrored states carry neither)."""
    e = ExactRiemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    l1 = {}
    for flux in (0, wl.RUSANOV):
        for n in (100, 200, 400):
            case, W = wl.sod(n)
            case["flags"] |= wl.WENO3 | wl.RK2 | flux
            U, t, _ = oracle.advance(case, oracle.state_init(case, W), 100000, t_end=0.2)
            rho = oracle.interior(case, U).reshape(5, n)[0]
            l1[(flux, n)] = float(np.mean(np.abs(rho - e.cell_average_profile(n, 0.2)[0])))
        assert l1[(flux, 100)] > l1[(flux, 200)] > l1[(flux, 400)], l1
    for n in (100, 200, 400):
        assert l1[(wl.RUSANOV, n)] > l1[(0, n)], l1
    for flux in (0, wl.RUSANOV):
        case, W = wl.implosion(32, flags=wl.INVISCID | wl.WENO3 | wl.RK2 | flux)
        U0 = oracle.state_init(case, W)
        U, _, _ = oracle.advance(case, U0, 40, fixed_dt=1e-3)
        a, b = oracle.interior(case, U0), oracle.interior(case, U)
        for v in (0, 4):
            s0 = math.fsum(a[v].ravel().tolist())
            s1 = math.fsum(b[v].ravel().tolist())
            assert abs(s1 - s0) <= 1e-13 * abs(s0), (flux, v, s0, s1)
        assert np.max(np.abs(b - a)) > 1e-3  # the state has moved


def _nn_numpy(th, f):
    """The §7.4 network through numpy matrix products (a second implementation
    of the same definition: different code, same layer order)."""
    o = 0

    def take(k, shape):
        nonlocal o
        a = th[o:o + k].reshape(shape)
        o += k
        return a
    h = np.asarray(f, dtype=np.float64)
    for fan_in in (4, 32, 32):
        W = take(32 * fan_in, (32, fan_in))
        b = take(32, (32,))
        h = np.maximum(W @ h + b, 0.0)
    W4 = take(32, (32,))
    b4 = take(1, ())
    assert o == th.size
    return float(np.exp(W4 @ h + b4))


def _select_net(k):
    """Weights whose output is alpha = exp(relu(f_k)): hidden unit 0 passes input
    k through the three layers, everything else is zero."""
    th = np.zeros(wl.NN_PARAMS)
    th[0 * 4 + k] = 1.0                     # W1[0, k]
    o = 128 + 32
    th[o] = 1.0                              # W2[0, 0]
    o += 1024 + 32
    th[o] = 1.0                              # W3[0, 0]
    o += 1024 + 32
    th[o] = 1.0                              # W4[0]
    return th


def _const_net(alpha):
    th = np.zeros(wl.NN_PARAMS)
    th[-1] = math.log(alpha)
    return th


def test_nn_alpha_matches_matrix_form():
    """The network of §7.4 (4 -> 32 -> 32 -> 32 -> 1, ReLU, exp output) against
    numpy matrix products, for random weights and inputs of both signs."""
    rng = np.random.default_rng(11)
    try:
        for seed in range(4):
            th = wl.nn_weights(seed=seed, alpha0=1.3, scale=1.0)
            th[np.r_[128:160, 1184:1216, 2240:2272]] = rng.normal(0, 0.3, 96)  # nonzero biases
            oracle.set_nn(th)
            for _ in range(20):
                f = rng.normal(0, 1, 4)
                a = oracle.nn_alpha(f)
                assert a > 0.0
                assert abs(a - _nn_numpy(th, f)) <= 1e-13 * a
    finally:
        oracle.set_nn(None)


def test_rusanov_nn_flux_pins():
    """Rusanov-NN (§7.4): with a constant network (alpha = exp(b4)) it is the
    Rusanov flux of the same alpha, so a constant equal to the classical alpha
    reproduces the classical Rusanov flux; equal states give the physical flux
    for any weights; each input feature, selected alone, gives its closed form:
    |u_R - u_L|, (u_L + u_R)/2, (c_L + c_R)/2 and |s_R - s_L| with
    s = ln(p / rho^gamma)/(gamma - 1) (zero for an isentropic pair)."""
    g = 1.4
    wL = np.array([1.0, 0.3, -0.1, 0.2, 1.0])
    wR = np.array([0.5, -0.2, 0.1, 0.0, 0.4])
    try:
        for d in range(3):
            uL, uR = wL[1 + d], wR[1 + d]
            cL, cR = math.sqrt(g * wL[4] / wL[0]), math.sqrt(g * wR[4] / wR[0])
            a_cls = max(abs(uL - cL), abs(uL + cL), abs(uR - cR), abs(uR + cR))
            oracle.set_nn(_const_net(a_cls))
            np.testing.assert_allclose(oracle.rusanov_nn(g, wL, wR, d), oracle.rusanov(g, wL, wR, d),
                                       rtol=1e-14, atol=1e-15)
            oracle.set_nn(wl.nn_weights(seed=d, alpha0=2.0, scale=1.0))
            np.testing.assert_allclose(oracle.rusanov_nn(g, wL, wL, d), oracle.euler_flux(g, wL, d),
                                       rtol=1e-15, atol=1e-15)

        def alpha_of(th, a, b, d=0):
            # alpha recovered from the flux: F(alpha) = F(1) - (alpha - 1) (U_R - U_L) / 2
            oracle.set_nn(th)
            Fa = oracle.rusanov_nn(g, a, b, d)
            oracle.set_nn(_const_net(1.0))
            F1 = oracle.rusanov_nn(g, a, b, d)
            oracle.set_nn(_const_net(2.0))
            F2 = oracle.rusanov_nn(g, a, b, d)
            return 1.0 + (Fa[0] - F1[0]) / (F2[0] - F1[0])

        a = np.array([1.0, 0.3, 0.0, 0.0, 1.0])
        b = np.array([0.5, -0.2, 0.0, 0.0, 1.0])
        assert abs(alpha_of(_select_net(0), a, b) - math.exp(0.5)) < 1e-13
        assert abs(alpha_of(_select_net(1), a, b) - math.exp(0.05)) < 1e-13
        a2 = np.array([1.0, 0.0, 0.0, 0.0, 1.0 / g])      # c = 1
        b2 = np.array([0.25, 0.0, 0.0, 0.0, 1.0 / g])     # c = 2
        assert abs(alpha_of(_select_net(2), a2, b2) - math.exp(1.5)) < 1e-13
        a3 = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
        b3 = np.array([1.0 + 1e-3, 0.0, 0.0, 0.0, 2.0])   # rho nearly equal, p doubled
        ds = (math.log(2.0) - g * math.log(1.0 + 1e-3)) / (g - 1.0)
        assert abs(alpha_of(_select_net(3), a3, b3) - math.exp(ds)) < 1e-12
        b4 = np.array([2.0, 0.0, 0.0, 0.0, 2.0 ** g])     # isentropic: p / rho^gamma equal
        assert abs(alpha_of(_select_net(3), a3, b4) - 1.0) < 1e-13
        # the features do not depend on the side: swapping L and R and negating
        # the normal velocity leaves |du|, c_M and |ds| alone and negates u_M
        for k in (0, 2, 3):
            m = lambda w: w * np.array([1, -1, 1, 1, 1])
            assert abs(alpha_of(_select_net(k), a, b) - alpha_of(_select_net(k), m(b), m(a))) < 1e-13
    finally:
        oracle.set_nn(None)


def _nn_case(n=10):
    case, W = wl.implosion(n, flags=wl.INVISCID | wl.WENO3 | wl.RK2 | wl.RUSANOV_NN)
    rng = np.random.default_rng(5)
    W = W.copy()
    W[0] *= 1.0 + 0.1 * rng.random(W[0].shape)
    W[1] = 0.1 * rng.standard_normal(W[1].shape)
    W[2] = 0.1 * rng.standard_normal(W[2].shape)
    return case, W


def test_rusanov_nn_taped_gradients_match_central_differences():
    """The taped step derivative with the Rusanov-NN flux (walled implosion,
    WENO3-JS + TVD-RK2, §7.4), with respect to the state and to the network
    weights, against second-order central differences of the oracle step."""
    case, W = _nn_case()
    dt = 1e-3
    th = wl.nn_weights(seed=3, alpha0=1.5, scale=0.5)
    rng = np.random.default_rng(8)
    try:
        oracle.set_nn(th)
        U0 = oracle.state_init(case, W)
        Ub = np.zeros_like(U0)
        oracle.interior(case, Ub)[...] = rng.standard_normal(oracle.interior(case, Ub).shape)

        def L(U, t):
            oracle.set_nn(t)
            out, _ = oracle.rk3_step(case, U, dt)
            return float(np.sum(oracle.interior(case, out) * oracle.interior(case, Ub)))
        oracle.set_nn(th)
        Ubar, tbar = oracle.vjp_step_theta(case, U0, dt, Ub)
        assert np.any(tbar != 0.0)
        for trial in range(3):
            v = rng.standard_normal(th.size)
            h = 1e-6  # small enough that no ReLU unit of any face changes side
            fd = (L(U0, th + h * v) - L(U0, th - h * v)) / (2 * h)
            ad = float(tbar @ v)
            assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)), (trial, fd, ad)
        dU = np.zeros_like(U0)
        oracle.interior(case, dU)[...] = rng.standard_normal(oracle.interior(case, dU).shape)
        dU[0] *= 0.01
        # A ReLU pre-activation of some face may sit within the step of zero on
        # one side; a kink on one side spoils only that side's difference, so
        # the central, forward or backward difference must agree.
        h = 1e-8
        L0 = L(U0, th)
        Lp = L(oracle.fill_halo(case, U0 + h * dU), th)
        Lm = L(oracle.fill_halo(case, U0 - h * dU), th)
        ad = float(np.sum(oracle.interior(case, Ubar) * oracle.interior(case, dU)))
        fds = ((Lp - Lm) / (2 * h), (Lp - L0) / h, (L0 - Lm) / h)
        assert min(abs(f - ad) for f in fds) <= 1e-6 * max(1.0, abs(ad)), (fds, ad)
    finally:
        oracle.set_nn(None)


def test_rusanov_nn_rhs_weight_gradient_matches_central_differences():
    """The taped right-hand-side derivative with respect to the network weights
    (the reference the device's weight gradient is compared with) against
    central differences of <Rbar, R(U; theta)> along random weight directions
    (a one-sided difference where a ReLU unit of some face changes side)."""
    case, W = _nn_case(12)
    th = wl.nn_weights(seed=7, alpha0=1.1, scale=0.8)
    rng = np.random.default_rng(17)
    try:
        oracle.set_nn(th)
        U0 = oracle.state_init(case, W)
        Rb = np.zeros_like(U0)
        oracle.interior(case, Rb)[...] = rng.standard_normal(oracle.interior(case, Rb).shape)
        _, tbar = oracle.vjp_rhs_theta(case, U0, Rb)

        def L(t):
            oracle.set_nn(t)
            return float(np.sum(oracle.rhs(case, U0) * Rb))
        L0 = L(th)
        for trial in range(3):
            v = rng.standard_normal(th.size)
            h = 1e-7
            Lp, Lm = L(th + h * v), L(th - h * v)
            ad = float(tbar @ v)
            fds = ((Lp - Lm) / (2 * h), (Lp - L0) / h, (L0 - Lm) / h)
            assert min(abs(f - ad) for f in fds) <= 1e-6 * max(1.0, abs(ad)), (trial, fds, ad)
    finally:
        oracle.set_nn(None)


def test_rusanov_nn_needs_weights():
    case, W = _nn_case(8)
    oracle.set_nn(None)
    with pytest.raises(ValueError):
        oracle.state_init(case, W)


# ---------------------------------------------------------------- O1/O2 ----
@pytest.mark.parametrize("bc", [wl.PERIODIC, wl.ZERO_GRADIENT])
def test_halo_fill_matches_independent_padding(bc):
    case = wl.make_case((7, 5, 4), bc=(bc,) * 6)
    rng = np.random.default_rng(3)
    inner = rng.standard_normal((5, 4, 5, 7))
    U = np.zeros(oracle.padded_shape(case))
    oracle.interior(case, U)[...] = inner
    got = oracle.fill_halo(case, U)
    mode = "wrap" if bc == wl.PERIODIC else "edge"
    want = np.pad(inner, ((0, 0), (3, 3), (3, 3), (3, 3)), mode=mode)
    assert np.array_equal(got, want)


def test_state_init_and_dt_hand_values():
    case = wl.make_case((4, 1, 1), gamma=1.4, cfl=0.5, bc=(wl.PERIODIC,) * 6)
    W = np.zeros((5, 1, 1, 4))
    W[0], W[1], W[2], W[3], W[4] = 2.0, 1.0, 2.0, 3.0, 3.0
    U = oracle.state_init(case, W)
    Ui = oracle.interior(case, U)
    # E = p/(gamma-1) + rho |u|^2 / 2 = 7.5 + 14
    np.testing.assert_array_equal(Ui[:, 0, 0, 0], [2.0, 2.0, 4.0, 6.0, 21.5])
    # dt = CFL / ((|u| + c)/dx) on the single active axis
    c = math.sqrt(1.4 * 3.0 / 2.0)
    assert abs(oracle.cfl_dt(case, U) - 0.5 / ((1.0 + c) / 0.25)) < 1e-15
    assert abs(oracle.cfl_dt(case, U, t=0.1, t_end=0.1001) - 1e-4) < 1e-15


# ---------------------------------------------------------------- P9 -------
def _dot_test(fun, vjp, U, rng, h=1e-7):
    v = rng.standard_normal(U.shape)
    w = rng.standard_normal(U.shape)
    fd = (fun(U + h * v) - fun(U - h * v)) / (2 * h)
    lhs = float(np.sum(w * fd))
    rhs_ = float(np.sum(vjp(U, w) * v))
    return lhs, rhs_


@pytest.mark.parametrize("kind", ["smooth", "shocky"])
def test_taped_rhs_derivative_matches_finite_differences(kind):
    rng = np.random.default_rng(5)
    if kind == "smooth":
        case, W = wl.random_smooth((6, 5, 4), seed=1, mu=0.05)
    else:
        case, W = wl.random_shocky((8, 5, 1), seed=2)
    U = oracle.state_init(case, W)
    mask = np.zeros_like(U)
    oracle.interior(case, mask)[...] = 1.0
    fun = lambda X: oracle.rhs(case, X * mask + U * (1 - mask))
    vjp = lambda X, w: oracle.vjp_rhs(case, X, w * mask) * mask
    # central differences with h = 1e-7: truncation error ~1e-7 relative on
    # these data (it falls as h^2, checked at h = 1e-4 .. 1e-7)
    lhs, r = _dot_test(fun, lambda X, w: vjp(X, w), U, rng)
    assert abs(lhs - r) <= 3e-6 * max(abs(lhs), abs(r)), (lhs, r)


@pytest.mark.parametrize("bc", [wl.PERIODIC, wl.ZERO_GRADIENT, wl.REFLECT])
def test_taped_state_init_derivative_matches_finite_differences(bc):
    """The taped reverse mode of state_init (primitive point values to the
    padded conservative state with its halos, §2, §3.7): <w, J v> by central
    differences against <J^T w, v>; the map is at most cubic in W, so the
    differences are exact to rounding. A cotangent on the halo cells reaches
    their interior sources."""
    flags = wl.INVISCID
    case = wl.make_case((5, 4, 3), bc=(bc,) * 4 + (wl.PERIODIC,) * 2, flags=flags)
    rng = np.random.default_rng(33)
    W = np.stack([rng.uniform(0.5, 2, (3, 4, 5)), *rng.uniform(-1, 1, (3, 3, 4, 5)),
                  rng.uniform(0.5, 2, (3, 4, 5))])
    v = rng.standard_normal(W.shape)
    w = rng.standard_normal(oracle.padded_shape(case))
    h = 1e-5
    fd = (oracle.state_init(case, W + h * v) - oracle.state_init(case, W - h * v)) / (2 * h)
    lhs = float(np.sum(w * fd))
    rhs_ = float(np.sum(oracle.vjp_state_init(case, W, w) * v))
    assert abs(lhs - rhs_) <= 1e-9 * abs(lhs), (lhs, rhs_)
    # a halo-only cotangent gives a nonzero gradient on the cells it mirrors
    wh = w.copy()
    oracle.interior(case, wh)[...] = 0.0
    assert np.max(np.abs(oracle.vjp_state_init(case, W, wh))) > 0.1


def test_taped_step_and_loss_gradient_match_finite_differences():
    case, W = wl.taylor_green_noisy(6, sigma=1e-3, seed=4)
    U = oracle.state_init(case, W)
    dt = 0.5 * oracle.cfl_dt(case, U)
    rng = np.random.default_rng(6)
    mask = np.zeros_like(U)
    oracle.interior(case, mask)[...] = 1.0
    fun = lambda X: oracle.rk3_step(case, X, dt)[0] * mask
    vjp = lambda X, w: oracle.vjp_rk3_step(case, X, dt, w * mask) * mask
    lhs, r = _dot_test(fun, vjp, U, rng)
    assert abs(lhs - r) <= 3e-6 * max(abs(lhs), abs(r)), (lhs, r)

    nsteps = 3
    L, g = oracle.grad_kinetic_energy(case, W, nsteps, dt)
    dV = (2 * np.pi / 6) ** 3

    def loss(Wx):
        Ux, _, _ = oracle.advance(case, oracle.state_init(case, Wx), nsteps, fixed_dt=dt)
        Ui = oracle.interior(case, Ux)
        return float(np.sum(0.5 * (Ui[1] ** 2 + Ui[2] ** 2 + Ui[3] ** 2) / Ui[0]) * dV)

    assert abs(loss(W) - L) <= 1e-13 * abs(L)
    h = 1e-7
    d = rng.standard_normal((3,) + W.shape[1:])
    Wp, Wm = W.copy(), W.copy()
    Wp[1:4] += h * d
    Wm[1:4] -= h * d
    fd = (loss(Wp) - loss(Wm)) / (2 * h)
    ad = float(np.sum(g * d))
    assert abs(fd - ad) <= 3e-6 * abs(ad), (fd, ad)
