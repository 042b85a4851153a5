"""Term-by-term pins of the CPU oracle (no GPU).

Each test fixes one part of the oracle's arithmetic against something other
than the oracle's own formula: an integral definition evaluated by quadrature,
an algebraic identity between two independently pinned quantities, an exact
flux of a smooth field, an invariance of the equations, or a hand value.

  WENO5-JS, WENO5-Z and WENO3-JS: smoothness indicators, candidates and
      linear weights from their integral and polynomial definitions (Jiang &
      Shu 1996, Borges et al. 2008; §3.3, §7.4)
  Einfeldt signal speeds against the Roe average of the pinned Roe
      decomposition (§3.3, Appendix A "EINFELDT")
  compressive viscous stress and work term against exact face fluxes (§2, §3.4)
  the cross derivatives (DC4 then RC4) against the exact face fluxes of a 3D
      field with unequal cell sizes, at fourth order (§3.4)
  the primitive map's tangential kinetic energy: a shock tube with constant
      tangential velocities evolves rho, u, p exactly as without them (§2)
  the CFL step in 3D with unequal cells, and where the viscous bound binds (§3.2)
"""
import math

import numpy as np
import pytest

import oracle
from paper_2203_13760_amd import workloads as wl


# ------------------------------------------------------------ WENO5-JS -----
def _cell_avg_rows(cells):
    # cell average over [m - 1/2, m + 1/2] of 1, x, x^2 (unit cells)
    return np.array([[1.0, m, m * m + 1.0 / 12.0] for m in cells])


def _quad_fit(cells, avgs):
    """Coefficients (c0, c1, c2) of the quadratic whose cell averages over the
    given unit cells equal avgs."""
    return np.linalg.solve(_cell_avg_rows(cells), np.asarray(avgs, dtype=float))


def _beta_integral(coef):
    """Jiang & Shu's smoothness indicator of a candidate polynomial on the centre
    cell [-1/2, 1/2] (unit width): sum over l = 1, 2 of dx^(2l-1) times the
    integral of the squared l-th derivative, by Gauss-Legendre quadrature."""
    xg, wg = np.polynomial.legendre.leggauss(4)
    x, w = 0.5 * xg, 0.5 * wg
    d1 = coef[1] + 2.0 * coef[2] * x
    d2 = 2.0 * coef[2] * np.ones_like(x)
    return float(np.sum(w * d1 * d1) + np.sum(w * d2 * d2))


def _linear_weights():
    """d_k with sum_k d_k p_k(1/2) = P(1/2) for every data set, P the quartic
    with the five cell averages: solved on the five unit data sets."""
    A, b = [], []
    for e in np.eye(5):
        P = np.linalg.solve(np.array([[((m + 0.5) ** (j + 1) - (m - 0.5) ** (j + 1)) / (j + 1)
                                       for j in range(5)] for m in (-2, -1, 0, 1, 2)]), e)
        A.append([np.polyval(_quad_fit(c, e[k:k + 3])[::-1], 0.5) for k, c in
                  enumerate(((-2, -1, 0), (-1, 0, 1), (0, 1, 2)))])
        b.append(np.polyval(P[::-1], 0.5))
    d, res, _, _ = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)
    assert np.max(np.abs(np.array(A) @ d - np.array(b))) < 1e-13
    return d


def _weno5_from_definitions(s, eps=1.0e-6):
    d = _linear_weights()
    cand, beta = [], []
    for k, cells in enumerate(((-2, -1, 0), (-1, 0, 1), (0, 1, 2))):
        coef = _quad_fit(cells, s[k:k + 3])
        cand.append(coef[0] + 0.5 * coef[1] + 0.25 * coef[2])
        beta.append(_beta_integral(coef))
    alpha = d / (eps + np.array(beta)) ** 2
    return float(np.dot(alpha, cand) / np.sum(alpha)), d, beta


def test_weno5_js_from_integral_smoothness_indicators():
    """WENO5-JS (Jiang & Shu 1996; §3.3 names it, R3 reads eps = 1e-6 and the
    power 2): candidates from quadratic fits to cell averages, smoothness
    indicators from their integral definition, linear weights from the
    quartic fit; the oracle's value agrees on non-smooth stencils of every
    scale, down to scales where eps decides the weights."""
    _, d, _ = _weno5_from_definitions(np.zeros(5))
    np.testing.assert_allclose(d, [0.1, 0.6, 0.3], rtol=0, atol=1e-14)
    rng = np.random.default_rng(21)
    worst = 0.0
    for t in range(400):
        scale = 10.0 ** rng.uniform(-4, 2)
        s = rng.standard_normal(5) * scale
        if t % 4 == 1:  # a jump somewhere in the stencil
            s[rng.integers(1, 5):] += rng.choice([-1, 1]) * scale * rng.uniform(2, 10)
        want, _, _ = _weno5_from_definitions(s)
        got = oracle.weno5(*s)
        worst = max(worst, abs(got - want) / np.max(np.abs(s)))
    assert worst < 1e-12, worst


def _weno5z_from_definitions(s, eps=1.0e-40):
    d = _linear_weights()
    cand, beta = [], []
    for k, cells in enumerate(((-2, -1, 0), (-1, 0, 1), (0, 1, 2))):
        coef = _quad_fit(cells, s[k:k + 3])
        cand.append(coef[0] + 0.5 * coef[1] + 0.25 * coef[2])
        beta.append(_beta_integral(coef))
    tau5 = abs(beta[0] - beta[2])
    alpha = d * (1.0 + tau5 / (np.array(beta) + eps))
    return float(np.dot(alpha, cand) / np.sum(alpha))


def test_weno5_z_from_integral_smoothness_indicators():
    """WENO5-Z (Borges et al. 2008; R25): the same candidates, indicators and
    linear weights as WENO5-JS, the global indicator tau5 = |beta_0 - beta_2|
    and alpha_k = d_k (1 + tau5 / (beta_k + 1e-40))."""
    rng = np.random.default_rng(24)
    worst = 0.0
    for t in range(400):
        scale = 10.0 ** rng.uniform(-4, 2)
        s = rng.standard_normal(5) * scale
        if t % 4 == 1:
            s[rng.integers(1, 5):] += rng.choice([-1, 1]) * scale * rng.uniform(2, 10)
        worst = max(worst, abs(oracle.weno5z(*s) - _weno5z_from_definitions(s)) / np.max(np.abs(s)))
    assert worst < 1e-12, worst


def test_weno3_js_from_integral_smoothness_indicators():
    """WENO3-JS (Jiang & Shu 1996 with r = 2; R29): linear candidates through the
    cell averages of (i-1, i) and (i, i+1) evaluated at the face, indicators
    dx * integral of the squared first derivative, linear weights (1/3, 2/3)
    from the quadratic through all three averages, eps = 1e-6, power 2."""
    def lin_fit(cells, avgs):  # c0 + c1 x with the given cell averages
        return np.linalg.solve(np.array([[1.0, m] for m in cells]), np.asarray(avgs, dtype=float))

    A, b = [], []
    for e in np.eye(3):
        q = _quad_fit((-1, 0, 1), e)
        A.append([lin_fit((-1, 0), e[0:2]) @ [1, 0.5], lin_fit((0, 1), e[1:3]) @ [1, 0.5]])
        b.append(q[0] + 0.5 * q[1] + 0.25 * q[2])
    d = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
    np.testing.assert_allclose(d, [1.0 / 3.0, 2.0 / 3.0], rtol=0, atol=1e-14)
    rng = np.random.default_rng(25)
    worst = 0.0
    for t in range(300):
        scale = 10.0 ** rng.uniform(-4, 2)
        s = rng.standard_normal(3) * scale
        cand, beta = [], []
        for k, cells in enumerate(((-1, 0), (0, 1))):
            c = lin_fit(cells, s[k:k + 2])
            cand.append(c[0] + 0.5 * c[1])
            beta.append(c[1] ** 2)  # integral over the unit cell of (p')^2
        alpha = d / (1e-6 + np.array(beta)) ** 2
        want = float(np.dot(alpha, cand) / np.sum(alpha))
        worst = max(worst, abs(oracle.weno3(*s) - want) / np.max(np.abs(s)))
    assert worst < 1e-12, worst


def test_weno5_js_candidate_weights_differ_from_linear_at_a_kink():
    """At a kink the three indicators differ by orders of magnitude, so the
    result depends on them (guards the test above against stencils on which
    any indicator gives the same answer)."""
    s = np.array([0.0, 0.0, 0.0, 1.0, 2.0])
    want, _, beta = _weno5_from_definitions(s)
    lin = (2 * s[0] - 13 * s[1] + 47 * s[2] + 27 * s[3] - 3 * s[4]) / 60
    assert beta[0] < 1e-12 < 0.1 < beta[1]
    assert abs(want - lin) > 1e-2
    assert abs(oracle.weno5(*s) - want) < 1e-13


# ------------------------------------------------------------ Einfeldt -----
def test_einfeldt_speeds_against_roe_average():
    """Einfeldt's bound (R5): with tangential velocities equal on both sides,
    dbar^2 exceeds the Roe-averaged sound speed squared by
    (2 - gamma)/2 r_L r_R (u_R - u_L)^2 / (r_L + r_R)^2 (r = sqrt(rho)), and
    ubar is the Roe-averaged normal velocity; the Roe average comes from the
    Roe decomposition, pinned by A (U_R - U_L) = F(U_R) - F(U_L). S_L and S_R
    take the min/max against u_L - c_L and u_R + c_R."""
    rng = np.random.default_rng(22)
    for t in range(120):
        g = [1.4, 1.67, 2.0, 1.1][t % 4]
        d = t % 3
        wl_ = np.array([rng.uniform(0.1, 5), *rng.uniform(-3, 3, 3), rng.uniform(0.05, 5)])
        wr_ = np.array([rng.uniform(0.1, 5), *rng.uniform(-3, 3, 3), rng.uniform(0.05, 5)])
        for a in range(3):
            if a != d:
                wr_[1 + a] = wl_[1 + a]
        ubar, dbar, SL, SR = oracle.einfeldt(g, wl_, wr_, d)
        _, _, lam = oracle.roe_eigen(g, wl_, wr_, d)
        u_roe, a_roe = lam[1], 0.5 * (lam[4] - lam[0])
        rl, rr = math.sqrt(wl_[0]), math.sqrt(wr_[0])
        jump = 0.5 * (2.0 - g) * rl * rr * (wr_[1 + d] - wl_[1 + d]) ** 2 / (rl + rr) ** 2
        assert abs(ubar - u_roe) <= 1e-13 * max(1.0, abs(u_roe)), t
        assert abs(dbar ** 2 - (a_roe ** 2 + jump)) <= 1e-12 * dbar ** 2, (t, dbar ** 2, a_roe ** 2 + jump)
        if g == 2.0:
            assert abs(dbar - a_roe) <= 1e-13 * a_roe
        cl, cr = math.sqrt(g * wl_[4] / wl_[0]), math.sqrt(g * wr_[4] / wr_[0])
        assert SL == min(wl_[1 + d] - cl, ubar - dbar) or abs(SL - min(wl_[1 + d] - cl, ubar - dbar)) < 1e-14
        assert SR == max(wr_[1 + d] + cr, ubar + dbar) or abs(SR - max(wr_[1 + d] + cr, ubar + dbar)) < 1e-14
    # each bound binds in its regime: the states' own speeds for a strong
    # expansion, Einfeldt's Roe-averaged speeds for a strong compression
    ubar, dbar, SL, SR = oracle.einfeldt(1.4, np.array([1.0, -2.0, 0, 0, 1.0]), np.array([1.0, 2.0, 0, 0, 1.0]), 0)
    assert SL == -2.0 - math.sqrt(1.4) and SR == 2.0 + math.sqrt(1.4)
    ubar, dbar, SL, SR = oracle.einfeldt(1.4, np.array([1.0, 2.0, 0, 0, 1.0]), np.array([1.0, -2.0, 0, 0, 1.0]), 0)
    assert SL == ubar - dbar and SR == ubar + dbar


def test_hllc_uses_the_einfeldt_speeds():
    """The HLLC flux in the single-wave-region cases depends only on S_L or S_R
    through the star state: for a left-facing subsonic fan (S_L < 0 <= S*) the
    mass flux is F_L + S_L (U*_L - U_L) with U*_L[0] = rho_L (S_L - u_L)/(S_L - S*)
    (Toro's star state, R6); recompute it from the exposed speeds."""
    rng = np.random.default_rng(23)
    checked = 0
    for t in range(200):
        g = 1.4
        wl_ = np.array([rng.uniform(0.2, 3), *rng.uniform(-0.5, 0.5, 3), rng.uniform(0.2, 3)])
        wr_ = np.array([rng.uniform(0.2, 3), *rng.uniform(-0.5, 0.5, 3), rng.uniform(0.2, 3)])
        _, _, SL, SR = oracle.einfeldt(g, wl_, wr_, 0)
        rl, ul, pl = wl_[0], wl_[1], wl_[4]
        rr, ur, pr = wr_[0], wr_[1], wr_[4]
        Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))
        F = oracle.hllc(g, wl_, wr_, 0)
        if SL < 0 <= Ss:
            want = rl * ul + SL * (rl * (SL - ul) / (SL - Ss) - rl)
        elif Ss < 0 < SR:
            want = rr * ur + SR * (rr * (SR - ur) / (SR - Ss) - rr)
        else:
            continue
        checked += 1
        assert abs(F[0] - want) <= 1e-12 * max(1.0, abs(want)), t
    assert checked > 150


# ------------------------------------------------------------ viscous ------
def test_compressive_viscous_wave_stress_and_work():
    """1D velocity wave u = A sin 2 pi x with rho = p = 1, viscous flux only:
    tau_xx = mu (2 u' - 2/3 u') = 4/3 mu u' and the energy flux is the work
    u tau_xx (§2, Stokes hypothesis; §3.4 face values). The momentum and
    energy right-hand sides equal the face differences of the exact fluxes at
    fourth order (which also fixes the fourth-order face velocity)."""
    mu, A = 0.1, 0.3
    errs_m, errs_e = [], []
    for n in (16, 32, 64):
        case = wl.make_case((n, 1, 1), mu=mu, flags=wl.VISCOUS)
        x = wl.cell_centres(case, 0)
        W = np.zeros((5, 1, 1, n))
        W[0] = 1.0
        W[1] = A * np.sin(2 * np.pi * x)
        W[4] = 1.0
        R = oracle.interior(case, oracle.rhs(case, oracle.state_init(case, W))).reshape(5, n)
        dx = 1.0 / n
        u = lambda s: A * np.sin(2 * np.pi * s)
        du = lambda s: 2 * np.pi * A * np.cos(2 * np.pi * s)
        tau = lambda s: 4.0 / 3.0 * mu * du(s)
        work = lambda s: u(s) * tau(s)
        em = np.max(np.abs(R[1] - (tau(x + dx / 2) - tau(x - dx / 2)) / dx))
        ee = np.max(np.abs(R[4] - (work(x + dx / 2) - work(x - dx / 2)) / dx))
        errs_m.append(em)
        errs_e.append(ee)
        assert np.all(R[0] == 0.0) and np.all(R[2] == 0.0) and np.all(R[3] == 0.0)
    for errs in (errs_m, errs_e):
        order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(order > 3.8), (errs, order)
    assert errs_m[-1] < 1e-5 and errs_e[-1] < 1e-5


def _field(X, Y, Z):
    """A smooth periodic compressive 3D velocity on the box (1, 2, 1.5): each
    component A_a sin(k_a . x + phi_a) with wave vectors mixing all axes."""
    L = np.array([1.0, 2.0, 1.5])
    m = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 1]], dtype=float)
    k = 2 * np.pi * m / L
    A = np.array([0.3, -0.2, 0.25])
    ph = np.array([0.1, 0.7, -0.4])
    arg = [k[a, 0] * X + k[a, 1] * Y + k[a, 2] * Z + ph[a] for a in range(3)]
    u = [A[a] * np.sin(arg[a]) for a in range(3)]
    grad = [[A[a] * k[a, b] * np.cos(arg[a]) for b in range(3)] for a in range(3)]
    return u, grad


def _exact_face_flux(mu, d, X, Y, Z):
    u, grad = _field(X, Y, Z)
    div = grad[0][0] + grad[1][1] + grad[2][2]
    tau = [mu * (grad[d][b] + grad[b][d]) - (2.0 / 3.0 * mu * div if b == d else 0.0) for b in range(3)]
    return tau + [u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2]]


def test_viscous_flux_of_a_3d_field_fourth_order():
    """3D compressive velocity field with all nine gradient entries nonzero,
    uniform rho and p, unequal cell sizes per axis, viscous flux only: the
    momentum and energy right-hand sides equal the face differences of the
    exact face fluxes (tau_d and u . tau_d, §2) at fourth order. This pins
    the fourth-order centred tangential derivatives (DC4) interpolated to the
    face (RC4) with each axis's own cell size, the normal derivative (DF4),
    the -2/3 mu div u term with its tangential parts, and the work term."""
    mu = 0.05
    errs = []
    for n in (12, 24, 48):
        case = wl.make_case((n, n, n), hi=(1.0, 2.0, 1.5), mu=mu, flags=wl.VISCOUS)
        X, Y, Z = wl._mesh(case)
        u, _ = _field(X, Y, Z)
        W = np.stack([np.ones_like(X), u[0], u[1], u[2], np.ones_like(X)])
        R = oracle.interior(case, oracle.rhs(case, oracle.state_init(case, W)))
        dx = [(case["hi"][a] - case["lo"][a]) / n for a in range(3)]
        exact = np.zeros((4,) + X.shape)
        for d in range(3):
            off = [np.zeros(1)] * 3
            sh = [0.0, 0.0, 0.0]
            sh[d] = dx[d] / 2
            Fp = _exact_face_flux(mu, d, X + sh[0], Y + sh[1], Z + sh[2])
            Fm = _exact_face_flux(mu, d, X - sh[0], Y - sh[1], Z - sh[2])
            for v in range(4):
                exact[v] += (Fp[v] - Fm[v]) / dx[d]
        err = max(float(np.max(np.abs(R[1 + v] - exact[v]))) for v in range(4))
        errs.append(err)
        assert np.all(R[0] == 0.0)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 3.8), (errs, order)


# ------------------------------------------------------ primitive map ------
def test_tangential_velocity_is_passive_in_a_shock_tube():
    """Sod's tube (§5.1.2) with constant tangential velocities (v, w) =
    (0.3, -0.7): the x-split Euler equations carry them passively, so rho, u
    and p evolve exactly as with (v, w) = (0, 0) (to rounding). The pressure
    of the primitive map must subtract the whole kinetic energy (§2)."""
    case, W0 = wl.sod(100)
    W1 = W0.copy()
    W1[2] = 0.3
    W1[3] = -0.7
    out = []
    for W in (W0, W1):
        U = oracle.state_init(case, W)
        U, t, steps = oracle.advance(case, U, 100000, t_end=case["t_end"])
        Ui = oracle.interior(case, U).reshape(5, -1)
        rho = Ui[0]
        u = Ui[1] / rho
        p = 0.4 * (Ui[4] - 0.5 * (Ui[1] ** 2 + Ui[2] ** 2 + Ui[3] ** 2) / rho)
        out.append((rho, u, p, steps, Ui[2] / rho, Ui[3] / rho))
    (r0, u0, p0, s0, _, _), (r1, u1, p1, s1, v1, w1) = out
    assert s0 == s1
    for a, b in ((r0, r1), (u0, u1), (p0, p1)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a)), np.max(np.abs(a - b))
    assert np.max(np.abs(v1 - 0.3)) < 1e-12 and np.max(np.abs(w1 + 0.7)) < 1e-12


# ------------------------------------------------------------ CFL step -----
def test_cfl_step_3d_hand_values():
    """dt = CFL / max over cells of max(sum_d (|u_d| + c)/dx_d,
    2 (mu/rho) max(4/3, gamma/Pr) sum_d dx_d^-2) (R1), on a 4 x 5 x 6 grid of
    the box (1, 2, 3): dx = (0.25, 0.4, 0.5)."""
    def run(W, mu, pr, flags):
        case = wl.make_case((4, 5, 6), hi=(1.0, 2.0, 3.0), mu=mu, prandtl=pr, cfl=0.5, flags=flags)
        return oracle.cfl_dt(case, oracle.state_init(case, W))

    W = np.empty((5, 6, 5, 4))
    for v, val in enumerate((2.0, 1.0, -2.0, 0.5, 3.0)):
        W[v] = val
    c = math.sqrt(1.4 * 3.0 / 2.0)
    s = (1.0 + c) / 0.25 + (2.0 + c) / 0.4 + (0.5 + c) / 0.5
    assert abs(run(W, 0.0, 0.72, wl.INVISCID) - 0.5 / s) <= 1e-15
    # one faster cell decides the maximum
    W2 = W.copy()
    W2[3, 4, 2, 1] = -3.0
    s2 = (1.0 + c) / 0.25 + (2.0 + c) / 0.4 + (3.0 + c) / 0.5
    assert abs(run(W2, 0.0, 0.72, wl.INVISCID) - 0.5 / s2) <= 1e-15
    # viscous bound binding: mu = 5, rho = 2, sum dx^-2 = 16 + 6.25 + 4
    inv2 = 16.0 + 6.25 + 4.0
    sv = 2.0 * (5.0 / 2.0) * (1.4 / 0.72) * inv2
    assert sv > s
    assert abs(run(W, 5.0, 0.72, wl.ALL_PHYSICS) - 0.5 / sv) <= 1e-15
    # with Pr = 2 the factor 4/3 binds instead of gamma/Pr = 0.7
    sv43 = 2.0 * (5.0 / 2.0) * (4.0 / 3.0) * inv2
    assert abs(run(W, 5.0, 2.0, wl.VISCOUS) - 0.5 / sv43) <= 1e-15
    # the viscous bound follows the densest-weighted cell: mu/rho largest where rho is smallest
    W3 = W.copy()
    W3[0, 1, 1, 1] = 0.5
    sv3 = 2.0 * (5.0 / 0.5) * (1.4 / 0.72) * inv2
    assert abs(run(W3, 5.0, 0.72, wl.HEAT | wl.INVISCID) - 0.5 / sv3) <= 1e-15
    # below the crossover the convective rate decides
    assert abs(run(W, 0.01, 0.72, wl.ALL_PHYSICS) - 0.5 / s) <= 1e-15


# ------------------------------------------------------ safe reconstruction -
def _pocket_case(flags):
    """1D periodic pressure pocket: p = 3 with two cells at 0.1, rho = 1,
    u = 0.2. WENO5-JS across the pocket reconstructs a negative pressure
    (the stencil (3, 3, 0.1, 0.1, 3) gives about -0.42 at the right face of
    its centre cell)."""
    n = 16
    case = wl.make_case((n, 1, 1), flags=flags)
    W = np.zeros((5, 1, 1, n))
    W[0] = 1.0
    W[1] = 0.2
    W[4] = 3.0
    W[4, 0, 0, 6:8] = 0.1
    return case, W


def test_safe_reconstruction_first_order_at_flagged_faces():
    """Reading of Appendix A's is_safe_reconstruction (flag 512): at a face
    whose WENO5-JS states have rho <= 0 or p <= 0, both states fall back to
    the two adjacent cell values; the health word's bit 3 records such faces
    with or without the flag. The right-hand side is rebuilt here face by
    face from the pinned WENO5-JS value and HLLC flux."""
    case, W = _pocket_case(wl.INVISCID | 512)
    n, g = case["n"][0], case["gamma"]
    dx = 1.0 / n
    U = oracle.state_init(case, W)
    oracle.status()
    R = oracle.interior(case, oracle.rhs(case, U)).reshape(5, n)
    assert oracle.status() & 8
    q = W.reshape(5, n)
    F = np.zeros((n, 5))  # F[i]: flux at the face between cells i and i+1 (periodic)
    flagged = 0
    for i in range(n):
        st = [q[:, (i + o) % n] for o in (-2, -1, 0, 1, 2, 3)]
        WL = np.array([oracle.weno5(*[s[v] for s in st[0:5]]) for v in range(5)])
        WR = np.array([oracle.weno5(*[s[v] for s in st[5:0:-1]]) for v in range(5)])
        if min(WL[0], WL[4], WR[0], WR[4]) <= 0.0:
            WL, WR = st[2].copy(), st[3].copy()
            flagged += 1
        F[i] = oracle.hllc(g, WL, WR, 0)
    assert flagged >= 1
    want = -(F - np.roll(F, 1, axis=0)).T / dx
    np.testing.assert_allclose(R, want, rtol=0, atol=1e-12 * np.max(np.abs(want)))
    # without the flag the flagged faces keep their non-physical states: the
    # health word still reports them and the result differs there
    case0, _ = _pocket_case(wl.INVISCID)
    oracle.status()
    R0 = oracle.interior(case0, oracle.rhs(case0, oracle.state_init(case0, W))).reshape(5, n)
    assert oracle.status() & 8
    assert np.max(np.abs(R0 - R)) > 1e-3


def test_health_word_of_stage_states():
    """Bits 0-2 of the health word cover every state of a step (input, stages,
    output): a state with a negative pressure in one cell is reported by the
    step that starts from it, and a clean run reports nothing."""
    case, W = wl.sod(50)
    oracle.status()
    oracle.rk3_step(case, oracle.state_init(case, W))
    assert oracle.status() == 0
    W2 = W.copy()
    W2[4, 0, 0, 10] = -0.5
    oracle.rk3_step(case, oracle.state_init(case, W2))
    assert oracle.status() & 4
