"""The Rusanov-NN flux of §7.4 on the HIP path (WENO3-JS, TVD-RK2, reflecting
walls) against the oracle: the right-hand side, one step and 100 steps of the
forward path, and the discrete adjoint with respect to the state and to the
network weights against the oracle's taped reverse mode.

Tolerances as for the other schemes: the right-hand side to 1e-12 normwise or
the rounding bound of its flux differences, one step to 1e-12, 100 steps to
1e-10; adjoints (state and weights) to 1e-10 normwise.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2203_13760_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NN_FLAGS = wl.INVISCID | wl.WENO3 | wl.RK2 | wl.RUSANOV_NN


def normwise(a, b):
    err = 0.0
    for v in range(a.shape[0]):
        den = float(np.max(np.abs(b[v])))
        num = float(np.max(np.abs(a[v] - b[v])))
        if num == 0.0:
            continue
        err = max(err, num / den if den > 0 else math.inf)
    return err


def vecwise(a, b):
    den = float(np.max(np.abs(b)))
    num = float(np.max(np.abs(a - b)))
    return 0.0 if num == 0.0 else (num / den if den > 0 else math.inf)


@pytest.fixture(scope="module")
def Solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_13760_amd.solver import Solver as S
    return S


@pytest.fixture(autouse=True)
def _clear_oracle_weights():
    yield
    oracle.set_nn(None)


def _say(msg):
    print(msg, flush=True)


def _perturbed(n, seed=5):
    """The implosion with a density perturbation and random velocities, so that
    every feature of the network varies from face to face."""
    case, W = wl.implosion(n, flags=NN_FLAGS)
    rng = np.random.default_rng(seed)
    W = W.copy()
    W[0] *= 1.0 + 0.1 * rng.random(W[0].shape)
    W[1] = 0.1 * rng.standard_normal(W[1].shape)
    W[2] = 0.1 * rng.standard_normal(W[2].shape)
    return case, W


THETAS = {
    "near_const": wl.nn_weights(seed=3, alpha0=1.5, scale=0.5),
    "wide": wl.nn_weights(seed=4, alpha0=0.8, scale=1.0),
}

CASES = {
    "implosion24": wl.implosion(24, flags=NN_FLAGS),
    "perturbed20x20": _perturbed(20),
    "perturbed_x_only": (lambda c: (dict(c[0], n=(37, 1, 1), bc=(wl.REFLECT,) * 2 + (wl.PERIODIC,) * 4),
                                    np.ascontiguousarray(c[1][:, :, :1, :])))(_perturbed(37)),
}


def _solver(Solver, case, theta, with_bar=False):
    s = Solver(case)
    th = torch.from_numpy(theta).cuda()
    tb = torch.zeros_like(th) if with_bar else None
    s.set_nn_weights(th, tb)
    oracle.set_nn(theta)
    return s, th, tb


@pytest.mark.parametrize("tname", sorted(THETAS))
@pytest.mark.parametrize("name", sorted(CASES))
def test_nn_rhs_and_step_match_oracle(Solver, name, tname):
    case, W = CASES[name]
    _say(f"Rusanov-NN rhs + step parity: {name} / {tname}")
    s, th, _ = _solver(Solver, case, THETAS[tname])
    U = s.init(W)
    R = s.rhs(U).cpu().numpy()
    Uo = oracle.state_init(case, W)
    Ro = oracle.rhs(case, Uo)
    bound = oracle.rhs_rounding_bound(case, Uo)
    for v in range(5):
        err = float(np.max(np.abs(R[v] - Ro[v])))
        assert err <= max(1e-12 * float(np.max(np.abs(Ro[v]))), bound[v]), (name, v, err, bound[v])
    s.step(U, 1e-3)
    Uo1, _ = oracle.rk3_step(case, Uo, 1e-3)
    e = normwise(U.cpu().numpy(), Uo1)
    s.close()
    assert e <= 1e-12, (name, tname, e)


@pytest.mark.parametrize("name", ["implosion24", "perturbed20x20"])
def test_nn_100_fixed_steps_match_oracle(Solver, name):
    """100 fixed steps of the coarse step 1e-3 of §7.4 (graph-replayed)."""
    case, W = CASES[name]
    _say(f"Rusanov-NN 100-step parity: {name}")
    s, th, _ = _solver(Solver, case, THETAS["wide"])
    U = s.init(W)
    s.advance_fixed(U, 100, 1e-3)
    Uo, _, _ = oracle.advance(case, oracle.state_init(case, W), 100, fixed_dt=1e-3)
    e = normwise(U.cpu().numpy(), Uo)
    s.close()
    assert e <= 1e-10, (name, e)


def _interior_noise(case, shape, seed):
    rng = np.random.default_rng(seed)
    m = np.zeros(shape)
    oracle.interior(case, m)[...] = rng.standard_normal(oracle.interior(case, m).shape)
    return m


@pytest.mark.parametrize("tname", sorted(THETAS))
@pytest.mark.parametrize("name", ["perturbed20x20", "perturbed_x_only", "implosion24"])
def test_nn_rhs_adjoint_matches_oracle_tape(Solver, name, tname):
    case, W = CASES[name]
    _say(f"Rusanov-NN rhs adjoint parity: {name} / {tname}")
    if name == "implosion24":
        # after 30 steps the shock has reached the corner walls
        oracle.set_nn(THETAS[tname])
        W0 = W
        U0, _, _ = oracle.advance(case, oracle.state_init(case, W0), 30, fixed_dt=1e-3)
    s, th, tb = _solver(Solver, case, THETAS[tname], with_bar=True)
    U = s.init(W)
    if name == "implosion24":
        s.advance_fixed(U, 30, 1e-3)
        Uo = U0
    else:
        Uo = oracle.state_init(case, W)
    Rb = _interior_noise(case, Uo.shape, 7)
    want_u, want_t = oracle.vjp_rhs_theta(case, Uo, Rb)
    got_u = s.rhs_adjoint(U, torch.from_numpy(Rb).cuda()).cpu().numpy()
    got_t = tb.cpu().numpy()
    s.close()
    assert normwise(got_u, want_u) <= 1e-10, (name, tname, normwise(got_u, want_u))
    assert np.any(want_t != 0.0)
    assert vecwise(got_t, want_t) <= 1e-10, (name, tname, vecwise(got_t, want_t))


@pytest.mark.parametrize("tname", sorted(THETAS))
@pytest.mark.parametrize("name", ["perturbed20x20", "perturbed_x_only"])
def test_nn_step_adjoint_matches_oracle_tape(Solver, name, tname):
    """TVD-RK2 step adjoint: the state adjoint and the weight gradient."""
    case, W = CASES[name]
    _say(f"Rusanov-NN step adjoint parity: {name} / {tname}")
    s, th, tb = _solver(Solver, case, THETAS[tname], with_bar=True)
    U = s.init(W)
    Uo = oracle.state_init(case, W)
    Ub = _interior_noise(case, Uo.shape, 8)
    want_u, want_t = oracle.vjp_step_theta(case, Uo, 1e-3, Ub)
    got_u = s.step_adjoint(U, 1e-3, torch.from_numpy(Ub).cuda()).cpu().numpy()
    got_t = tb.cpu().numpy()
    s.close()
    assert normwise(got_u, want_u) <= 1e-10, (name, tname, normwise(got_u, want_u))
    assert vecwise(got_t, want_t) <= 1e-10, (name, tname, vecwise(got_t, want_t))


def test_nn_weight_gradient_is_repeatable_and_accumulates(Solver):
    """For a given Rbar the right-hand side's weight gradient is summed over the
    faces in a fixed order: a second identical call adds exactly the same
    values (the accumulator then holds twice the first). (Through a step the
    second stage's Rbar is a state adjoint summed with atomics, so there the
    weight gradient varies in its last bits like the state adjoint.)"""
    case, W = CASES["perturbed20x20"]
    _say("Rusanov-NN weight gradient repeatability")
    s, th, tb = _solver(Solver, case, THETAS["wide"], with_bar=True)
    U = s.init(W)
    Rb = torch.from_numpy(_interior_noise(case, tuple(U.shape), 9)).cuda()
    s.rhs_adjoint(U, Rb)
    first = tb.clone()
    s.rhs_adjoint(U, Rb)
    torch.cuda.synchronize()
    s.close()
    assert torch.any(first != 0)
    assert torch.equal(tb, 2.0 * first)


def test_nn_weights_update_in_place(Solver):
    """The weights are read at every launch: changing them in place changes the
    next step (captured steps included) as the oracle with the new weights."""
    case, W = CASES["perturbed20x20"]
    _say("Rusanov-NN in-place weight update")
    s, th, _ = _solver(Solver, case, THETAS["wide"])
    U = s.init(W)
    s.advance_fixed(U, 3, 1e-3)
    th.copy_(torch.from_numpy(THETAS["near_const"]))
    s.advance_fixed(U, 3, 1e-3)
    oracle.set_nn(THETAS["wide"])
    Uo, _, _ = oracle.advance(case, oracle.state_init(case, W), 3, fixed_dt=1e-3)
    oracle.set_nn(THETAS["near_const"])
    Uo, _, _ = oracle.advance(case, Uo, 3, fixed_dt=1e-3)
    e = normwise(U.cpu().numpy(), Uo)
    s.close()
    assert e <= 1e-12, e


def test_default_scheme_rk2_step_adjoint_matches_oracle_tape(Solver):
    """TVD-RK2 in the step adjoint also with the default scheme (WENO5-JS, HLLC)."""
    case, W = wl.random_smooth((14, 11, 9), seed=3, mu=0.02, flags=wl.ALL_PHYSICS | wl.RK2)
    _say("default scheme RK2 step adjoint")
    s = Solver(case)
    U = s.init(W)
    Uo = oracle.state_init(case, W)
    dt = 0.5 * oracle.cfl_dt(case, Uo)
    Ub = _interior_noise(case, Uo.shape, 10)
    want = oracle.vjp_rk3_step(case, Uo, dt, Ub)
    got = s.step_adjoint(U, dt, torch.from_numpy(Ub).cuda()).cpu().numpy()
    s.close()
    assert normwise(got, want) <= 1e-10, normwise(got, want)


def test_nn_configuration_errors(Solver):
    from paper_2203_13760_amd import cfd
    case, W = CASES["perturbed20x20"]
    s = Solver(case)
    U = s.init(W)
    with pytest.raises(cfd.CfdError) as e:  # no weights yet
        s.rhs(U)
    assert e.value.code == cfd.CFD_EINVAL
    s.close()
    for bad in (wl.INVISCID | wl.RUSANOV_NN, NN_FLAGS | wl.RUSANOV, NN_FLAGS | wl.WENOZ, NN_FLAGS | wl.ROE):
        with pytest.raises(cfd.CfdError) as e:
            Solver(dict(case, flags=bad))
        assert e.value.code == cfd.CFD_EINVAL
    plain = Solver(dict(case, flags=wl.INVISCID | wl.WENO3 | wl.RK2))
    with pytest.raises(cfd.CfdError) as e:
        plain.set_nn_weights(torch.zeros(cfd.CFD_NN_PARAMS, dtype=torch.float64, device="cuda"))
    assert e.value.code == cfd.CFD_EINVAL
    plain.close()
    visc = Solver(dict(case, flags=NN_FLAGS | wl.VISCOUS, mu=0.01))
    th = torch.from_numpy(THETAS["wide"]).cuda()
    visc.set_nn_weights(th)
    U = visc.init(W)
    with pytest.raises(cfd.CfdError) as e:
        visc.step_adjoint(U, 1e-3, torch.ones_like(U))
    assert e.value.code == cfd.CFD_EUNSUPPORTED
    visc.close()
    b = cfd.cfd_batch_create(4, 1 << 26)
    try:
        with pytest.raises(cfd.CfdError) as e:
            cfd.cfd_batch_add(b, case, torch.from_numpy(W).cuda())
        assert e.value.code == cfd.CFD_EUNSUPPORTED
    finally:
        torch.cuda.synchronize()
        cfd.cfd_batch_destroy(b)


def test_training_gradient_matches_central_differences(Solver):
    """The §7.4 training loss of a window (unrolled coarse steps against a
    coarse-grained truth) and its weight gradient from the step adjoints,
    against central differences of the loss along random weight directions (a
    one-sided difference where a ReLU unit of some face changes side within
    the step)."""
    from paper_2203_13760_amd.experiments import RusanovNNTrainer, cg_trajectory
    _say("Rusanov-NN training gradient vs central differences")
    traj = cg_trajectory(n_fine=64, n_cg=16, n_cg_steps=12)
    th0 = wl.nn_weights(seed=2, alpha0=1.2, scale=0.5)
    tr = RusanovNNTrainer(traj, th0, n_unroll=4)
    try:
        tr.theta_bar.zero_()
        L0 = float(tr._window(3) + tr._window(7))
        g = tr.theta_bar.clone()
        assert torch.any(g != 0)
        rng = np.random.default_rng(4)
        base = tr.theta.clone()
        for trial in range(3):
            v = torch.from_numpy(rng.standard_normal(base.numel())).cuda()
            h = 1e-6

            def L(t):
                tr.theta.copy_(t)
                return float(tr._window(3) + tr._window(7))
            Lp, Lm = L(base + h * v), L(base - h * v)
            tr.theta.copy_(base)
            ad = float(g @ v)
            fds = ((Lp - Lm) / (2 * h), (Lp - L0) / h, (L0 - Lm) / h)
            assert min(abs(f - ad) for f in fds) <= 1e-6 * max(abs(ad), 1e-3 * abs(L0)), (trial, fds, ad)
    finally:
        tr.close()


def _random_nn_config(rng):
    """A small Rusanov-NN configuration: 1-3 active ragged axes of 3..16 cells
    (3D included, so every axis's network kernels run), per-axis periodic,
    zero-gradient, wall or mixed boundaries, TVD-RK2 or RK3, smooth seeded data
    with 1 % seeded cell noise, seeded weights. (A smooth field whose velocity
    does not vary along an axis has |u_R - u_L| = 0 at every face of that axis,
    the kink of |x|: there the oracle sees an exact zero and the device, whose
    u = m (1/rho) rounds differently from m / rho, a jump of an ulp of either
    sign, so the two take different one-sided derivatives. The noise keeps
    every face off the kink.)"""
    while True:
        n = [int(rng.integers(3, 17)) if rng.random() < 0.8 else 1 for _ in range(3)]
        if any(x > 1 for x in n):
            break
    bc = []
    for d in range(3):
        bc += [[wl.PERIODIC] * 2, [wl.ZERO_GRADIENT] * 2, [wl.REFLECT] * 2,
               [wl.ZERO_GRADIENT, wl.REFLECT]][int(rng.integers(0, 4))]
    flags = wl.INVISCID | wl.WENO3 | wl.RUSANOV_NN | (wl.RK2 if rng.random() < 0.5 else 0)
    case, W = wl.random_smooth(tuple(n), seed=int(rng.integers(1 << 30)), mu=0.0, flags=flags, bc=tuple(bc))
    W = W * (1.0 + 0.01 * rng.standard_normal(W.shape))
    theta = wl.nn_weights(seed=int(rng.integers(1 << 30)), alpha0=float(rng.uniform(0.6, 2.0)),
                          scale=float(rng.uniform(0.2, 1.0)))
    return case, W, theta


@pytest.mark.parametrize("k", range(6))
def test_nn_random_configurations_match_oracle(Solver, k):
    """Seeded random Rusanov-NN configurations: the right-hand side, one fixed
    step, and the step adjoint (state and weights) against the oracle."""
    rng = np.random.default_rng(20230 + k)
    case, W, theta = _random_nn_config(rng)
    _say(f"Rusanov-NN random configuration {k}: n={case['n']} bc={case['bc']} flags={case['flags']}")
    s, th, tb = _solver(Solver, case, theta, with_bar=True)
    U = s.init(W)
    Uo = oracle.state_init(case, W)
    R = s.rhs(U).cpu().numpy()
    Ro = oracle.rhs(case, Uo)
    bound = oracle.rhs_rounding_bound(case, Uo)
    for v in range(5):
        err = float(np.max(np.abs(R[v] - Ro[v])))
        assert err <= max(1e-12 * float(np.max(np.abs(Ro[v]))), bound[v]), (k, v, err, bound[v])
    dt = 0.5 * oracle.cfl_dt(case, Uo)
    Ub = _interior_noise(case, Uo.shape, 30 + k)
    want_u, want_t = oracle.vjp_step_theta(case, Uo, dt, Ub)
    got_u = s.step_adjoint(U, dt, torch.from_numpy(Ub).cuda()).cpu().numpy()
    got_t = tb.cpu().numpy()
    assert normwise(got_u, want_u) <= 1e-10, (k, normwise(got_u, want_u))
    assert vecwise(got_t, want_t) <= 1e-10, (k, vecwise(got_t, want_t))
    s.step(U, dt)
    Uo1, _ = oracle.rk3_step(case, Uo, dt)
    e = normwise(U.cpu().numpy(), Uo1)
    s.close()
    assert e <= 1e-12, (k, e)


def test_nn_rk3_kept_stages_adjoint_matches_oracle_tape(Solver):
    """The Rusanov-NN flux with TVD-RK3: the kept-stage step and its adjoint
    (state and weights) against the oracle."""
    case, W = wl.random_smooth((13, 11, 7), seed=21, mu=0.0, flags=wl.INVISCID | wl.WENO3 | wl.RUSANOV_NN,
                               bc=(wl.REFLECT,) * 2 + (wl.PERIODIC,) * 2 + (wl.ZERO_GRADIENT,) * 2)
    _say("Rusanov-NN RK3 kept stages adjoint")
    s, th, tb = _solver(Solver, case, THETAS["wide"], with_bar=True)
    U = s.init(W)
    Uo = oracle.state_init(case, W)
    dt = 0.5 * oracle.cfl_dt(case, Uo)
    Un = U.clone()
    U1, U2 = torch.empty_like(U), torch.empty_like(U)
    s.step_stages(U, dt, U1, U2)
    Uo1, _ = oracle.rk3_step(case, Uo, dt)
    assert normwise(U.cpu().numpy(), Uo1) <= 1e-12
    Ub = _interior_noise(case, Uo.shape, 40)
    want_u, want_t = oracle.vjp_step_theta(case, Uo, dt, Ub)
    got_u = s.step_adjoint_stages(Un, U1, U2, dt, torch.from_numpy(Ub).cuda()).cpu().numpy()
    got_t = tb.cpu().numpy()
    s.close()
    assert normwise(got_u, want_u) <= 1e-10, normwise(got_u, want_u)
    assert vecwise(got_t, want_t) <= 1e-10, vecwise(got_t, want_t)


def test_training_window_graph_matches_eager(Solver):
    """The training window captured as one HIP graph (15 steps, the loss
    gradients, 15 step adjoints) against the same window run eagerly: every
    replay, with eager work and synchronisations between replays, gives the
    eager loss and weight gradient (to the run-to-run rounding of the
    adjoint's atomics), and a captured Adam batch equals an eager one."""
    from paper_2203_13760_amd.experiments import RusanovNNTrainer, cg_trajectory
    _say("Rusanov-NN training window: graph replays against eager")
    traj = cg_trajectory(n_fine=64, n_cg=16, n_cg_steps=30)
    th0 = wl.nn_weights(seed=2, alpha0=1.2, scale=0.5)
    eager = RusanovNNTrainer(traj, th0, n_unroll=6)
    graph = RusanovNNTrainer(traj, th0, n_unroll=6, graph=True)
    try:
        assert graph.solver.check() == 0  # the capture leaves no bad state behind
        for s0 in (0, 9, 4, 17):
            eager.theta_bar.zero_()
            graph.theta_bar.zero_()
            le = float(eager._window(s0))
            torch.cuda.synchronize()
            lg = float(graph._window(s0))
            torch.cuda.synchronize()
            assert abs(lg - le) <= 1e-12 * abs(le), (s0, lg, le)
            assert vecwise(graph.theta_bar.cpu().numpy(), eager.theta_bar.cpu().numpy()) <= 1e-10, s0
        for b in ([1, 5, 9], [2, 3]):
            le = eager.train_batch(b)
            lg = graph.train_batch(b)
            assert abs(lg - le) <= 1e-12 * abs(le), (b, lg, le)
            assert vecwise(graph.theta.cpu().numpy(), eager.theta.cpu().numpy()) <= 1e-12, b
        assert graph.solver.check() == 0 and eager.solver.check() == 0
    finally:
        eager.close()
        graph.close()


def test_nn_viscous_forward_matches_oracle(Solver):
    """The Rusanov-NN convective flux with the viscous and heat fluxes (forward
    only; the adjoint covers the inviscid Rusanov-NN): right-hand side, one
    CFL step and 20 fixed steps against the oracle, on a 3D walled grid."""
    case, W = wl.random_smooth((15, 12, 10), seed=31, mu=0.02,
                               flags=wl.ALL_PHYSICS | wl.WENO3 | wl.RUSANOV_NN | wl.RK2,
                               bc=(wl.REFLECT,) * 2 + (wl.ZERO_GRADIENT,) * 2 + (wl.PERIODIC,) * 2)
    W = W * (1.0 + 0.01 * np.random.default_rng(32).standard_normal(W.shape))
    _say("Rusanov-NN viscous forward")
    s, th, _ = _solver(Solver, case, THETAS["wide"])
    U = s.init(W)
    Uo = oracle.state_init(case, W)
    R = s.rhs(U).cpu().numpy()
    Ro = oracle.rhs(case, Uo)
    bound = oracle.rhs_rounding_bound(case, Uo)
    for v in range(5):
        err = float(np.max(np.abs(R[v] - Ro[v])))
        assert err <= max(1e-12 * float(np.max(np.abs(Ro[v]))), bound[v]), (v, err, bound[v])
    dt = s.step(U)
    Uo1, dto = oracle.rk3_step(case, Uo)
    assert abs(float(dt.item()) - dto) <= 1e-14 * dto
    assert normwise(U.cpu().numpy(), Uo1) <= 1e-12
    s.advance_fixed(U, 20, 0.5 * dto)
    Uo20, _, _ = oracle.advance(case, Uo1, 20, fixed_dt=0.5 * dto)
    e = normwise(U.cpu().numpy(), Uo20)
    s.close()
    assert e <= 1e-10, e
