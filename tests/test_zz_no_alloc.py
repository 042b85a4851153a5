"""The allocation-free TVD-RK3 step (cfd_rk3_step_noalloc, static device
scratch) against the solver-handle step cfd_rk3_step on the same inputs: the
same kernels run on the same data, so the results are bitwise equal. Two
calls in a row, the second on a smaller grid (the scratch keeps the first
call's contents), then the first grid again with a fixed step."""
import numpy as np
import pytest

from paper_2203_13760_amd import cfd
from paper_2203_13760_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver_step(case, W, dt):
    from paper_2203_13760_amd.solver import Solver
    s = Solver(case)
    U = s.init(W)
    dt_used = s.step(U, dt)
    out = (U.clone(), float(dt_used.item()), s.check())
    s.close()
    return out


def _noalloc_step(case, W, dt):
    from paper_2203_13760_amd.solver import Solver
    s = Solver(case)  # only to build the initial state
    U = s.init(W)
    s.close()
    dt_used = torch.zeros(1, dtype=torch.float64, device="cuda")
    cfd.cfd_rk3_step_noalloc(case, U, dt, dt_used)
    torch.cuda.synchronize()
    return U, float(dt_used.item())


def test_noalloc_step_equals_solver_step():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = wl.taylor_green(0, shape=(40, 36, 34))
    small = wl.kelvin_helmholtz(24, seed=3)
    walls = wl.implosion(20, flags=wl.INVISCID)
    for (case, W), dt in ((big, 0.0), (small, 0.0), (walls, 0.0), (big, 1e-3)):
        print(f"noalloc step vs solver step: n={case['n']} dt={dt}", flush=True)
        Ua, dta = _noalloc_step(case, W, dt)
        Ub, dtb, health = _solver_step(case, W, dt)
        # bits 0-2: every state of the step is physical (bit 3 may report faces
        # of the implosion's corner where WENO5-JS reconstructs a non-positive
        # pressure next to the walls)
        assert health & 7 == 0
        assert dta == dtb and dta > 0
        assert torch.equal(Ua, Ub), float((Ua - Ub).abs().max())


def test_noalloc_step_rejects_grids_beyond_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    case, W = wl.taylor_green(0, shape=(72, 72, 72))  # 78^3 padded cells > 386309
    U = torch.zeros((5, 78, 78, 78), dtype=torch.float64, device="cuda")
    with pytest.raises(cfd.CfdError) as e:
        cfd.cfd_rk3_step_noalloc(case, U, 0.0)
    assert e.value.code == cfd.CFD_EINVAL and "too large" in str(e.value)
    assert float(U.abs().max()) == 0.0
