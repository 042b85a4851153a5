"""Serving batch: the batched persistent path against the CPU oracle, the same
result alone and in a mix of other grids (bitwise), admission by arena
footprint, and the scheduler end to end (batched vs one at a time)."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_13760_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def normwise(a, b):
    err = 0.0
    for v in range(a.shape[0]):
        den = float(np.max(np.abs(b[v])))
        num = float(np.max(np.abs(a[v] - b[v])))
        if num:
            err = max(err, num / den if den > 0 else math.inf)
    return err


@pytest.fixture(scope="module")
def cfd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_13760_amd import cfd as c
    return c


def _mix():
    P, Z = wl.PERIODIC, wl.ZERO_GRADIENT
    return [
        wl.taylor_green(0, shape=(20, 18, 16)),
        wl.kelvin_helmholtz(48, seed=1),
        wl.random_shocky((37, 13, 9), seed=11),
        wl.sod(200),
        wl.random_smooth((33, 29, 35), seed=3, mu=0.02, bc=(P, P, Z, Z, P, P)),
        # no x axis: the primitive pass at every stage instead of the x sweep's
        wl.random_shocky((1, 26, 19), seed=5),
        # reflecting walls (the implosion of §7.4 with the default scheme)
        wl.implosion(40, flags=wl.INVISCID),
    ]


def _run(cfd, grids, steps):
    b = cfd.cfd_batch_create(16, 2 << 30)
    slots = []
    for case, W in grids:
        s = cfd.cfd_batch_add(b, case, torch.from_numpy(np.ascontiguousarray(W)).cuda())
        assert s is not None
        slots.append(s)
    assert cfd.cfd_batch_count(b) == len(grids)
    for _ in range(steps):
        cfd.cfd_batch_step(b)
    out = []
    from paper_2203_13760_amd.solver import padded_shape
    for (case, _), s in zip(grids, slots):
        cfd.cfd_batch_finish(b, s)
        U = torch.empty(padded_shape(case), dtype=torch.float64, device="cuda")
        cfd.cfd_batch_copy_state(b, s, U)
        out.append(U.cpu().numpy())
    torch.cuda.synchronize()
    cfd.cfd_batch_destroy(b)
    return out


def test_batched_path_matches_oracle(cfd):
    grids = _mix()
    print("batched parity: 7 mixed grids, 20 steps", flush=True)
    got = _run(cfd, grids, 20)
    for (case, W), U in zip(grids, got):
        Uo, _, n = oracle.advance(case, oracle.state_init(case, W), 20)
        e = normwise(U, Uo)
        assert e <= 1e-10, (case["n"], e)


def test_alone_equals_in_mix_bitwise(cfd):
    grids = _mix()
    print("alone vs in the mix", flush=True)
    together = _run(cfd, grids, 10)
    for k in (0, 1, 4, 5, 6):
        alone = _run(cfd, [grids[k]], 10)[0]
        assert np.array_equal(alone, together[k]), k


def _march_blocks(case, seg):
    """Workgroups of a grid's y (or z) march at a segment length (the launch
    shape of sweep_march_blocks: 64 x per block row, four columns per block)."""
    n = case["n"]
    return -(-n[0] // 64) * -(-(n[2] * -(-n[1] // seg)) // 4)


def test_long_march_segments_of_a_full_batch_equal_each_grid_alone(cfd):
    """A resident set whose y and z march phases hold a block for every one of
    the 2048 persistent workgroups with 128-cell segments marches with those;
    each grid alone keeps 32-cell segments. The results agree bitwise (every
    face flux is computed the same way whatever the segment length), and the
    grid alone is the path the oracle parity tests cover."""
    grids = [wl.taylor_green_noisy(192, sigma=1e-3, seed=40 + k) for k in range(8)]
    assert sum(_march_blocks(c, 128) for c, _ in grids) >= 2048
    assert _march_blocks(grids[0][0], 64) < 2048
    print("long march segments: 8 x TGV 192^3 + noise, 2 steps, mix vs alone", flush=True)

    def run(sel, arena):
        b = cfd.cfd_batch_create(8, arena)
        slots = [cfd.cfd_batch_add(b, grids[k][0], torch.from_numpy(np.ascontiguousarray(grids[k][1])).cuda())
                 for k in sel]
        assert None not in slots
        for _ in range(2):
            cfd.cfd_batch_step(b)
        from paper_2203_13760_amd.solver import padded_shape
        out = []
        for k, sl in zip(sel, slots):
            cfd.cfd_batch_finish(b, sl)
            U = torch.empty(padded_shape(grids[k][0]), dtype=torch.float64, device="cuda")
            cfd.cfd_batch_copy_state(b, sl, U)
            out.append(U.cpu().numpy())
        torch.cuda.synchronize()
        cfd.cfd_batch_destroy(b)
        return out

    mix = run(list(range(8)), 24 << 30)
    for k in (0, 5):
        alone = run([k], 4 << 30)[0]
        assert np.array_equal(alone, mix[k]), k


def test_step_graphs_beyond_the_cache_keep_results(cfd):
    """The step graph is kept per pattern of launched phases (chain count and
    each sub-batch's phases and launch widths), 16 patterns at most. Cycling
    one batch through the singles, pairs and triples of the mix's grids (3D,
    2D, 1D along x, no x axis: different phase sets) meets more patterns than
    that, so the kept graphs are dropped and captured again; a resident set
    stepped afterwards gives the same bits as in a fresh batch."""
    import itertools
    grids = _mix()
    Ws = [torch.from_numpy(np.ascontiguousarray(W)).cuda() for _, W in grids]
    subsets = [c for r in (1, 2, 3) for c in itertools.combinations(range(len(grids)), r)]
    print(f"step graph cache: {len(subsets)} resident sets, one step each", flush=True)
    b = cfd.cfd_batch_create(16, 2 << 30)
    for sub in subsets:
        slots = [cfd.cfd_batch_add(b, grids[k][0], Ws[k]) for k in sub]
        assert None not in slots
        cfd.cfd_batch_step(b)
        torch.cuda.synchronize()
        for sl in slots:
            cfd.cfd_batch_remove(b, sl)
    final = (0, 1, 5)
    slots = [cfd.cfd_batch_add(b, grids[k][0], Ws[k]) for k in final]
    for _ in range(3):
        cfd.cfd_batch_step(b)
    from paper_2203_13760_amd.solver import padded_shape
    got = []
    for k, sl in zip(final, slots):
        cfd.cfd_batch_finish(b, sl)
        U = torch.empty(padded_shape(grids[k][0]), dtype=torch.float64, device="cuda")
        cfd.cfd_batch_copy_state(b, sl, U)
        got.append(U.cpu().numpy())
    torch.cuda.synchronize()
    cfd.cfd_batch_destroy(b)
    fresh = _run(cfd, [grids[k] for k in final], 3)
    for k, U, V in zip(final, got, fresh):
        assert np.array_equal(U, V), k


def test_admission_by_footprint(cfd):
    case, W = wl.taylor_green(32)
    need = cfd.cfd_batch_footprint(case)
    print(f"admission: footprint {need} bytes", flush=True)
    b = cfd.cfd_batch_create(8, int(2.5 * need))
    Wt = torch.from_numpy(W).cuda()
    s0 = cfd.cfd_batch_add(b, case, Wt)
    s1 = cfd.cfd_batch_add(b, case, Wt)
    s2 = cfd.cfd_batch_add(b, case, Wt)
    assert s0 is not None and s1 is not None and s2 is None
    cfd.cfd_batch_step(b)
    torch.cuda.synchronize()
    cfd.cfd_batch_remove(b, s0)
    s3 = cfd.cfd_batch_add(b, case, Wt)
    assert s3 is not None and cfd.cfd_batch_count(b) == 2
    cfd.cfd_batch_step(b)
    torch.cuda.synchronize()
    cfd.cfd_batch_destroy(b)


def test_server_batched_and_one_at_a_time_agree(cfd):
    from paper_2203_13760_amd import serving
    reqs_a = serving.mixed_workload(n_requests=10, rate=500.0, seed=5, steps=15,
                                    kh_range=(64, 96), tgv_range=(24, 40))
    reqs_b = serving.mixed_workload(n_requests=10, rate=500.0, seed=5, steps=15,
                                    kh_range=(64, 96), tgv_range=(24, 40))
    print("server: 10 requests batched and one at a time", flush=True)
    srv = serving.BatchServer(max_grids=32, arena_bytes=4 << 30)
    ra = srv.run(reqs_a, keep_results=True)
    rb = srv.run(reqs_b, max_resident=1, keep_results=True)
    srv.close()
    assert ra["requests"] == rb["requests"] == 10
    for x, y in zip(sorted(reqs_a, key=lambda r: r.rid), sorted(reqs_b, key=lambda r: r.rid)):
        assert torch.equal(x.result, y.result), x.rid
    # the torch-built initial conditions are the generator's fields
    r0 = sorted(reqs_a, key=lambda r: r.rid)[0]
    n = r0.case["n"][0]
    ref = wl.kelvin_helmholtz(n)[1] if r0.case["n"][2] == 1 else wl.taylor_green(n)[1]
    if r0.case["n"][2] != 1:
        assert np.allclose(r0.make_W().cpu().numpy(), ref, rtol=0, atol=1e-14)


def test_random_mix_matches_oracle(cfd):
    """Eight seeded random grids of the default scheme (1-3 active axes,
    periodic, zero-gradient or reflecting boundaries, with and without viscous
    and heat fluxes) resident together, 10 steps each, against the oracle."""
    rng = np.random.default_rng(77)
    grids = []
    while len(grids) < 8:
        n = tuple(int(rng.integers(3, 30)) if rng.random() < 0.75 else 1 for _ in range(3))
        if all(x == 1 for x in n):
            continue
        bc = []
        for _ in range(3):
            bc += [[wl.PERIODIC] * 2, [wl.ZERO_GRADIENT] * 2, [wl.REFLECT] * 2][int(rng.integers(0, 3))]
        flags = wl.INVISCID | [0, wl.VISCOUS | wl.HEAT][int(rng.integers(0, 2))]
        grids.append(wl.random_smooth(n, seed=int(rng.integers(1 << 30)), mu=0.02, flags=flags, bc=tuple(bc)))
    print("random batched mix: 8 grids, 10 steps", flush=True)
    got = _run(cfd, grids, 10)
    for (case, W), U in zip(grids, got):
        Uo, _, _ = oracle.advance(case, oracle.state_init(case, W), 10)
        assert normwise(U, Uo) <= 1e-10, (case["n"], case["bc"], case["flags"])
