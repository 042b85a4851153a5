"""Long oracle computations behind the full-size GPU parity tests.

Each job is a plain call of the oracle on seeded inputs. A job starts in a
background thread as soon as a selected test that needs it has been collected
(see conftest.py), so that it runs beside the GPU tests: the oracle's C entry
points release the interpreter lock. A test then waits for its result.
"""
from __future__ import annotations

import threading

import numpy as np

import oracle
from paper_2203_13760_amd import workloads as wl

_JOBS = {}
_STATE = {}
_LOCK = threading.Lock()


def job(fn):
    _JOBS[fn.__name__] = fn
    return fn


def start(name):
    with _LOCK:
        if name in _STATE:
            return
        box = {"done": threading.Event(), "value": None, "error": None}

        def run():
            try:
                box["value"] = _JOBS[name]()
            except BaseException as e:  # re-raised in the waiting test
                box["error"] = e
            finally:
                box["done"].set()

        t = threading.Thread(target=run, name=f"oracle-{name}", daemon=True)
        _STATE[name] = box
        t.start()


def result(name, timeout=900.0):
    start(name)
    box = _STATE[name]
    if not box["done"].wait(timeout):
        raise TimeoutError(f"oracle job {name} did not finish in {timeout} s")
    if box["error"] is not None:
        raise box["error"]
    return box["value"]


# ---------------------------------------------------------------- jobs
@job
def tgv64_100():
    """Taylor-Green vortex 64^3 (Re 1600, Ma 0.1) after 100 CFL steps."""
    case, W = wl.taylor_green(64)
    U, t, n = oracle.advance(case, oracle.state_init(case, W), 100)
    return {"U": U, "t": t, "steps": n}


HIT_PLANES = (100, 8)  # first z-plane and count of the compared planes
HIT_MARGIN = 9  # a step depends on cells within 3 per stage


@job
def hit256_planes():
    """One fixed-dt step of the 256^3 headline field on the z-slab of the
    compared planes plus 9 margin planes on each side (zero-gradient ends:
    the margins absorb the wrong halo, exactly 3 cells per stage), with the
    CFL step of the whole field."""
    case, W = wl.isotropic_turbulence(256, seed=2203)
    dt = oracle.cfl_dt(case, oracle.state_init(case, W))
    k0, nk = HIT_PLANES
    lo, hi = k0 - HIT_MARGIN, k0 + nk + HIT_MARGIN
    sub = dict(case)
    dz = (case["hi"][2] - case["lo"][2]) / case["n"][2]
    sub["n"] = (case["n"][0], case["n"][1], hi - lo)
    sub["lo"] = (case["lo"][0], case["lo"][1], case["lo"][2] + dz * lo)
    sub["hi"] = (case["hi"][0], case["hi"][1], case["lo"][2] + dz * hi)
    sub["bc"] = case["bc"][:4] + (wl.ZERO_GRADIENT, wl.ZERO_GRADIENT)
    Us = oracle.state_init(sub, np.ascontiguousarray(W[:, lo:hi]))
    Us, _ = oracle.rk3_step(sub, Us, dt)
    planes = oracle.interior(sub, Us)[:, HIT_MARGIN:HIT_MARGIN + nk].copy()
    return {"dt": dt, "planes": planes}


def serving_large_mix():
    """The serving grids whose x-sweep phase exceeds the batch kernel's
    dynamic threshold together: a Taylor-Green vortex at 128^3 and two
    Kelvin-Helmholtz layers at 1024^2."""
    return [wl.taylor_green(128), wl.kelvin_helmholtz(1024, seed=7), wl.kelvin_helmholtz(1024, seed=8)]


SERVING_STEPS = 3


@job
def serving_large():
    out = []
    for case, W in serving_large_mix():
        U, _, _ = oracle.advance(case, oracle.state_init(case, W), SERVING_STEPS)
        out.append(U)
    return out
