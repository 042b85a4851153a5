"""Continuous-batching serving loop over the libcfd batch.

Requests (an initial condition plus a number of TVD-RK3 steps) arrive over
time. Each tick the scheduler admits queued requests in arrival order while a
slot and arena space are free (admission by HBM footprint), advances every
resident grid by one step with one replay of the batch's step graph, and
retires the grids that have taken all their steps. Requests that arrive while
others are running join at the next tick, so their work overlaps on the GPU.
`max_resident=1` gives the one-solve-at-a-time baseline with the same kernels
and graph.
"""
from __future__ import annotations

import collections
import math
import time

import numpy as np
import torch

from . import cfd
from . import workloads as wl


class Request:
    __slots__ = ("rid", "arrival", "case", "make_W", "steps", "slot", "done_steps", "admitted",
                 "completed", "cells", "result")

    def __init__(self, rid, arrival, case, make_W, steps):
        self.rid, self.arrival, self.case, self.make_W, self.steps = rid, arrival, case, make_W, steps
        self.slot = None
        self.done_steps = 0
        self.admitted = None
        self.completed = None
        self.cells = int(np.prod(case["n"]))
        self.result = None


# ---------------------------------------------------------------- workloads
def _centres(n, lo, hi, device):
    dx = (hi - lo) / n
    return lo + (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * dx


def tgv_request_W(n, device="cuda", ma=0.1, gamma=1.4):
    """Taylor-Green initial primitives on the GPU (same fields as workloads.taylor_green)."""
    x = _centres(n, 0.0, 2 * math.pi, device)
    Z, Y, X = torch.meshgrid(x, x, x, indexing="ij")
    W = torch.empty((5, n, n, n), dtype=torch.float64, device=device)
    W[0] = 1.0
    W[1] = torch.sin(X) * torch.cos(Y) * torch.cos(Z)
    W[2] = -torch.cos(X) * torch.sin(Y) * torch.cos(Z)
    W[3] = 0.0
    W[4] = 1.0 / (gamma * ma * ma) + (torch.cos(2 * X) + torch.cos(2 * Y)) * (torch.cos(2 * Z) + 2.0) / 16.0
    return W


def kh_request_W(n, phase, device="cuda", amplitude=0.01):
    """Kelvin-Helmholtz initial primitives on the GPU (same fields as workloads.kelvin_helmholtz)."""
    x = _centres(n, 0.0, 1.0, device)
    Y, X = torch.meshgrid(x, x, indexing="ij")
    inside = (Y - 0.5).abs() < 0.25
    W = torch.empty((5, 1, n, n), dtype=torch.float64, device=device)
    W[0, 0] = torch.where(inside, 2.0, 1.0)
    W[1, 0] = torch.where(inside, 0.5, -0.5)
    W[2, 0] = amplitude * torch.sin(4 * math.pi * (X + phase))
    W[3, 0] = 0.0
    W[4, 0] = 2.5
    return W


def mixed_workload(n_requests=400, rate=200.0, seed=3, steps=200, kh_fraction=0.6,
                   kh_range=(64, 1024), tgv_range=(32, 128)):
    """Seeded Poisson arrivals of Kelvin-Helmholtz (2D, inviscid) and
    Taylor-Green (3D, viscous) solves with uniformly drawn grid sides."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        if rng.random() < kh_fraction:
            n = int(rng.integers(kh_range[0], kh_range[1] + 1))
            phase = float(np.random.default_rng(int(rng.integers(1 << 31))).random())
            case = wl.make_case((n, n, 1), bc=(wl.PERIODIC,) * 6, flags=wl.INVISCID)
            make_W = (lambda n=n, phase=phase: kh_request_W(n, phase))
        else:
            n = int(rng.integers(tgv_range[0], tgv_range[1] + 1))
            case, _ = wl.taylor_green(0, shape=(3, 3, 3))
            case = dict(case)
            case["n"] = (n, n, n)
            make_W = (lambda n=n: tgv_request_W(n))
        reqs.append(Request(rid, t, case, make_W, steps))
    return reqs


# ---------------------------------------------------------------- server
class BatchServer:
    def __init__(self, max_grids=256, arena_bytes=64 << 30):
        self.b = cfd.cfd_batch_create(max_grids, arena_bytes)
        self.max_grids = max_grids

    def close(self):
        if self.b:
            torch.cuda.synchronize()
            cfd.cfd_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def read_state(self, slot, case):
        """Copy of a resident grid's padded state (halos refreshed)."""
        from .solver import padded_shape
        cfd.cfd_batch_finish(self.b, slot)
        out = torch.empty(padded_shape(case), dtype=torch.float64, device="cuda")
        cfd.cfd_batch_copy_state(self.b, slot, out)
        return out

    def run(self, requests, max_resident=None, realtime=True, keep_results=False, log=None):
        """Serve `requests` (sorted by arrival); returns per-request records and totals.
        realtime=False admits every request at time 0 (closed-loop throughput).

        Continuous batching: requests that arrive while a step runs are
        admitted on a side stream during that step (initial field, state and
        primitives of the new grid, in arena space no running step touches)
        and join at the next step; the step stream waits for the admissions
        before the next step uploads the grid table. With one resident grid at
        most, a request is admitted only once the previous one has left."""
        max_resident = max_resident or self.max_grids
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        resident = []
        stream = torch.cuda.current_stream()
        side = torch.cuda.Stream()  # default priority, like every stream here
        done = []
        ticks = 0
        cell_updates = 0
        t0 = time.perf_counter()
        last_log = t0

        def arrivals():
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                queue.append(pending.popleft())

        def admit(limit):
            out = []
            while queue and limit(len(out)):
                r = queue[0]
                with torch.cuda.stream(side):
                    W = r.make_W()
                    slot = cfd.cfd_batch_add(self.b, r.case, W, stream=side)
                    del W
                if slot is None:
                    break  # wait for memory to free up
                r.slot = slot
                r.admitted = time.perf_counter() - t0
                out.append(queue.popleft())
            return out

        while pending or queue or resident:
            arrivals()
            if not resident:
                resident = admit(lambda k: k < max_resident)
                stream.wait_stream(side)
                if not resident:
                    if pending:
                        time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
                    continue
            cfd.cfd_batch_step(self.b)
            # admissions overlap the running step; they start at the next one
            arrivals()
            joining = admit(lambda k: len(resident) + k < max_resident)
            stream.synchronize()
            ticks += 1
            tnow = time.perf_counter() - t0
            still = []
            for r in resident:
                r.done_steps += 1
                cell_updates += r.cells
                if r.done_steps >= r.steps:
                    r.completed = tnow
                    if keep_results:
                        r.result = self.read_state(r.slot, r.case)
                    stream.synchronize()
                    cfd.cfd_batch_remove(self.b, r.slot)
                    done.append(r)
                else:
                    still.append(r)
            resident = still + joining
            stream.wait_stream(side)
            if log and time.perf_counter() - last_log > 5.0:
                last_log = time.perf_counter()
                log(f"serving: t={tnow:.1f}s done={len(done)} resident={len(resident)} queued={len(queue)} "
                    f"pending={len(pending)}")
        wall = time.perf_counter() - t0
        lat = np.array([r.completed - r.arrival for r in done]) if realtime else \
            np.array([r.completed for r in done])
        return {
            "requests": len(done), "wall_s": wall, "ticks": ticks,
            "throughput_req_s": len(done) / wall,
            "mcell_updates_s": cell_updates / wall / 1e6,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()),
        }
