"""Serving form: forward+adjoint+gradient solves of mixed grid sizes served
with continuous batching on one GPU.

Requests arrive over time.  The server admits the oldest arrived request
whose grid size is below its concurrency cap, as soon as a batch slot is free
and its HBM footprint (``hyb_footprint``) fits in the budget.  Admitted
requests run as slots of one ``hyb_batch``: every tick advances every running
slot by one time step; slots of the same grid size share each kernel launch
while sitting at different steps and phases, and each grid size has its own
stream so that work of different sizes overlaps on the device.  Contexts
(wavefields, history, traces) stay resident in a per-size pool and are
reused by later requests.  Latency is measured from arrival to the moment
the server observes the result.  ``run_unbatched`` is the baseline: the same
library, one request at a time in arrival order.

This module schedules and measures; every step of the method runs in the HIP
library.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import hyb, synth


@dataclasses.dataclass
class Request:
    id: int
    n: int
    C: int
    nt: int
    dt: float
    omega: float
    sigma: object        # device tensor [C, C, C] (FP64)
    sigma_max: float
    arrival: float       # seconds after the start of the run


@dataclasses.dataclass
class Result:
    id: int
    n: int
    arrival: float
    admitted: float
    finished: float
    J: float
    grad: object = None  # host copy when kept
    obs: object = None   # host copy of the trace when kept

    @property
    def latency(self):
        return self.finished - self.arrival


class _Entry:
    """A resident context with its trace and gradient buffers, on the stream
    of its grid size."""

    def __init__(self, n, C, f32, stream):
        import torch
        self.stream = stream
        self.solver = hyb.Solver(n, C=C, f32=f32, stream=stream.cuda_stream)
        self.obs = torch.zeros((5 * n + 1, n + 1, n + 1), dtype=torch.float64, device="cuda")
        self.grad = torch.zeros((C, C, C), dtype=torch.float64, device="cuda")
        self.busy = False


class Pool:
    """Per-size pool of resident contexts under an HBM budget (bytes).  Each
    grid size gets its own stream (default priority), so work of different
    sizes overlaps on the device."""

    def __init__(self, budget, f32=True):
        import torch
        self.budget = budget
        self.f32 = f32
        self.entries = {}
        self.streams = {}
        self.used = 0
        self._fp = {}
        self._torch = torch

    def stream(self, n):
        if n not in self.streams:
            self.streams[n] = self._torch.cuda.Stream()
        return self.streams[n]

    def footprint(self, n, C, nt):
        key = (n, C, nt)
        if key not in self._fp:
            grid = hyb.make_grid(n)
            mesh = hyb.make_mesh(*synth.kuhn_box_mesh((n - C) // 2, C, 1.0 / n))
            b = hyb.hyb_footprint(grid, mesh, 2, hyb.make_opts(self.f32), nt)
            trace = 2 * (nt + 1) * (n + 1) ** 2 * 8 + C ** 3 * 8  # caller buffers
            self._fp[key] = b + trace
        return self._fp[key]

    def acquire(self, n, C, nt):
        for e in self.entries.get(n, []):
            if not e.busy:
                e.busy = True
                return e
        fp = self.footprint(n, C, nt)
        if self.used + fp > self.budget:
            return None
        e = _Entry(n, C, self.f32, self.stream(n))
        e.busy = True
        self.entries.setdefault(n, []).append(e)
        self.used += fp
        return e

    def release(self, e):
        e.busy = False

    def warm(self, caps, shapes):
        """Create the resident contexts up front, as a server does at start-up:
        up to caps[n] per grid size n (shapes[n] = (C, nt)), smallest sizes
        first, within the HBM budget."""
        import torch
        for n in sorted(caps):
            C, nt = shapes[n]
            have = len(self.entries.get(n, []))
            for _ in range(caps[n] - have):
                fp = self.footprint(n, C, nt)
                if self.used + fp > self.budget:
                    break
                e = _Entry(n, C, self.f32, self.stream(n))
                self.entries.setdefault(n, []).append(e)
                self.used += fp
        torch.cuda.synchronize()

    def close(self):
        self._torch.cuda.synchronize()
        for lst in self.entries.values():
            for e in lst:
                e.solver.close()
        self.entries.clear()
        self.used = 0


def background_data(sizes, f32=True, omega=40.0):
    """Per grid size: the trace of the homogeneous medium (a = 1), the data
    every request of that size is fitted against (device, FP64)."""
    import torch
    out = {}
    for n in sizes:
        C = 3 * n // 8
        s = hyb.Solver(n, C=C, f32=f32)
        out[n] = s.forward(None, 5 * n, 0.25 / n, omega=omega).clone()
        s.close()
    torch.cuda.synchronize()
    return out


def make_requests(n_req, seed, rate, sizes=synth.SERVE_SIZES):
    """Seeded request stream: sizes uniform over `sizes`, FEM box 3/8 of the
    edge, 1-4 cubic inclusions, nt = 5 n, dt = 0.25 h, Poisson arrivals at
    `rate` per second.  sigma is staged on the device up front."""
    import torch
    specs = synth.serve_requests(n_req, seed, sizes)
    arr = synth.poisson_arrivals(n_req, rate, seed + 1)
    out = []
    for sp, t in zip(specs, arr):
        sig = synth.cubes(sp["C"], sp["sigma_seed"])
        out.append(Request(sp["id"], sp["n"], sp["C"], sp["nt"], 0.25 / sp["n"], sp["omega"],
                           torch.as_tensor(sig, dtype=torch.float64, device="cuda"), float(sig.max()),
                           float(t)))
    torch.cuda.synchronize()
    return out


# Concurrency caps per grid size: enough same-size slots to fill the device
# in one launch (a 64^3 step alone is launch-bound, a 256^3 step alone already
# streams at HBM rate), few enough that every admitted request advances.
DEFAULT_CAPS = {64: 64, 96: 32, 128: 16, 192: 4, 256: 4}
# Time steps enqueued per scheduler pass: the host plans them 32 at a time
# and polls for finished requests between passes.
DEFAULT_STEPS_PER_CALL = 128


def shapes_of(requests):
    """(C, nt) per grid size, for Pool.warm."""
    return {r.n: (r.C, r.nt) for r in requests}


def run_batched(requests, data, budget=200e9, max_slots=64, f32=True, keep_grads=False, pool=None,
                caps=None, steps_per_call=DEFAULT_STEPS_PER_CALL, keep_obs=False):
    """Continuous batching.  Admission: the oldest arrived request whose size
    is below its concurrency cap and whose footprint fits.  Returns (results
    sorted by id, wall seconds)."""
    import torch
    caps = caps or DEFAULT_CAPS
    own_pool = pool is None
    pool = pool or Pool(budget, f32)
    b = hyb.hyb_batch_create(max_slots, None)
    waiting = sorted(requests, key=lambda r: r.arrival)
    queued = []                      # arrived, not admitted (arrival order)
    head = 0
    running = {}                     # slot -> (request, entry, admitted)
    n_run = {}
    results = []
    t0 = time.perf_counter()
    try:
        while head < len(waiting) or queued or running:
            now = time.perf_counter() - t0
            while head < len(waiting) and waiting[head].arrival <= now:
                queued.append(waiting[head])
                head += 1
            i = 0
            while i < len(queued) and len(running) < max_slots:
                r = queued[i]
                if n_run.get(r.n, 0) >= caps.get(r.n, 1):
                    i += 1
                    continue
                e = pool.acquire(r.n, r.C, r.nt)
                if e is None:
                    i += 1
                    continue
                slot = hyb.hyb_batch_submit(b, e.solver.ctx, r.sigma, r.sigma_max,
                                            hyb.make_source(r.omega), r.nt, r.dt, data[r.n], e.obs, e.grad)
                running[slot] = (r, e, now)
                n_run[r.n] = n_run.get(r.n, 0) + 1
                queued.pop(i)
            n_act = hyb.hyb_batch_tick(b, steps_per_call) if running else 0
            states, Js = hyb.hyb_batch_poll_all(b, max_slots) if running else ([], [])
            for slot in list(running):
                st, J = states[slot], Js[slot]
                if st >= 2:
                    r, e, adm = running.pop(slot)
                    n_run[r.n] -= 1
                    fin = time.perf_counter() - t0
                    g = o = None
                    if keep_grads or keep_obs:
                        with torch.cuda.stream(e.stream):
                            g = e.grad.cpu().numpy().copy() if keep_grads else None
                            o = e.obs[:r.nt + 1].cpu().numpy().copy() if keep_obs else None
                    hyb.hyb_batch_release(b, slot)
                    pool.release(e)
                    if st == 3:
                        raise RuntimeError(f"request {r.id} failed: {hyb.hyb_batch_last_error(b)}")
                    results.append(Result(r.id, r.n, r.arrival, adm, fin, J, g, o))
            if not running and not queued and head < len(waiting):
                wait = waiting[head].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif n_act == 0 and running:
                time.sleep(0.0002)  # all work enqueued; wait for the device
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        hyb.hyb_batch_destroy(b)
        if own_pool:
            pool.close()
    return sorted(results, key=lambda x: x.id), wall


def run_unbatched(requests, data, f32=True, keep_grads=False, pool=None, keep_obs=False):
    """Baseline: one request at a time, in arrival order, through hyb_forward,
    hyb_adjoint and hyb_gradient on resident contexts."""
    import torch
    own_pool = pool is None
    pool = pool or Pool(float("inf"), f32)
    results = []
    t0 = time.perf_counter()
    try:
        for r in sorted(requests, key=lambda q: q.arrival):
            now = time.perf_counter() - t0
            if r.arrival > now:
                time.sleep(r.arrival - now)
            adm = time.perf_counter() - t0
            e = pool.acquire(r.n, r.C, r.nt)
            s = e.solver
            with torch.cuda.stream(e.stream):
                obs = s.forward(r.sigma, r.nt, r.dt, omega=r.omega, obs=e.obs)
                s.adjoint(obs - data[r.n], mode=0)
                _, J = s.gradient(e.grad, want_J=True)
                fin = time.perf_counter() - t0
                g = e.grad.cpu().numpy().copy() if keep_grads else None
                o = obs[:r.nt + 1].cpu().numpy().copy() if keep_obs else None
            pool.release(e)
            results.append(Result(r.id, r.n, r.arrival, adm, fin, J, g, o))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        if own_pool:
            pool.close()
    return sorted(results, key=lambda x: x.id), wall


def summarize(results, wall, requests):
    lat = np.array([r.latency for r in results])
    upd = 0.0
    by_n = {r.id: r for r in requests}
    for res in results:
        r = by_n[res.id]
        n, C = r.n, r.C
        nodes = (n + 1) ** 3 - (C - 3) ** 3 + (C - 1) ** 3
        upd += 2.0 * nodes * r.nt
    return {"requests": len(results), "wall_s": round(wall, 3),
            "throughput_req_s": round(len(results) / wall, 3),
            "gupd_s": round(upd / wall / 1e9, 2),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_ms": round(float(lat.mean()) * 1e3, 2)}
