"""Benchmark: forward+adjoint grid-point updates per second of the hybrid
FEM/FDM solver on one MI355X, on the 256^3 reconstruction workload (FEM box
96^3 cells x 6 tetrahedra, 1200 steps, 1-4 cubic inclusions, 3% noise).

One timed step = one iteration of Algorithm 3: the adjoint sweep at the
current iterate with the fused FP64 gradient integral, the gradient
finalisation, the direction, and one forward sweep per trial step of the
step search (the accepted trial's sweep serves the next iteration), all on
the device with inputs resident in HBM.  value = (forward + adjoint sweeps
run) * (FDM-updated + FEM-updated nodes) * nt / wall time.  The line also
carries the roofline of the dominant kernel (the fused FDM/FEM interior
update), timed with HIP events on the solver's stream, the CPU oracle timed
on a bounded window of the same workload (all host threads and one), and
legs for the other workloads: the 40^3 parity case (time and errors against
the oracle), the differentiation workload at 384^3 and the precision
workload at 512^3 (rate and interior roofline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--workload cg256] [--probe {interior,copy}]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def interior_bytes(n, C, s, streams=3):
    """Algorithmic bytes of one forward interior launch (fused FDM + FEM),
    the minimum the leapfrog must move with perfect neighbour reuse: per FDM
    node read u^k, read u^{k-1}, write u^{k+1} (3 s, s the field element
    size).  FEM nodes: the same plus one coefficient per cube (s) and one
    history write per stored node (s).  Rows of the six absorbing faces
    away from the edges (the launch computes them): read u^k, write
    u^{k+1}.  The overlap copy: one write per node of omega_diamond (into the
    grid level; the FEM rows read omega_o from the grid).  streams=4 counts
    what the FP32 increment form moves: read u^k, d^k, write d^{k+1}, u^{k+1}
    (4 s per node, d^{k+1} also on the faces)."""
    m = streams
    fdm_int = (n - 1) ** 3 - (C - 3) ** 3 if C else (n - 1) ** 3
    fem = (C - 1) ** 3 if C else 0
    faces = 6 * (n - 1) ** 2 * (m - 1) * s
    if not C:
        return m * s * fdm_int + faces
    copies = s * ((C - 3) ** 3 - (C - 5) ** 3)
    return m * s * fdm_int + m * s * fem + s * C ** 3 + s * (C - 3) ** 3 + faces + copies


def setup(wl_name, f32, seed=0):
    import numpy as np
    import torch

    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS[wl_name]
    sig_true = synth.sigma_for(wl, seed)
    dt = synth.dt_rule(wl.h, sig_true.max())
    solver = hyb.Solver(wl.n, C=wl.C, f32=f32)
    st = torch.as_tensor(sig_true, dtype=torch.float64, device="cuda")
    obs = solver.forward(st, wl.nt, dt, omega=wl.omega)
    data = synth.add_noise(obs.cpu().numpy(), wl.noise, seed + 1)
    data = torch.as_tensor(data, dtype=torch.float64, device="cuda")
    del obs
    return wl, dt, solver, data, sig_true


def run_cg(wl, dt, solver, data, steps, warmup):
    """warmup + steps CG iterations from sigma = 0; returns the time of the
    timed ones, the (|g|, J) log, sigma, the forward + adjoint sweeps the
    timed iterations ran, and their trial counts."""
    import torch

    from paper_1509_01399_amd import hyb
    sig = torch.zeros((wl.C,) * 3, dtype=torch.float64, device="cuda")
    state = hyb.hyb_cg_state()
    log = []
    for _ in range(warmup):
        log.append(solver.cg_step(data, sig, wl.nt, dt, state, omega=wl.omega))
    torch.cuda.synchronize()
    sweeps, trials = 0, []
    t0 = time.perf_counter()
    for _ in range(steps):
        log.append(solver.cg_step(data, sig, wl.nt, dt, state, omega=wl.omega))
        sweeps += state.forwards + 1
        trials.append(state.trials)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0), log, sig, sweeps, trials


def _oracle_window(wl, dt, window, threads):
    """Marginal oracle rate on the full grid between windows of 2 and
    `window` forward+adjoint steps (one oracle gradient evaluation each), so
    the oracle's mesh set-up is not charged to it."""
    import numpy as np

    import oracle
    from paper_1509_01399_amd import synth
    used = oracle.threads(threads)
    g = oracle.Geometry(wl.n, fem_o=wl.o, fem_c=wl.C)
    sz = g.sizes()
    sig = synth.sigma_for(wl, 0).ravel()
    ts = []
    for w in (2, window):
        data = np.zeros((w + 1, wl.n + 1, wl.n + 1))
        t0 = time.perf_counter()
        oracle.gradient(g, sig, w, dt, data, omega=wl.omega)
        ts.append(time.perf_counter() - t0)
    upd = 2 * (sz["fdm_updated"] + sz["fem_updated"]) * (window - 2)
    return upd / (ts[1] - ts[0]) / 1e9, ts, used


def cpu_baseline(wl, dt, window):
    """The CPU oracle (plain FP64 C; OpenMP over z planes in its FDM rows, the
    FEM and boundary rows on one thread) on windows of the same workload,
    once with every host thread and once with one."""
    import oracle
    from oracle.build import build, lib_path
    if not os.path.exists(lib_path()):
        build()
    keep = oracle.threads()
    all_threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    try:
        v_all, ts_all, used = _oracle_window(wl, dt, window, all_threads)
        v_one, ts_one, _ = _oracle_window(wl, dt, window, 1)
    finally:
        oracle.threads(keep)
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": round(v_all, 5), "unit": "Gpt-updates/s", "cores": used, "kind": "oracle",
            "single_thread": {"value": round(v_one, 5), "cores": 1},
            "sample": f"{wl.name} full grid ({wl.n}^3 cells, FEM {wl.C}^3): one oracle forward+adjoint of 2 and "
                      f"of {window} steps; marginal rate over the {window - 2} extra step pairs; {used} threads "
                      f"({ts_all[0]:.1f} s, {ts_all[1]:.1f} s) and 1 thread ({ts_one[0]:.1f} s, {ts_one[1]:.1f} s)"
                      f"; host: {os.cpu_count()} CPUs visible, {model}"}


def kernel_source_hash():
    """Hash of the code (comments and blank space left out) of the kernels,
    their launchers (grid, tiles, cache hints), the parameter blocks they
    read and the host function that fixes the tiles and z chunks."""
    import hashlib
    import re

    def code(text):
        text = re.sub(r"//[^\n]*", "", text)
        return re.sub(r"\s+", " ", text).strip().encode()

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1509_01399_amd", "csrc")
    for f in ("hyb_kernels.hip", "hyb_internal.h"):
        with open(os.path.join(csrc, f)) as fh:
            h.update(code(fh.read()))
    with open(os.path.join(csrc, "hyb_api.cpp")) as fh:
        api = fh.read()
    a = api.find("void setup_geo(")
    h.update(code(api[a:api.find("\n}\n", a)] if a >= 0 else api))
    return h.hexdigest()[:16]


def measured_traffic(wl_name, f32):
    """HBM bytes per launch of the interior kernel from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE passes, calibrated on a plain copy), or
    None when the summary is missing or was taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_interior_{wl_name}_{'f32' if f32 else 'f64'}_counters.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith(" ") and "|" not in line:
            k, _, v = line.strip().partition("=")
            kv[k] = v
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return int(float(kv["read_bytes"]) + float(kv["write_bytes"]))
    except (KeyError, ValueError):
        return None


def stream_reference(n, s, reps=20):
    """What plain streaming reaches on this GPU for arrays of n elements of s
    bytes (sized like the interior launch's streams, beyond the last-level
    cache): a copy (read 1, write 1) and an add c = a + b (read 2, write 1,
    the leapfrog's pattern), torch's elementwise kernels, HIP events on the
    current stream.  Context for the roofline fraction, not the peak."""
    import torch
    dt = torch.float32 if s == 4 else torch.float64
    a = torch.rand(n, dtype=dt, device="cuda")
    b = torch.rand(n, dtype=dt, device="cuda")
    c = torch.empty_like(a)
    out = {}
    for name, fn, streams in (("copy", lambda: c.copy_(a), 2), ("add", lambda: torch.add(a, b, out=c), 3)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_GBs"] = round(streams * n * s / (ms * 1e-3) / 1e9, 1)
    del a, b, c
    torch.cuda.empty_cache()
    out["elements"] = n
    return out


def roofline(wl, dt, solver, f32, reps=50):
    """Roofline of the forward interior launch: algorithmic bytes (three
    streams per node, the leapfrog's minimum) over the average launch time
    measured with HIP events on the solver's stream.  FP32 also reports the
    fraction by the bytes its increment form moves (four streams)."""
    import torch
    from paper_1509_01399_amd import hyb
    s = 4 if f32 else 8
    sig = torch.as_tensor(__import__("paper_1509_01399_amd.synth", fromlist=["x"]).sigma_for(wl, 0),
                          dtype=torch.float64, device="cuda")
    hyb.hyb_time_interior(solver.ctx, sig, dt, 5)  # warm
    ms = hyb.hyb_time_interior(solver.ctx, sig, dt, reps)
    b = interior_bytes(wl.n, wl.C, s)
    achieved = b / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(wl.name, f32),
           "kernel": "k_interior<%s,false,*> (forward FDM+FEM interior)" % ("float" if f32 else "double"),
           "bytes_per_launch": b, "avg_launch_ms": round(ms, 5)}
    ref = stream_reference((wl.n + 1) ** 3, s)
    out["stream_reference"] = ref
    out["frac_of_add"] = round(achieved / ref["add_GBs"], 4)
    if f32:
        b4 = interior_bytes(wl.n, wl.C, s, streams=4)
        out["increment_form"] = {"bytes_per_launch": b4, "achieved": round(b4 / (ms * 1e-3) / 1e9, 1),
                                 "frac": round(b4 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    return out


def same_horizon(wl, dt):
    """Steps that reach the workload's own final time nt * dt_rule with the
    step dt: a smaller step (a general mesh's or a faster medium's CFL bound)
    keeps the time the scattered wave needs to cross the FEM box and return
    to the observed face."""
    import numpy as np

    from paper_1509_01399_amd import synth
    T = wl.nt * synth.dt_rule(wl.h, synth.sigma_for(wl, 0).max())
    return int(np.ceil(T / dt - 1e-9))


def general_mesh_setup(wl, seed=0, amp=0.15):
    """The workload's geometry with a general FEM mesh: the 6-tetrahedra split
    of the box with every node strictly inside the inner box moved by up to
    amp * h per axis, the workload's inclusions sampled per tetrahedron, and a
    time step of 0.9 times an element-wise bound of the FEM rows' Gershgorin
    stability limit (the library checks the assembled one, which is lower)."""
    import numpy as np

    from paper_1509_01399_amd import synth
    xyz, tet = synth.perturbed_box_mesh(wl.o, wl.C, wl.h, seed=seed + 7, amp=amp)
    st = synth.tet_sigma(xyz, tet, synth.sigma_for(wl, seed), wl.o, wl.C, wl.h)
    X = xyz[tet]
    E = np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1))
    G = np.linalg.inv(E)
    G = np.concatenate([-G.sum(1, keepdims=True), G], 1)
    vol = np.abs(np.linalg.det(E)) / 6
    ke = vol[:, None, None] * (G @ np.transpose(G, (0, 2, 1)))
    a = 1.0 + st
    row = np.zeros(len(xyz))
    mass = np.zeros(len(xyz))
    np.add.at(row, tet.ravel(), (a[:, None] * np.abs(ke).sum(2)).ravel())
    np.add.at(mass, tet.ravel(), np.repeat(vol / 4, 4))
    dt = min(0.9 * 2.0 / np.sqrt((row / mass).max()), wl.h / np.sqrt(3.0) * 0.9)
    return xyz, tet, st, dt


def general_fem_bytes(xyz, tet, wl, s):
    """Algorithmic bytes of one launch of the general FEM row kernels (field
    element size s).  Per row: its column ids and kappa values (4 + s per mesh
    neighbour), the row's own levels (FP64: read v^k, v^{k-1}, write v^{k+1};
    FP32 increment form: read v^k, d^k, write d^{k+1}, v^{k+1}) and dt^2/m;
    the history level of the inner-box nodes; the omega_diamond copy (an
    8-byte grid index and the value written into the grid); the omega_o
    neighbours, read from the grid level (an 8-byte grid index and the
    value).  The adjoint also reads the neighbour lists of the box surface
    (its omega_o couplings, an index and a value written into the grid),
    the six grid multipliers around each omega_diamond node, and
    read-modify-writes one FP64 accumulator per edge of the inner box.
    Neighbour values gathered by several rows are counted once."""
    import numpy as np
    h, o, C = wl.h, wl.o, wl.C
    q = xyz / h - o
    qi = np.rint(q)
    grid = np.all(np.abs(q - qi) < 1e-7, axis=1)
    surf = np.any((np.abs(q) < 1e-7) | (np.abs(q - C) < 1e-7), axis=1)
    inner = np.all((q > 2 - 1e-7) & (q < C - 2 + 1e-7), axis=1)
    onD = grid & inner & np.any((np.abs(q - 2) < 1e-7) | (np.abs(q - (C - 2)) < 1e-7), axis=1)
    pairs = tet[:, [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]].reshape(-1, 2).astype(np.int64)
    pairs.sort(axis=1)
    key = np.unique(pairs[:, 0] * len(xyz) + pairs[:, 1])
    ea, eb = key // len(xyz), key % len(xyz)
    deg = np.bincount(ea, minlength=len(xyz)) + np.bincount(eb, minlength=len(xyz))
    rows = ~surf
    m = 4 if s == 4 else 3
    nR, nH, nA, nS = int(rows.sum()), int(inner.sum()), int(onD.sum()), int(surf.sum())
    ent_rows, ent_all = int(deg[rows].sum()), int(deg.sum())
    up_inner = int((inner[ea] & inner[eb]).sum())
    fwd = ent_rows * (4 + s) + nR * (m * s + s) + nH * s + nS * (8 + s) + nA * (8 + s)
    adj = ent_all * (4 + s) + nR * (m * s + s) + nH * s + up_inner * 16 + nS * (8 + s) + nA * (8 + 6 * s)
    return fwd, adj


def general_mesh(wl_name, steps, warmup, f32=False, seed=0):
    """The CG iteration of the benchmark on a general mesh of the FEM box (the
    general-mesh path of the library) over the workload's final time (more
    steps of the mesh's smaller dt), and the roofline of its FEM row kernels
    (forward, adjoint) timed with HIP events on the solver's stream."""
    import torch

    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS[wl_name]
    t0 = time.perf_counter()
    xyz, tet, st, dt = general_mesh_setup(wl, seed)
    nt = same_horizon(wl, dt)
    solver = hyb.Solver(wl.n, C=wl.C, mesh=(xyz, tet), f32=f32)
    t_setup = time.perf_counter() - t0
    assert solver.general
    sig_true = torch.as_tensor(st, dtype=torch.float64, device="cuda")
    obs = solver.forward(sig_true, nt, dt, omega=wl.omega)
    data = torch.as_tensor(synth.add_noise(obs.cpu().numpy(), wl.noise, seed + 1), dtype=torch.float64,
                           device="cuda")
    del obs
    sig = torch.zeros(len(tet), dtype=torch.float64, device="cuda")
    state = hyb.hyb_cg_state()
    warm = []
    for _ in range(warmup):
        solver.cg_step(data, sig, nt, dt, state, omega=wl.omega)
        warm.append((state.trials, state.stalled, state.J_next))
    torch.cuda.synchronize()
    sweeps, trials, stalls = 0, [], []
    t1 = time.perf_counter()
    for _ in range(steps):
        gn, J = solver.cg_step(data, sig, nt, dt, state, omega=wl.omega)
        sweeps += state.forwards + 1
        trials.append(state.trials)
        stalls.append(state.stalled)
    torch.cuda.synchronize()
    t = time.perf_counter() - t1
    nfdm, nfem = solver.counts()
    value = sweeps * (nfdm + nfem) * nt / t / 1e9
    s = 4 if f32 else 8
    bf, ba = general_fem_bytes(xyz, tet, wl, s)
    out = {"workload": f"{wl.name} grid, general FEM mesh", "tets": int(len(tet)), "fem_nodes": int(len(xyz)),
           "node_shift": "U(-0.15 h, 0.15 h) per axis inside the inner box", "dt_over_h": round(dt / wl.h, 4), "nt": nt,
           "dtype": "f32" if f32 else "f64", "value": round(value, 2), "unit": "Gpt-updates/s",
           "ms_per_step": round(t / steps * 1e3, 3), "sweeps_per_step": round(sweeps / steps, 2),
           "trials": trials, "stalled": stalls, "warmup_trials_stalled_Jnext": warm,
           "host_setup_s": round(t_setup, 2), "last_J": J, "last_gnorm": gn}
    for which, b, name in ((0, bf, "forward"), (1, ba, "adjoint")):
        # each timing call overwrites the sweeps it needs: a forward sweep
        # (and for the adjoint rows an adjoint sweep) before the warm-up
        # launches and again before the timed ones
        for reps in (5, 50):
            obs = solver.forward(sig, nt, dt, omega=wl.omega)
            if which == 1:
                solver.adjoint(obs - data, mode=0)
            del obs
            ms = hyb.hyb_time_fem(solver.ctx, which, reps)
        ach = b / (ms * 1e-3) / 1e9
        out[f"roofline_{name}"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                                   "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                                   "kernel": f"k_gen_{'fwd' if which == 0 else 'adj'}<"
                                             f"{'float' if f32 else 'double'}>",
                                   "bytes_per_launch": int(b), "avg_launch_ms": round(ms, 5)}
    solver.close()
    del data, sig, sig_true
    torch.cuda.empty_cache()
    return out


def model_forms(wl_name, steps, warmup, seed=0):
    """The two model extensions on the benchmark's grid, FP64 fields, one CG
    iteration per step as in the main line:
    - Model Problem 1 (IP1): data and every sweep start from the paper's
      Test 1 initial condition exp(-|x|^2) at rest (Taylor start);
    - variable wave speed: 1-4 regions with c ~ U(1, 2) in the free cubes
      (synth.wave_speed), dt = 0.95 h sqrt(min(1/c^2) / 15) (the CFL bound
      for a <= 5), plus the derivative with respect to 1/c^2 at the final
      iterate (hyb_gradient_eps), timed alone.
    Both run to the workload's final time (more steps for the smaller dt)."""
    import numpy as np
    import torch

    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS[wl_name]
    sig_true = synth.sigma_for(wl, seed)
    st = torch.as_tensor(sig_true, dtype=torch.float64, device="cuda")
    out = {}
    for form in ("model_problem_1", "wave_speed"):
        solver = hyb.Solver(wl.n, C=wl.C)
        dt = synth.dt_rule(wl.h, sig_true.max())
        if form == "model_problem_1":
            f0 = torch.as_tensor(synth.gaussian_initial(wl.n), dtype=torch.float64, device="cuda")
            solver.set_initial_taylor(f0, None)
            del f0
        else:
            eps = synth.wave_speed(wl.C, seed + 5)
            dt = 0.95 * wl.h * math.sqrt(float(eps.min()) / 15.0)
            solver.set_wave_speed(torch.as_tensor(eps, dtype=torch.float64, device="cuda"))
        nt = same_horizon(wl, dt)
        obs = solver.forward(st, nt, dt, omega=wl.omega)
        data = torch.as_tensor(synth.add_noise(obs.cpu().numpy(), wl.noise, seed + 1), device="cuda")
        del obs
        sig = torch.zeros_like(st)
        state = hyb.hyb_cg_state()
        geps = torch.zeros_like(st) if form == "wave_speed" else None
        for _ in range(warmup):
            solver.cg_step(data, sig, nt, dt, state, omega=wl.omega)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweeps, trials, stalls = 0, [], []
        for _ in range(steps):
            gn, J = solver.cg_step(data, sig, nt, dt, state, omega=wl.omega)
            sweeps += state.forwards + 1
            trials.append(state.trials)
            stalls.append(state.stalled)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        te = 0.0
        if geps is not None:
            # dJ/d(1/c^2) of the last adjoint: a sweep pair at the final
            # iterate, then the derivative alone timed
            obs = solver.forward(sig, nt, dt, omega=wl.omega)
            solver.adjoint(obs - data, mode=0)
            del obs
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            solver.gradient_eps(geps)
            torch.cuda.synchronize()
            te = time.perf_counter() - t1
        nfdm, nfem = solver.counts()
        res = {"value": round(sweeps * (nfdm + nfem) * nt / t / 1e9, 2),
               "unit": "Gpt-updates/s", "ms_per_step": round(t / steps * 1e3, 3),
               "sweeps_per_step": round(sweeps / steps, 2), "trials": trials, "stalled": stalls,
               "dt_over_h": round(dt / wl.h, 4), "nt": nt, "dtype": "f64", "last_J": J, "last_gnorm": gn}
        if geps is not None:
            res["eps_gradient_ms"] = round(te * 1e3, 3)
            res["min_inv_c2"] = round(float(eps.min()), 4)
            res["eps_gradient_norm"] = float(geps.norm())
        out[form] = res
        solver.close()
        del data, sig
        torch.cuda.empty_cache()
    return out


def serving(n_req=256, seed=0, budget=200e9):
    """Serving workload: n_req forward+adjoint+gradient requests, grid sizes
    uniform over {64,96,128,192,256}^3, FP32 fields, Poisson arrivals at
    twice the rate the unbatched path sustains (2 / mean unbatched service
    time, measured on one request per size), 200 GB HBM budget."""
    import numpy as np
    import torch

    from paper_1509_01399_amd import serve, synth
    sizes = synth.SERVE_SIZES
    data = serve.background_data(sizes)
    pool = serve.Pool(budget, True)
    # calibration: one request per size, alone
    cal = serve.make_requests(len(sizes) * 3, seed + 100, rate=1e9, sizes=sizes)
    seen, calib = set(), []
    for r in cal:
        if r.n not in seen:
            seen.add(r.n)
            r.arrival = 0.0
            calib.append(r)
    serve.run_unbatched(calib, data, pool=pool)          # warm (allocations, code)
    res, _ = serve.run_unbatched(calib, data, pool=pool)
    mean_service = float(np.mean([x.finished - x.admitted for x in res]))
    # offered load: twice what the unbatched path sustains, so that both
    # paths run at their capacity and the throughputs compare the servers
    rate = 2.0 / mean_service
    reqs = serve.make_requests(n_req, seed, rate, sizes)
    # resident contexts for every slot the scheduler may use, created before
    # either timed run (the unbatched path reuses one per size)
    pool.warm(serve.DEFAULT_CAPS, serve.shapes_of(reqs))
    rb, wb = serve.run_batched(reqs, data, budget=budget, pool=pool)
    ru, wu = serve.run_unbatched(reqs, data, pool=pool)
    peak = pool.used
    pool.close()
    del data
    torch.cuda.empty_cache()
    sb, su = serve.summarize(rb, wb, reqs), serve.summarize(ru, wu, reqs)
    jd = max(abs(a.J - b.J) / abs(b.J) for a, b in zip(rb, ru))
    return {"workload": f"{n_req} requests, n in {list(sizes)}, C = 3n/8, nt = 5n, fp32 fields",
            "arrival_rate_per_s": round(rate, 2), "budget_gb": budget / 1e9,
            "caps": {str(k): v for k, v in serve.DEFAULT_CAPS.items()},
            "steps_per_call": serve.DEFAULT_STEPS_PER_CALL,
            "resident_gb": round(peak / 1e9, 1), "batched": sb, "unbatched": su,
            "throughput_ratio": round(sb["throughput_req_s"] / su["throughput_req_s"], 3),
            "max_rel_J_diff_batched_vs_alone": jd}


def study_diff384(seed=0, n_dir=16):
    """Differentiation form at full size: 384^3 cells, FEM 128^3, nt = 2000,
    sqrt(nt) checkpoints with segment recompute.  Gradient of L = <w, obs>
    (w seeded Gaussian) through the autograd Function, with FP64 and with
    FP32 fields, against central differences of L along n_dir seeded random
    unit directions over the free cubes, the differences taken with FP64
    forward solves (largest change of sigma 0.02)."""
    import numpy as np
    import torch

    from paper_1509_01399_amd import autograd, hyb, synth
    wl = synth.WORKLOADS["diff384"]
    sig0 = synth.sigma_for(wl, seed)
    dt = synth.dt_rule(wl.h, sig0.max() + 0.05)
    gen = torch.Generator(device="cuda").manual_seed(seed + 11)
    w = None
    out = {"study": "diff384", "n": wl.n, "C": wl.C, "nt": wl.nt, "directions": n_dir, "max_sigma_step": 0.02,
           "checkpoints": "every ceil(sqrt(nt+1)) steps, field precision"}
    grads = {}
    for f32 in (False, True):
        solver = hyb.Solver(wl.n, C=wl.C, f32=f32, store_mode=1)
        sig = torch.as_tensor(sig0, dtype=torch.float64, device="cuda").requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obs = autograd.solve(sig, solver, wl.nt, dt, wl.omega)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if w is None:
            w = torch.randn(obs.shape, generator=gen, dtype=torch.float64, device="cuda")
        (w * obs).sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        key = "f32" if f32 else "f64"
        grads[key] = sig.grad.detach().clone()
        out[key] = {"forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
                    "footprint_gb": round(hyb.hyb_footprint(solver.grid, solver.mesh, 2, solver.opts, wl.nt) / 1e9,
                                          2)}
        if f32:
            solver.close()
        else:
            fd_solver = solver
        del obs
    free = torch.as_tensor(synth.eligible_mask(wl.C), device="cuda")
    rng = np.random.default_rng(seed + 12)
    rows = []
    with torch.no_grad():
        base = torch.as_tensor(sig0, dtype=torch.float64, device="cuda")
        for _ in range(n_dir):
            v = torch.as_tensor(rng.standard_normal(sig0.shape), device="cuda") * free
            v /= v.norm()
            eps = 0.02 / float(v.abs().max())
            lp = float((w * fd_solver.forward(base + eps * v, wl.nt, dt, omega=wl.omega)).sum())
            lm = float((w * fd_solver.forward(base - eps * v, wl.nt, dt, omega=wl.omega)).sum())
            rows.append(((lp - lm) / (2 * eps), float((grads["f64"] * v).sum()), float((grads["f32"] * v).sum())))
    fd_solver.close()
    fd, a64, a32 = np.array(rows).T
    for key, a in (("f64", a64), ("f32", a32)):
        out[key]["fd_vs_autograd_rel_l2"] = float(np.linalg.norm(fd - a) / np.linalg.norm(fd))
        out[key]["fd_vs_autograd_rel_max"] = float((np.abs(fd - a) / np.abs(fd)).max())
    out["f32_vs_f64_gradient_rel_l2"] = float((grads["f32"] - grads["f64"]).norm() / grads["f64"].norm())
    return out


def study_scale512(seed=0):
    """Precision form at scale: 512^3 cells, FEM 160^3, nt = 2500.  Data from
    an FP64 sweep at the true conductivity plus 3% noise; the misfit gradient
    at sigma = 0 (first CG iteration) with FP32 fields and checkpoints of
    each kind (BF16 increments, FP32 copies, 16-bit block-scaled increments),
    against the FP64 sweep with the full FP64 FEM history: relative L2 and
    element max-abs errors relative to the largest entry."""
    import torch

    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS["scale512"]
    sig_true = synth.sigma_for(wl, seed)
    dt = synth.dt_rule(wl.h, sig_true.max())
    st = torch.as_tensor(sig_true, dtype=torch.float64, device="cuda")
    s0 = torch.zeros_like(st)
    out = {"study": "scale512", "n": wl.n, "C": wl.C, "nt": wl.nt}
    ref = hyb.Solver(wl.n, C=wl.C, f32=False, store_mode=0)
    data = ref.forward(st, wl.nt, dt, omega=wl.omega).clone()
    gen = torch.Generator(device="cuda").manual_seed(seed + 21)
    data += wl.noise * data.abs().max() * torch.randn(data.shape, generator=gen, dtype=torch.float64,
                                                      device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs64 = ref.forward(s0, wl.nt, dt, omega=wl.omega).clone()
    ref.adjoint(obs64 - data, mode=0)
    g64, J64 = ref.gradient()
    torch.cuda.synchronize()
    out["f64_s"] = round(time.perf_counter() - t0, 3)
    res64 = obs64 - data
    out["residual_over_trace"] = float(res64.norm() / obs64.norm())
    out["f64_footprint_gb"] = round(hyb.hyb_footprint(ref.grid, ref.mesh, 2, ref.opts, wl.nt) / 1e9, 2)
    ref.close()
    torch.cuda.empty_cache()
    def mx(a, b):
        return float((a - b).abs().max() / b.abs().max())

    for mode, name in ((2, "f32_bf16ckpt"), (1, "f32_f32ckpt"), (3, "f32_q16ckpt")):
        s = hyb.Solver(wl.n, C=wl.C, f32=True, store_mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obs = s.forward(s0, wl.nt, dt, omega=wl.omega)
        s.adjoint(obs - data, mode=0)
        g, J = s.gradient()
        torch.cuda.synchronize()
        out[name] = {"s": round(time.perf_counter() - t0, 3),
                     "footprint_gb": round(hyb.hyb_footprint(s.grid, s.mesh, 2, s.opts, wl.nt) / 1e9, 2),
                     "trace_rel_l2": float((obs - obs64).norm() / obs64.norm()),
                     "residual_rel_l2": float((obs - obs64).norm() / res64.norm()),
                     "grad_rel_l2": float((g - g64).norm() / g64.norm()),
                     "trace_max_abs": mx(obs, obs64), "grad_max_abs": mx(g, g64),
                     "J_rel": abs(J - J64) / abs(J64)}
        s.close()
        del obs, g
        torch.cuda.empty_cache()
    return out


def leg_tiny40(seed=0):
    """The 40^3 correctness workload (FEM 16^3, 300 steps, two 3^3 inclusions
    of sigma = 2, noise-free data from the same grid): time of one forward +
    adjoint + gradient at sigma = 0 and of 3 CG iterations (FP64), and the
    errors of trace, gradient and J against the oracle.  Launch-bound: the
    roofline does not apply at this size."""
    import numpy as np
    import torch

    import oracle
    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS["tiny40"]
    sig_true = synth.sigma_for(wl, seed)
    dt = synth.dt_rule(wl.h, sig_true.max())
    g = oracle.Geometry(wl.n, fem_o=wl.o, fem_c=wl.C)
    data_h = oracle.forward(g, sig_true.ravel(), wl.nt, dt, omega=wl.omega)
    gref, Jref, oref = oracle.gradient(g, np.zeros(wl.C ** 3), wl.nt, dt, data_h, omega=wl.omega, want_obs=True)
    s = hyb.Solver(wl.n, C=wl.C)
    data = torch.as_tensor(data_h, device="cuda")
    s0 = torch.zeros((wl.C,) * 3, dtype=torch.float64, device="cuda")
    for _ in range(2):  # warm, then timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obs = s.forward(s0, wl.nt, dt, omega=wl.omega)
        s.adjoint(obs - data, mode=0)
        grad, J = s.gradient()
        t_grad = time.perf_counter() - t0
    sig = torch.zeros_like(s0)
    st = hyb.hyb_cg_state()
    sweeps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        s.cg_step(data, sig, wl.nt, dt, st, omega=wl.omega)
        sweeps += st.forwards + 1
    torch.cuda.synchronize()
    t_cg = time.perf_counter() - t0
    nfdm, nfem = s.counts()
    o, gr = obs.cpu().numpy(), grad.cpu().numpy().ravel()
    s.close()
    return {"workload": "tiny40: 40^3 cells, FEM 16^3, nt 300, dt 0.25 h, f64",
            "forward_adjoint_gradient_ms": round(t_grad * 1e3, 3), "cg3_ms": round(t_cg * 1e3, 3),
            "cg3_sweeps": sweeps, "cg3_value": round(sweeps * (nfdm + nfem) * wl.nt / t_cg / 1e9, 3),
            "unit": "Gpt-updates/s",
            "vs_oracle": {"trace_rel_l2": float(np.linalg.norm(o - oref) / np.linalg.norm(oref)),
                          "gradient_rel_l2": float(np.linalg.norm(gr - gref) / np.linalg.norm(gref)),
                          "J_rel": abs(J - Jref) / Jref}}


def leg_diff384(seed=0):
    """The differentiation workload's rate: 384^3 cells, FEM 128^3, 2000
    steps, FP32 fields with sqrt(nt) FP32 checkpoints; forward through the
    autograd Function and backward (adjoint with segment recompute, the
    recompute counted as time, not as updates), and the interior roofline
    at this size."""
    import torch

    from paper_1509_01399_amd import autograd, hyb, synth
    wl = synth.WORKLOADS["diff384"]
    sig0 = synth.sigma_for(wl, seed)
    dt = synth.dt_rule(wl.h, sig0.max() + 0.05)
    solver = hyb.Solver(wl.n, C=wl.C, f32=True, store_mode=1)
    gen = torch.Generator(device="cuda").manual_seed(seed + 11)
    w = torch.randn((wl.nt + 1, wl.n + 1, wl.n + 1), generator=gen, dtype=torch.float64, device="cuda")
    ts = []
    for _ in range(2):  # warm, then timed
        sig = torch.as_tensor(sig0, dtype=torch.float64, device="cuda").requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obs = autograd.solve(sig, solver, wl.nt, dt, wl.omega)
        (w * obs).sum().backward()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        del obs
    nfdm, nfem = solver.counts()
    rl = roofline(wl, dt, solver, True)
    solver.close()
    del w
    torch.cuda.empty_cache()
    return {"workload": "diff384: 384^3 cells, FEM 128^3, nt 2000, f32 fields, sqrt(nt) f32 checkpoints",
            "value": round(2.0 * (nfdm + nfem) * wl.nt / ts[1] / 1e9, 2), "unit": "Gpt-updates/s",
            "forward_backward_s": round(ts[1], 3), "dtype": "f32", "roofline": rl}


def leg_scale512(seed=0):
    """The precision workload's rate: 512^3 cells, FEM 160^3, 2500 steps, FP32
    fields with BF16 checkpoint increments; data from a sweep at the true
    conductivity plus 3% noise; one forward + adjoint + gradient at sigma = 0
    timed (recompute counted as time), and the interior roofline."""
    import torch

    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS["scale512"]
    sig_true = synth.sigma_for(wl, seed)
    dt = synth.dt_rule(wl.h, sig_true.max())
    s = hyb.Solver(wl.n, C=wl.C, f32=True, store_mode=2)
    st = torch.as_tensor(sig_true, dtype=torch.float64, device="cuda")
    data = s.forward(st, wl.nt, dt, omega=wl.omega).clone()
    gen = torch.Generator(device="cuda").manual_seed(seed + 21)
    data += wl.noise * data.abs().max() * torch.randn(data.shape, generator=gen, dtype=torch.float64,
                                                      device="cuda")
    s0 = torch.zeros_like(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = s.forward(s0, wl.nt, dt, omega=wl.omega)
    s.adjoint(obs - data, mode=0)
    s.gradient()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    nfdm, nfem = s.counts()
    fp = hyb.hyb_footprint(s.grid, s.mesh, 2, s.opts, wl.nt)
    rl = roofline(wl, dt, s, True)
    s.close()
    del data, obs
    torch.cuda.empty_cache()
    return {"workload": "scale512: 512^3 cells, FEM 160^3, nt 2500, f32 fields, bf16 checkpoint increments",
            "value": round(2.0 * (nfdm + nfem) * wl.nt / t / 1e9, 2), "unit": "Gpt-updates/s",
            "forward_adjoint_gradient_s": round(t, 3), "footprint_gb": round(fp / 1e9, 1), "dtype": "f32",
            "roofline": rl}


def probe(kind, wl_name, f32, reps):
    """Single-kernel runs for the counter passes (rocprofv3 --pmc)."""
    import torch

    from paper_1509_01399_amd import hyb, synth
    wl = synth.WORKLOADS[wl_name]
    if kind == "copy":
        nbytes = 512 * 2 ** 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(reps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))
        return
    sig_true = synth.sigma_for(wl, 0)
    dt = synth.dt_rule(wl.h, sig_true.max())
    solver = hyb.Solver(wl.n, C=wl.C, f32=f32)
    st = torch.as_tensor(sig_true, dtype=torch.float64, device="cuda")
    solver.forward(st, 2, dt, omega=wl.omega)
    ms = hyb.hyb_time_interior(solver.ctx, st, dt, reps)
    print(json.dumps({"probe": "interior", "workload": wl_name, "f32": f32, "reps": reps, "avg_ms": ms,
                      "bytes_per_launch": interior_bytes(wl.n, wl.C, 4 if f32 else 8)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cg256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=int, default=30)
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--no-general", action="store_true", help="skip the general-mesh leg")
    ap.add_argument("--no-legs", action="store_true", help="skip the tiny40, diff384 and scale512 legs")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the Model Problem 1 and wave-speed legs")
    ap.add_argument("--probe", choices=["interior", "copy"])
    ap.add_argument("--probe-f32", action="store_true")
    ap.add_argument("--probe-reps", type=int, default=20)
    ap.add_argument("--study", choices=["diff384", "scale512", "general", "recon"],
                    help="full-size check of a form instead of the benchmark line")
    ap.add_argument("--gamma", type=float, default=None,
                    help="Tikhonov weight of the reconstruction study (default: the paper's 0.01)")
    ap.add_argument("--noise-kind", choices=["additive", "relative"], default="additive",
                    help="noise of the reconstruction study's data (default: additive, max-scaled)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (a multi-GPU split of the "
              "grid is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    from paper_1509_01399_amd import hyb
    if not os.path.exists(hyb.LIB_PATH):
        from paper_1509_01399_amd.build import build
        build()
    if args.probe:
        probe(args.probe, args.workload, args.probe_f32, args.probe_reps)
        return
    if args.study:
        if args.study == "general":
            res = general_mesh(args.workload, args.steps, args.warmup, f32=args.probe_f32)
        elif args.study == "recon":
            from paper_1509_01399_amd import study
            kw = {} if args.gamma is None else {"gamma": args.gamma}
            res = study.tables(noise_kind=args.noise_kind, **kw)
        else:
            res = study_diff384() if args.study == "diff384" else study_scale512()
        print(json.dumps(res), flush=True)
        return

    wl, dt, solver, data, _ = setup(args.workload, False)
    nfdm, nfem = solver.counts()
    print(f"[bench] {wl.name}: n={wl.n} C={wl.C} nt={wl.nt} dt={dt:.6g} fdm={nfdm} fem={nfem}",
          file=sys.stderr, flush=True)
    t, log, _, sweeps, trials = run_cg(wl, dt, solver, data, args.steps, args.warmup)
    value = sweeps * (nfdm + nfem) * wl.nt / t / 1e9
    print(f"[bench] f64: {t / args.steps * 1e3:.1f} ms/CG-iteration, {sweeps} sweeps, trials {trials}, "
          f"{value:.1f} Gupd/s; |g| {log[-1][0]:.3e} J {log[-1][1]:.4e}", file=sys.stderr, flush=True)
    rl = roofline(wl, dt, solver, False)
    print(f"[bench] roofline f64 interior: {rl}", file=sys.stderr, flush=True)
    solver.close()
    del data
    torch.cuda.empty_cache()

    f32 = None
    if not args.no_f32:
        wl2, dt2, s2, d2, _ = setup(args.workload, True)
        t2, log2, _, sw2, tr2 = run_cg(wl2, dt2, s2, d2, args.steps, args.warmup)
        v2 = sw2 * (nfdm + nfem) * wl.nt / t2 / 1e9
        rl2 = roofline(wl2, dt2, s2, True)
        print(f"[bench] f32: {t2 / args.steps * 1e3:.1f} ms/CG-iteration, {sw2} sweeps, trials {tr2}, "
              f"{v2:.1f} Gupd/s; {rl2}", file=sys.stderr, flush=True)
        f32 = {"value": round(v2, 2), "ms_per_step": round(t2 / args.steps * 1e3, 3),
               "sweeps_per_step": round(sw2 / args.steps, 2), "ms_per_sweep": round(t2 / sw2 * 1e3, 3),
               "dtype": "f32", "roofline": rl2}
        s2.close()
        del d2
        torch.cuda.empty_cache()

    legs = {}
    if not args.no_legs:
        for name, fn in (("tiny40", leg_tiny40), ("diff384", leg_diff384), ("scale512", leg_scale512)):
            legs[name] = fn()
            print(f"[bench] {name}: {legs[name]}", file=sys.stderr, flush=True)

    gen = None
    if not args.no_general:
        gen = general_mesh(args.workload, args.steps, args.warmup)
        print(f"[bench] general mesh: {gen}", file=sys.stderr, flush=True)

    forms = None
    if not args.no_forms:
        forms = model_forms(args.workload, args.steps, args.warmup)
        print(f"[bench] model forms: {forms}", file=sys.stderr, flush=True)

    srv = None
    if not args.no_serve:
        srv = serving(args.serve_requests)
        print(f"[bench] serving: {srv}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, dt, args.cpu_window)
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    line = {
        "metric": "forward+adjoint Gpt-updates/s", "value": round(value, 2), "unit": "Gpt-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t / args.steps * 1e3, 3), "sweeps_per_step": round(sweeps / args.steps, 2),
        "ms_per_sweep": round(t / sweeps * 1e3, 3), "trials": trials,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "grid_cells": wl.n, "fem_cells": wl.C, "nt": wl.nt,
                   "dt_over_h": round(dt / wl.h, 4), "omega": wl.omega, "noise": wl.noise,
                   "step": "one CG iteration (adjoint + gradient + direction + one forward per trial step)",
                   "parallelism": "single GPU"},
        "roofline": rl, "cpu_baseline": cpu, "f32_form": f32, "legs": legs, "general_mesh": gen,
        "model_forms": forms,
        "p50_ms": srv["batched"]["p50_ms"] if srv else None,
        "p99_ms": srv["batched"]["p99_ms"] if srv else None,
        "serving": srv,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
