"""Serving form on the GPU: continuous batching over mixed grid sizes gives
each request the oracle's result and the same result as solving it alone,
and requests overlap."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


SIZES = (24, 32, 40)


@pytest.fixture(scope="module")
def oracle_case(orc):
    """Ten requests over three grid sizes, fitted against the trace of the
    homogeneous medium (a = 1) computed by the oracle; the oracle's trace, J
    and gradient of every request."""
    from paper_1509_01399_amd import serve, synth
    specs = synth.serve_requests(10, 5, SIZES)
    data, ref = {}, {}
    for n in SIZES:
        C = 3 * n // 8
        g = orc.Geometry(n, fem_o=(n - C) // 2, fem_c=C)
        data[n] = orc.forward(g, np.zeros(C ** 3), 5 * n, 0.25 / n, omega=40.0)
    for sp in specs:
        n, C = sp["n"], sp["C"]
        g = orc.Geometry(n, fem_o=sp["o"], fem_c=C)
        sig = synth.cubes(C, sp["sigma_seed"])
        gr, J, obs = orc.gradient(g, sig.ravel(), sp["nt"], 0.25 / n, data[n], omega=sp["omega"], want_obs=True)
        ref[sp["id"]] = (gr, J, obs)
    return data, ref


def _err(a, b):
    """Relative L2 error and element max-abs error relative to max|b|."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("f32", [True, False])
def test_batched_equals_alone_and_oracle(f32, oracle_case):
    """Every request's trace, J and gradient, served with continuous batching
    and served one at a time, against the oracle's forward, misfit and
    gradient (eq. (gradient1)) of the same request: FP64 1e-12; FP32
    wavefields the precision form's bars, trace 1e-5 and gradient 1e-4, J
    (a function of the residual, like the gradient) 1e-4; relative L2 and
    element max-abs relative to the largest entry.  Batched against alone:
    1e-12 (FP64); FP32 the same bars."""
    import torch
    from paper_1509_01399_amd import hyb, serve
    hyb.load()
    data_h, ref = oracle_case
    data = {n: torch.as_tensor(d, dtype=torch.float64, device="cuda") for n, d in data_h.items()}
    reqs = serve.make_requests(10, seed=5, rate=2000.0, sizes=SIZES)
    pool = serve.Pool(float("inf"), f32)
    res_b, _ = serve.run_batched(reqs, data, max_slots=8, f32=f32, keep_grads=True, pool=pool, keep_obs=True)
    res_u, _ = serve.run_unbatched(reqs, data, f32=f32, keep_grads=True, pool=pool, keep_obs=True)
    pool.close()
    assert [r.id for r in res_b] == [r.id for r in res_u] == list(range(10))
    bar_t, bar_g, bar_J = (1e-5, 1e-4, 1e-4) if f32 else (1e-12, 1e-12, 1e-12)
    worst = np.zeros(3)
    for a, b in zip(res_b, res_u):
        gref, Jref, oref = ref[a.id]
        assert np.isfinite(a.J) and a.J > 0 and np.linalg.norm(gref) > 0
        for res in (a, b):
            e = np.array([_err(res.obs, oref), _err(res.grad, gref), abs(res.J - Jref) / Jref])
            worst = np.maximum(worst, e)
        eba = np.array([_err(a.obs, b.obs), _err(a.grad, b.grad), abs(a.J - b.J) / abs(b.J)])
        assert np.all(eba <= np.array([bar_t, bar_g, bar_J]))
    print(f"f32={f32}: worst vs oracle: trace {worst[0]:.2e}, gradient {worst[1]:.2e}, J {worst[2]:.2e}",
          flush=True)
    assert worst[0] <= bar_t and worst[1] <= bar_g and worst[2] <= bar_J
    # the requests were in flight together
    overl = sum(1 for a in res_b for b in res_b if a.id != b.id and a.admitted < b.finished and b.admitted < a.finished)
    assert overl > 0


def test_batch_slot_errors():
    import torch
    from paper_1509_01399_amd import hyb
    hyb.load()
    b = hyb.hyb_batch_create(1)
    s = hyb.Solver(20, C=8)
    sig = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    obs = torch.zeros((101, 21, 21), dtype=torch.float64, device="cuda")
    grad = torch.zeros_like(sig)
    slot = hyb.hyb_batch_submit(b, s.ctx, sig, 0.0, hyb.make_source(30.0), 100, 0.25 / 20, obs, obs, grad)
    s2 = hyb.Solver(20, C=8)
    with pytest.raises(hyb.HybError) as e:  # no free slot
        hyb.hyb_batch_submit(b, s2.ctx, sig, 0.0, hyb.make_source(30.0), 100, 0.25 / 20, obs, obs, grad)
    assert e.value.status == hyb.HYB_E_STATE
    with pytest.raises(hyb.HybError) as e:  # busy context refuses single calls
        s.forward(sig, 10, 0.25 / 20)
    assert e.value.status == hyb.HYB_E_STATE
    with pytest.raises(hyb.HybError) as e:  # the slot is still running
        hyb.hyb_batch_release(b, slot)
    while hyb.hyb_batch_poll(b, slot)[0] < 1:
        hyb.hyb_batch_tick(b, 4)
    hyb.hyb_batch_release(b, slot)
    with pytest.raises(hyb.HybError) as e:  # CFL checked with the caller's sigma_max
        hyb.hyb_batch_submit(b, s2.ctx, sig, 4.0, hyb.make_source(30.0), 100, 0.4 / 20, obs, obs, grad)
    assert e.value.status == hyb.HYB_E_CFL
    # an understated sigma_max passes the submission's check (a = 1.5 allows
    # dt = 0.4 h) but the device maximum (sigma = 2, a = 3) does not: the slot
    # ends as failed and names the reason
    big = sig.clone()
    big[3:5, 3:5, 3:5] = 2.0
    slot = hyb.hyb_batch_submit(b, s2.ctx, big, 0.5, hyb.make_source(30.0), 40, 0.4 / 20, obs, obs, grad)
    while hyb.hyb_batch_poll(b, slot)[0] < 1:
        hyb.hyb_batch_tick(b, 8)
    torch.cuda.synchronize()
    assert hyb.hyb_batch_poll(b, slot)[0] == 3
    assert "sigma_max" in hyb.hyb_batch_last_error(b)
    hyb.hyb_batch_release(b, slot)
    hyb.hyb_batch_destroy(b)
    s.close()
    s2.close()


@pytest.mark.parametrize("f32", [False, True])
def test_batch_mixed_face_kinds(f32, orc):
    """Slots of one grid whose faces differ share the batched launches: the
    rows of absorbing faces are computed by the interior launch, Neumann rows
    by the boundary launch, each slot by its own face conditions.  Every
    slot's trace, misfit and gradient against the oracle with the same face
    conditions (bars as in test_batched_equals_alone_and_oracle)."""
    import torch
    from paper_1509_01399_amd import hyb
    hyb.load()
    N, A, S = 1, 0, 2
    bcs = [(A, A, A, A, A, S), (N, N, A, A, A, S), (A, N, N, A, A, S), (N, A, A, N, A, S)]
    n, C, nt, om = 24, 8, 120, 30.0
    o = (n - C) // 2
    dt = 0.25 / n
    rng = np.random.default_rng(61)
    sig = np.zeros((C,) * 3)
    sig[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(0, 2, (C - 4,) * 3)
    sg = torch.as_tensor(sig, dtype=torch.float64, device="cuda")
    data_h = [1e-3 * rng.standard_normal((nt + 1, n + 1, n + 1)) for _ in bcs]
    data = [torch.as_tensor(d, device="cuda") for d in data_h]
    ref = []
    for bc, d in zip(bcs, data_h):
        g = orc.Geometry(n, bc=bc, fem_o=o, fem_c=C)
        gr, J, obs = orc.gradient(g, sig.ravel(), nt, dt, d, omega=om, want_obs=True)
        ref.append((gr, J, obs))
    b = hyb.hyb_batch_create(len(bcs))
    solvers, outs = [], []  # the slots' buffers must outlive their slots
    for bc, d in zip(bcs, data):
        s = hyb.Solver(n, C=C, bc=bc, f32=f32)
        obs = torch.zeros((nt + 1, n + 1, n + 1), dtype=torch.float64, device="cuda")
        grad = torch.zeros((C,) * 3, dtype=torch.float64, device="cuda")
        slot = hyb.hyb_batch_submit(b, s.ctx, sg, float(sig.max()), hyb.make_source(om), nt, dt, d, obs, grad)
        solvers.append(s)
        outs.append((slot, grad, obs))
    # forward and adjoint sweeps: 2 (nt + 1) ticks at most, plus set-up
    # ticks; polling does not wait, so enqueue everything, then synchronise
    for _ in range(64):
        hyb.hyb_batch_tick(b, 16)
        states, _ = hyb.hyb_batch_poll_all(b, len(bcs))
        assert 3 not in states
        if all(st >= 1 for st in states):
            break
    torch.cuda.synchronize()
    states, Js = hyb.hyb_batch_poll_all(b, len(bcs))
    assert all(st == 2 for st in states), states
    bar_t, bar_g, bar_J = (1e-5, 1e-4, 1e-4) if f32 else (1e-12, 1e-12, 1e-12)
    errs = []
    for (slot, grad, obs), (gref, Jref, oref), bc in zip(outs, ref, bcs):
        eJ = abs(Js[slot] - Jref) / abs(Jref)
        eg = _err(grad.cpu().numpy(), gref)
        eo = _err(obs.cpu().numpy(), oref)
        print(f"f32={f32} bc={bc}: trace {eo:.2e}, J {eJ:.2e}, gradient {eg:.2e}", flush=True)
        errs.append((eo, eJ, eg))
    for eo, eJ, eg in errs:
        assert eo <= bar_t and eJ <= bar_J and eg <= bar_g
    for slot, _, _ in outs:
        hyb.hyb_batch_release(b, slot)
    hyb.hyb_batch_destroy(b)
    for s in solvers:
        s.close()
