"""Serving form on the GPU: continuous batching over mixed grid sizes gives
each request the same result as solving it alone, and requests overlap."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("f32", [True, False])
def test_batched_equals_alone(f32):
    import torch
    from paper_1509_01399_amd import hyb, serve
    hyb.load()
    sizes = (24, 32, 40)
    data = serve.background_data(sizes, f32=f32)
    reqs = serve.make_requests(10, seed=5, rate=2000.0, sizes=sizes)
    pool = serve.Pool(float("inf"), f32)
    res_b, _ = serve.run_batched(reqs, data, max_slots=8, f32=f32, keep_grads=True, pool=pool)
    res_u, _ = serve.run_unbatched(reqs, data, f32=f32, keep_grads=True, pool=pool)
    pool.close()
    assert [r.id for r in res_b] == [r.id for r in res_u] == list(range(10))
    # FP64: 1e-12; FP32 wavefields: the precision form's bars (1e-5 on the
    # misfit, which is a trace quantity, 1e-4 on the gradient).  The batched
    # kernels are separate instantiations, so FP32 rounding may differ by ulps.
    tol_J, tol_g = (1e-5, 1e-4) if f32 else (1e-12, 1e-12)
    worst, worst_J = 0.0, 0.0
    for a, b in zip(res_b, res_u):
        assert np.isfinite(a.J) and a.J > 0
        worst_J = max(worst_J, abs(a.J - b.J) / abs(b.J))
        worst = max(worst, np.linalg.norm(a.grad - b.grad) / np.linalg.norm(b.grad))
    print(f"f32={f32}: batched vs alone: worst rel J diff {worst_J:.2e}, worst rel gradient diff {worst:.2e}",
          flush=True)
    assert worst_J <= tol_J and worst <= tol_g
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
    hyb.hyb_batch_destroy(b)
    s.close()
    s2.close()


@pytest.mark.parametrize("f32", [False, True])
def test_batch_mixed_face_kinds(f32):
    """Slots of one grid whose x faces differ share the batched launches: the
    absorbing x-face rows are computed by the interior launch, Neumann rows
    by the boundary launch, each slot by its own face conditions.  Every
    slot's misfit and gradient match the plain path of the same context."""
    import torch
    from paper_1509_01399_amd import hyb
    hyb.load()
    N, A, S = 1, 0, 2
    bcs = [(A, A, A, A, A, S), (N, N, A, A, A, S), (A, N, N, A, A, S), (N, A, A, N, A, S)]
    n, C, nt, om = 24, 8, 120, 30.0
    dt = 0.25 / n
    rng = np.random.default_rng(61)
    sig = np.zeros((C,) * 3)
    sig[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(0, 2, (C - 4,) * 3)
    sg = torch.as_tensor(sig, dtype=torch.float64, device="cuda")
    data = [torch.as_tensor(1e-3 * rng.standard_normal((nt + 1, n + 1, n + 1)), device="cuda") for _ in bcs]
    ref = []
    for bc, d in zip(bcs, data):
        s = hyb.Solver(n, C=C, bc=bc, f32=f32)
        obs = s.forward(sg, nt, dt, omega=om)
        s.adjoint(obs - d, mode=0)
        g, J = s.gradient()
        ref.append((g.cpu().numpy(), J, obs.cpu().numpy()))
        s.close()
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
    tol_J, tol_g = (1e-5, 1e-4) if f32 else (1e-12, 1e-12)
    errs = []
    for (slot, grad, obs), (gref, Jref, oref), bc in zip(outs, ref, bcs):
        eJ = abs(Js[slot] - Jref) / abs(Jref)
        eg = np.linalg.norm(grad.cpu().numpy() - gref) / np.linalg.norm(gref)
        eo = np.linalg.norm(obs.cpu().numpy() - oref) / np.linalg.norm(oref)
        print(f"f32={f32} bc={bc}: trace {eo:.2e}, J {eJ:.2e}, gradient {eg:.2e}", flush=True)
        errs.append((eo, eJ, eg))
    for eo, eJ, eg in errs:
        assert eo <= tol_J and eJ <= tol_J and eg <= tol_g
    for slot, _, _ in outs:
        hyb.hyb_batch_release(b, slot)
    hyb.hyb_batch_destroy(b)
    for s in solvers:
        s.close()
