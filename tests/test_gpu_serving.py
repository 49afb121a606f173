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
