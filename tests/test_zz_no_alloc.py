"""hyb_gradient_noalloc, the entry point for callers that cannot allocate
device memory, against hyb_gradient through the C ABI: two calls in a row on
the same GPU (the second on a smaller problem, so the shared scratch holds
the first call's partials), misfit and cotangent adjoints, the general-mesh
path, and the refusal of a problem whose partials do not fit the scratch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _pair(torch, hyb, n, C, mode, seed, mesh=None, general=False):
    """(hyb_gradient, J) and (hyb_gradient_noalloc, J) after one adjoint."""
    from paper_1509_01399_amd import synth
    rng = np.random.default_rng(seed)
    s = hyb.Solver(n, C=C, mesh=mesh, general=general)
    np_ = s.n_params
    sig = np.zeros(np_) if general else np.zeros((C,) * 3)
    if general:
        sig[:] = rng.uniform(0, 1.5, np_)
    else:
        sig[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(0, 1.5, (C - 4,) * 3)
    sg = torch.as_tensor(sig, dtype=torch.float64, device="cuda")
    dt, nt = 0.25 / n, 4 * n
    obs = s.forward(sg, nt, dt, omega=30.0)
    r = torch.as_tensor(rng.standard_normal(tuple(obs.shape)) * 1e-3, device="cuda")
    s.adjoint(obs - r if mode == 0 else r, mode=mode)
    g_ref, J_ref = s.gradient()
    g_na = torch.full_like(g_ref, np.nan)
    J_na = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    hyb.hyb_gradient_noalloc(s.ctx, g_na, J_na)
    torch.cuda.synchronize()
    out = (g_ref.cpu().numpy(), J_ref, g_na.cpu().numpy(), float(J_na.cpu().numpy()[0]))
    s.close()
    return out


def test_noalloc_gradient_matches_gradient():
    import torch
    from paper_1509_01399_amd import hyb, synth
    assert torch.cuda.is_available()
    hyb.load()
    cases = [("tiny40", 40, 16, 0, None, False), ("smaller", 24, 10, 0, None, False),
             ("cotangent", 24, 10, 1, None, False)]
    o, C, h = 7, 10, 1.0 / 24
    cases.append(("general", 24, C, 0, synth.perturbed_box_mesh(o, C, h, seed=3, amp=0.1), True))
    for tag, n, C, mode, mesh, general in cases:
        print(f"[noalloc] {tag}: n={n} C={C} mode={mode} general={general}", flush=True)
        g, J, gn, Jn = _pair(torch, hyb, n, C, mode, seed=len(tag), mesh=mesh, general=general)
        eg = _rel(gn, g)
        print(f"[noalloc] {tag}: gradient rel {eg:.2e} (bitwise {np.array_equal(gn, g)}), J {Jn!r} vs {J!r}",
              flush=True)
        assert np.all(np.isfinite(gn)) and np.linalg.norm(g) > 0
        assert eg <= TOL
        if mode == 0:
            assert abs(Jn - J) <= TOL * abs(J) and J > 0
        else:
            assert Jn == 0.0


def test_noalloc_refuses_beyond_scratch():
    """More than 4 194 304 parameters: one partial per 256 no longer fits the
    16 384 partials of the scratch."""
    import torch
    from paper_1509_01399_amd import hyb
    assert torch.cuda.is_available()
    hyb.load()
    n, C = 166, 162                     # 162^3 = 4 251 528 cubes
    s = hyb.Solver(n, C=C, o=2)
    g = torch.zeros((C,) * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_gradient_noalloc(s.ctx, g, None)
    assert e.value.status == hyb.HYB_E_UNSUPPORTED
    assert "4194304" in hyb.hyb_last_error(s.ctx)
    s.close()
