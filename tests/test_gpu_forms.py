"""GPU tests of the three added forms, each compared with the plain method:
sqrt(nt) checkpointing (FP32/FP64 state copies, BF16 increments), the
differentiation form (torch.autograd.Function over the forward solve) and
the FP32 precision form at a larger size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    from paper_1509_01399_amd import hyb
    assert t.cuda.is_available()
    hyb.load()
    return t


def _t(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _grad_J(torch, n, C, sig, data, nt, dt, om, f32=False, store_mode=0):
    from paper_1509_01399_amd.hyb import Solver
    s = Solver(n, C=C, f32=f32, store_mode=store_mode)
    obs = s.forward(_t(torch, sig), nt, dt, omega=om)
    s.adjoint(obs - _t(torch, data), mode=0)
    g, J = s.gradient()
    out = (g.cpu().numpy(), J, obs.cpu().numpy())
    s.close()
    return out


def _problem(orc, n=40, C=16, nt=300, om=40.0, seed=0):
    from paper_1509_01399_amd import synth
    sig_true = synth.symmetric_pair(C, seed)
    h = 1.0 / n
    dt = synth.dt_rule(h, sig_true.max())
    g = orc.Geometry(n, fem_o=(n - C) // 2, fem_c=C)
    data = synth.add_noise(orc.forward(g, sig_true.ravel(), nt, dt, omega=om), 0.03, 7)
    return g, 0.5 * sig_true, data, dt


@pytest.mark.parametrize("f32", [False, True])
def test_checkpoints_reproduce_history_bitwise(torch, orc, f32):
    """Store mode 1 restores exact states and recomputes the same kernels, so
    the gradient equals the full-history gradient bit for bit."""
    g, sig, data, dt = _problem(orc)
    g0, J0, _ = _grad_J(torch, 40, 16, sig, data, 300, dt, 40.0, f32=f32, store_mode=0)
    g1, J1, _ = _grad_J(torch, 40, 16, sig, data, 300, dt, 40.0, f32=f32, store_mode=1)
    assert np.array_equal(g0, g1) and J0 == J1


def test_bf16_checkpoints_error(torch, orc):
    """FP32 fields with BF16 checkpoint increments: gradient error against the
    FP64 oracle (reported; bound 1e-3) and against FP32 full history."""
    g, sig, data, dt = _problem(orc)
    gref, Jref = orc.gradient(g, sig.ravel(), 300, dt, data, omega=40.0)
    g32, J32, _ = _grad_J(torch, 40, 16, sig, data, 300, dt, 40.0, f32=True, store_mode=0)
    gb, Jb, _ = _grad_J(torch, 40, 16, sig, data, 300, dt, 40.0, f32=True, store_mode=2)
    e32, eb = rel(g32, gref), rel(gb, gref)
    print(f"gradient rel err vs oracle: fp32 history {e32:.2e}, fp32+bf16 checkpoints {eb:.2e}; "
          f"bf16 vs fp32 history {rel(gb, g32):.2e}", flush=True)
    assert e32 <= 1e-4
    assert eb <= 1e-3


def test_autograd_matches_oracle_adjoint(torch, orc):
    from paper_1509_01399_amd.autograd import HybSolve
    from paper_1509_01399_amd.hyb import Solver
    n, C, nt, om = 24, 10, 120, 30.0
    h = 1.0 / n
    rng = np.random.default_rng(2)
    sig = np.zeros((C, C, C))
    sig[2:C - 2, 2:C - 2, 2:C - 2] = rng.uniform(0, 2, (C - 4,) * 3)
    dt = 0.25 * h
    W = rng.standard_normal((nt + 1, n + 1, n + 1))
    for store_mode in (0, 1):
        s = Solver(n, C=C, store_mode=store_mode)
        x = _t(torch, sig).requires_grad_(True)
        obs = HybSolve.apply(x, s, nt, dt, om)
        loss = (obs * _t(torch, W)).sum()
        loss.backward()
        g = orc.Geometry(n, fem_o=(n - C) // 2, fem_c=C)
        ref = orc.adjoint(g, sig.ravel(), nt, dt, W, omega=om)
        assert rel(x.grad.cpu().numpy(), ref) <= 1e-12
        s.close()


def test_autograd_central_differences(torch):
    """d loss / d sigma along seeded random directions vs central finite
    differences of the forward solve (FP64 fields, checkpointed backward)."""
    from paper_1509_01399_amd.autograd import HybSolve
    from paper_1509_01399_amd.hyb import Solver
    from paper_1509_01399_amd import synth
    n, C, nt, om = 32, 12, 200, 30.0
    h = 1.0 / n
    sig = synth.bumps(C, h, seed=3)
    dt = synth.dt_rule(h, sig.max() + 0.1)
    rng = np.random.default_rng(4)
    W = _t(torch, rng.standard_normal((nt + 1, n + 1, n + 1)))
    s = Solver(n, C=C, store_mode=1)
    x = _t(torch, sig).requires_grad_(True)
    loss = (HybSolve.apply(x, s, nt, dt, om) * W).sum()
    loss.backward()
    grad = x.grad.cpu().numpy()
    el = synth.eligible_mask(C)
    worst = 0.0
    for q in range(8):
        d = rng.standard_normal((C, C, C)) * el
        d /= np.linalg.norm(d)
        eps = 1e-4
        lp = (s.forward(_t(torch, sig + eps * d), nt, dt, omega=om) * W).sum().item()
        lm = (s.forward(_t(torch, sig - eps * d), nt, dt, omega=om) * W).sum().item()
        fd = (lp - lm) / (2 * eps)
        an = float((grad * d).sum())
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-30))
    print("worst FD rel err", worst, flush=True)
    assert worst <= 1e-6
    s.close()
